/*
 * fastergs.h -- C ABI of the MI355X (gfx950) training-step library for 3D
 * Gaussian Splatting: differentiable tile-based rasterization (forward and
 * backward) and a fused Adam update, after Faster-GS (Hahlbohm et al.,
 * arXiv 2602.09999).
 *
 * Conventions (all entry points):
 *  - Every pointer is a DEVICE pointer unless marked (host).  All buffers
 *    belong to the caller.  The library allocates no device memory; the
 *    workspace is a caller-owned byte buffer.  State kept between calls:
 *    per thread, the last error message (fgs_last_error) and the armed
 *    timing hook (fgs_time_next_launch); per device, the static scratch
 *    array of fgs_sort_pairs_noalloc and its looked-up address.  Nothing
 *    else survives a call outside the caller's buffers (in the workspace,
 *    with FGS_FLAG_KEEP_ACCUM_ZERO: whether its accumulators are zero).
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t, NULL = the
 *    default stream).  fgs_rasterize_forward alone synchronises `stream` once
 *    to read the instance count (see there).
 *  - Arguments are validated before anything is launched; an invalid call
 *    returns FGS_ERR_INVALID_ARGUMENT (or FGS_ERR_UNSUPPORTED for a valid
 *    but unimplemented option) and enqueues nothing.  HIP runtime failures
 *    return FGS_ERR_HIP.  fgs_last_error() gives a thread-local message.
 *  - Layouts are structure-of-arrays, float32, index i of Gaussian i in
 *    every plane ("[k][n]" = k planes of n floats, plane-major).
 *  - Entry points are re-entrant; calls that share a workspace must not
 *    overlap.  No exception crosses the ABI.
 */
#ifndef FASTERGS_H
#define FASTERGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGS_ABI_VERSION 13

typedef enum fgs_status {
  FGS_OK = 0,
  FGS_ERR_INVALID_ARGUMENT = 1,
  FGS_ERR_CAPACITY = 2,    /* instance buffers too small; see fgs_rasterize_forward */
  FGS_ERR_HIP = 3,
  FGS_ERR_UNSUPPORTED = 4
} fgs_status;

typedef enum fgs_dtype { FGS_F32 = 0, FGS_BF16 = 1 } fgs_dtype;

/* fgs_settings.flags bits.
 * FGS_FLAG_FP64_CONIC: the precision form's float64 path for the
 *   near-degenerate 2x2 covariance: the determinant guard and the inverse of
 *   the dilated matrix are formed in float64 from the float32 entries and the
 *   conic is rounded to float32 (everything else stays float32). */
#define FGS_FLAG_FP64_CONIC 1u
/* FGS_FLAG_LOOKBACK_FALLBACK: a test aid.  The duplication's look-back
 *   (which finds each visible Gaussian's first instance slot) polls no
 *   status at all, so every workgroup after the first sums the counts of all
 *   earlier entries directly, the exact path otherwise taken only when a
 *   bounded wait runs out.  Same results, much slower; for tests of that
 *   path. */
#define FGS_FLAG_LOOKBACK_FALLBACK 2u
/* FGS_FLAG_BLEND_QUEUE: the blend kernels (forward and backward) run as
 *   persistent waves, as many as the device holds at once, that take tiles
 *   from one queue per XCD (each XCD owns a band of consecutive tiles)
 *   instead of one workgroup per tile.  Same results; a scheduling choice
 *   for workloads with many more tiles than the device holds waves. */
#define FGS_FLAG_BLEND_QUEUE 4u
/* FGS_FLAG_SORT_LARGE_BLOCKS: the tile sort ranks and scatters blocks of
 *   8192 pairs instead of 4096 (longer digit runs per block to write out,
 *   fewer waves per SIMD).  Same results; a blocking choice for the
 *   autotuner, which times both on the workload. */
#define FGS_FLAG_SORT_LARGE_BLOCKS 8u
/* FGS_FLAG_KEEP_ACCUM_ZERO: for a caller that keeps its workspace for this
 *   library alone between calls (it writes no byte of it and hands its memory
 *   to no other use).  A backward pass whose chain rule reads the
 *   accumulators (fgs_rasterize_backward_adam, and every backward over
 *   several views) then clears each row and mark it reads, leaving accum and
 *   marks all zero, and records that in counters[12..13]; the next backward
 *   on the same layout skips their clear (n_views * n * 37 bytes).  Before
 *   the first call on a new workspace, or after its memory served anything
 *   else, zero counters[12..13] (or the whole workspace).  Same results. */
#define FGS_FLAG_KEEP_ACCUM_ZERO 16u

/* The Gaussian parameters of Sec. 2.1 ("3D Gaussian Splatting"): mean mu,
 * log-scales (scale = exp, "Activation Functions"), rotation quaternion
 * (w, x, y, z; normalised before use), opacity logit (opacity = sigmoid) and
 * degree-3 SH colour coefficients, with the DC band and the 15 higher bands
 * in separate buffers (Sec. 3.2, "Rasterization Kernel Fusion").
 *   means          [3][n]   world-space x, y, z planes
 *   log_scales     [3][n]
 *   quats          [4][n]   w, x, y, z planes (need not be normalised)
 *   opacity_logits [n]
 *   sh_dc          [3][n]   plane c = colour channel c
 *   sh_rest        [45][n]  plane (k-1)*3 + c for SH index k = 1..15
 * sh_dtype: FGS_F32, or FGS_BF16 for the precision form (SH coefficients
 * and their gradients stored as bfloat16; everything else, including all
 * blending, transmittance and gradient accumulation, stays float32).
 * sh_degree in 0..3 (planes beyond the degree are not read). n may be 0.
 * Dynamic scenes (the batched entry points, one time per view), two models:
 * - polynomial motion: velocity and accel [3][n] (both or neither; NULL =
 *   static) give the mean at time t as (means + velocity t) + accel t^2 in
 *   float32;
 * - conditional 4D Gaussians (Sec. 3.4 "Extension to Dynamic Scenes"):
 *   mean_t [n] (time of the mean), log_scale_t [n] (temporal log-scale) and
 *   quats_r [4][n] (right-isoclinic quaternion; quats is then the left one),
 *   all three or none, not together with velocity/accel.  The 4D rotation
 *   maps (x, y, z, t), read as the quaternion t + xi + yj + zk, to
 *   quats v quats_r (both normalised); Sigma4 = R diag(s^2) R^T; at time t a
 *   Gaussian is rendered as its conditional 3D Gaussian (mean mu_xyz +
 *   Sigma_xyz,t (t - mean_t) / Sigma_tt, covariance Sigma_xyz,xyz -
 *   Sigma_xyz,t Sigma_t,xyz / Sigma_tt) with opacity sigmoid(logit) times
 *   exp(-(t - mean_t)^2 / (2 Sigma_tt)); both quaternions are guarded
 *   against degenerate norms.                                              */
typedef struct fgs_gaussians {
  int64_t n;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const void* sh_dc;
  const void* sh_rest;
  int32_t sh_dtype;
  int32_t sh_degree;
  const float* velocity;
  const float* accel;
  const float* mean_t;
  const float* log_scale_t;
  const float* quats_r;
} fgs_gaussians;

/* Gradient planes with the layout of fgs_gaussians (all written in full);
 * sh_dc and sh_rest have the element type of the SH coefficients; velocity
 * and accel are written for polynomial motion, mean_t, log_scale_t and
 * quats_r for conditional 4D Gaussians (else unused). */
typedef struct fgs_gaussian_grads {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  void* sh_dc;
  void* sh_rest;
  float* velocity;
  float* accel;
  float* mean_t;
  float* log_scale_t;
  float* quats_r;
} fgs_gaussian_grads;

/* Pinhole camera of Eq. (1)-(2).  (host struct)
 * world_to_cam: W, row-major 4x4 (only rows 0-2 are used).  fx, fy, cx, cy:
 * intrinsics in pixels; pixel (i, j) is sampled at (i + 0.5, j + 0.5).
 * near_z: Gaussians with camera-space z below it are not rendered.
 * bg: background colour c_bg of Eq. (4).                                    */
typedef struct fgs_camera {
  float world_to_cam[16];
  float fx, fy, cx, cy;
  int32_t width, height;
  float near_z;
  float bg[3];
} fgs_camera;

/* Thresholds (host struct).  Defaults from fgs_default_settings:
 *   tile 16 (16x16 pixel tiles, Sec. 3.1)
 *   alpha_min 1/255  (skip fragments below it, Sec. 3.2 "Splat Bounding")
 *   alpha_max 0.99   (alpha cap, App. B.1; must be below 1, since the backward
 *                     divides by 1 - alpha)
 *   t_min 1e-4       (stop once the transmittance falls below it, App. B.1)
 *   dilation 0.3     (Sigma2D + 0.3 I, App. C.2)
 *   quat_min 1e-4, det_min 1e-6 (degenerate-Gaussian guard, App. B.1)
 * tile: 8, 16 or 32 pixels (one wavefront per tile in every case).         */
typedef struct fgs_settings {
  int32_t tile;
  float alpha_min;
  float alpha_max;
  float t_min;
  float dilation;
  float quat_min;
  float det_min;
  uint32_t flags; /* FGS_FLAG_* bits; others must be 0 */
} fgs_settings;

/* Filled by fgs_rasterize_forward when non-NULL (host struct). */
typedef struct fgs_forward_stats {
  int64_t n_visible;    /* Gaussians with at least one tile instance        */
  int64_t n_instances;  /* (tile, Gaussian) instances I                     */
  int64_t tiles_x, tiles_y;
  int64_t depth_key_bits; /* bits the depth sort needs: the visible depth
                             keys are sorted as key - min key, so 32 -
                             clz(max key - min key), 0 when all are equal
                             (see FGS_FORWARD_DEPTH_BITS)                  */
} fgs_forward_stats;

/* Byte offsets of the workspace regions (host struct), for inspection.
 * All regions are 256-byte aligned.  The forward pass leaves there:
 *   rec        float4[4*n]  per-Gaussian splat record (64 bytes), Gaussian order:
 *                           {mu2D.x, mu2D.y, opacity, 2 ln(opacity/alpha_min)},
 *                           {conic a, b, c (inverse of the dilated Sigma2D
 *                            [[a,b],[b,c]]), camera z}, {r, g, b, flags},
 *                           {tile rectangle (tx0 | ty0<<16, tx1 | ty1<<16) and
 *                            instance count, as uint32 bits; 0}
 *   n_tiles    uint32[n]    instances per Gaussian (0 = not rendered)
 *   depth_key  uint32[n]    bits of the FP32 camera z
 *   counters   uint32[16]   [0] visible count, [1] smallest and [2] largest
 *                           visible depth key, [3] index of the ping-pong buffer
 *                           holding the depth-sorted visible ids, [4..5] the
 *                           instance count I (uint64), [6] min(I, capacity),
 *                           [7] bit 0: I exceeded the capacity, bit 1: the
 *                           depth keys need more than FGS_FORWARD_DEPTH_BITS,
 *                           [8] the Gaussians with a gradient (fused backward),
 *                           [10..11] {0, max - min visible depth key},
 *                           [12..13] FGS_FLAG_KEEP_ACCUM_ZERO: a marker and
 *                           a tag of the layout while accum and marks are
 *                           known to be zero (any other value: not known)
 * With several views, the per-Gaussian regions (rec, n_tiles, depth_key,
 * vis_*, accum) hold n_views * n entries, entry v * n + i for view v.
 *   vis_ids    uint32[n] x2 ping-pong (see counters[3])
 *   dup_scan   the duplication's look-back words (offsets of each visible
 *                           Gaussian's instances are found in the kernel):
 *                           word 0 the number of workgroups whose look-back
 *                           wait ran out and that summed the earlier counts
 *                           directly (exact, only slower; 0 in normal
 *                           operation), from word 64 one 64-bit status per
 *                           256 entries
 *   inst_keys  uint16 or uint32 (inst_key_bytes) [cap] x2, inst_vals
 *                           uint32[cap] x2: global tile ids and Gaussian ids;
 *                           sorted in [inst_final].  Keys are 16-bit when
 *                           total_tiles < 65536, else 32-bit.
 *   ranges     uint32[2*tiles] [start, end) of each tile's list
 *   accum      float[n][9]  backward: dL/d(mu2D.x, mu2D.y, a, b, c, opacity, r, g, b),
 *                           one row of nine per (view, Gaussian) entry
 *   marks      uint8[n]     backward: nonzero when the entry's accumulator row
 *                           received a nonzero value (directly after accum)
 *   touched    uint8[ceil(n/4)]  fused backward + Adam: bit j of byte k set when
 *                           Gaussian 4k+j received a gradient
 *   touched_list uint32[n]  fused: the marked Gaussians (count in counters[8])
 *   slot_of    uint32[n]    fused: slot s of a marked Gaussian i (list[s] = i)
 *   sparse_grads float[59][n]  fused: plane p's gradient of list[s] at [p][s]
 *   queues     uint32[256]  FGS_FLAG_BLEND_QUEUE: the eight per-XCD tile
 *                           counters, 32 words apart */
typedef struct fgs_layout {
  size_t rec, n_tiles, depth_key, counters;
  size_t vis_keys[2], vis_ids[2];
  size_t dup_scan;
  size_t inst_keys[2], inst_vals[2];
  size_t ranges, accum, marks, touched, touched_list, slot_of, sparse_grads, queues, scratch, total;
  int32_t inst_final;
  int32_t inst_key_bytes;        /* 2 or 4: width of the inst_keys entries */
  int32_t tiles_x, tiles_y;      /* tile grid of view 0 */
  int64_t instance_capacity;
  int64_t n_views;
  int64_t total_tiles;           /* all views; tile ranges and sort keys span them */
} fgs_layout;

/* One Adam parameter group (host struct).  param and grad: [numel] of
 * `dtype` (FGS_F32, or FGS_BF16: widened, updated in float32 and rounded back
 * to nearest-even); exp_avg and exp_avg_sq: float32 [numel] in both cases.
 * lr: this group's learning rate. */
typedef struct fgs_adam_group {
  void* param;
  const void* grad;
  float* exp_avg;
  float* exp_avg_sq;
  int64_t numel;
  float lr;
  int32_t dtype;
} fgs_adam_group;

/* Optimizer state for fgs_rasterize_backward_adam (host struct of device
 * pointers).  Index order: means, log_scales, quats, opacity_logits, sh_dc,
 * sh_rest.  exp_avg[k] and exp_avg_sq[k] are float32 planes shaped like
 * parameter k (sh_rest: all 45 planes); lr[k] is its learning rate. */
typedef struct fgs_adam_moments {
  float* exp_avg[6];
  float* exp_avg_sq[6];
  float lr[6];
} fgs_adam_moments;

int32_t fgs_abi_version(void);
const char* fgs_status_string(fgs_status s);
/* Message of the last failing call on this thread ("" if none). */
const char* fgs_last_error(void);

/* Fills *out (host) with the defaults listed at fgs_settings. */
fgs_status fgs_default_settings(fgs_settings* out);

/* Workspace size in bytes (host *bytes) for n Gaussians, one camera, and
 * room for `instance_capacity` (tile, Gaussian) instances.  n (times the
 * views of a batch) and instance_capacity must stay below 2^30 (the limit of
 * the device sorts); larger values give FGS_ERR_INVALID_ARGUMENT. */
fgs_status fgs_workspace_size(int64_t n, const fgs_camera* cam, const fgs_settings* st,
                              int64_t instance_capacity, size_t* bytes);

/* Region offsets of that workspace (host *out). */
fgs_status fgs_workspace_layout(int64_t n, const fgs_camera* cam, const fgs_settings* st,
                                int64_t instance_capacity, fgs_layout* out);

/* Forward rasterization of one view (Sec. 2.1 Eq. (1)-(4); Sec. 3.2 "Splat
 * Bounding", "Tile-based Culling", "Sorting"; App. B.1-B.2):
 *  1. per Gaussian: activations, EWA projection to the dilated 2D conic,
 *     SH colour (clipped at 0), culling, opacity-aware tile rectangle, exact
 *     per-tile test, depth key;
 *  2. compaction of the visible Gaussians and a 32-bit radix sort by depth
 *     (stable, so depth ties keep index order; digit passes on bits that all
 *     visible keys share are skipped);
 *  3. duplication into (tile, Gaussian) instances and a stable radix sort by
 *     tile -- per-tile lists in (depth key, index) order -- and tile ranges;
 *  4. per tile, front-to-back blending with the 0.99 alpha cap, the
 *     alpha_min skip and termination once T < t_min (blend, then check).
 * Outputs (caller-allocated):
 *   image   float[3][height][width]  colour incl. T_final * bg, not clipped
 *   t_final float[height][width]     transmittance after the last fragment (nullable)
 *   last    uint32[height][width]    1 + position, in the pixel's tile list, of
 *                                    the last blended fragment (0 = none);
 *                                    required by fgs_rasterize_backward
 *   stats   (host, nullable)
 * The workspace must hold fgs_workspace_size(n, cam, st, instance_capacity)
 * bytes and is read again by fgs_rasterize_backward.  The call synchronises
 * `stream` once, after the preprocess, to read I.  If I > instance_capacity
 * it returns FGS_ERR_CAPACITY with stats->n_instances = I, having written no
 * image; grow the workspace and call again. */
fgs_status fgs_rasterize_forward(const fgs_gaussians* g, const fgs_camera* cam,
                                 const fgs_settings* st, void* workspace, size_t workspace_bytes,
                                 int64_t instance_capacity, float* image, float* t_final,
                                 uint32_t* last, fgs_forward_stats* stats, void* stream);

/* Backward pass of fgs_rasterize_forward (Sec. 3.2 "Per-Gaussian Backward",
 * App. B.1 front-to-back gradients, App. B.3): each tile is walked again in
 * the same order up to its last blended fragment, per-fragment gradients of
 * the loss w.r.t. mu2D, the conic, opacity and colour are reduced across the
 * pixels of a wavefront and accumulated per Gaussian, then chained back to
 * the raw parameters through the activations (Sec. 3.2 "Rasterization Kernel
 * Fusion").  Inputs: the same g, cam, st and workspace as the forward call
 * (unchanged since), its `image` and `last`, and dl_dimage float[3][h][w].
 * Output: every plane of *grads (host struct of device pointers) is written
 * in full; Gaussians that received no gradient get zeros. */
fgs_status fgs_rasterize_backward(const fgs_gaussians* g, const fgs_camera* cam,
                                  const fgs_settings* st, void* workspace, size_t workspace_bytes,
                                  int64_t instance_capacity, const float* image,
                                  const uint32_t* last, const float* dl_dimage,
                                  const fgs_gaussian_grads* grads, void* stream);

/* Backward pass fused with the Adam step (Sec. 3.3 "Fusing Backward and
 * Optimizer"): the blend backward of fgs_rasterize_backward; then one pass
 * marks and lists the Gaussians that received a gradient, the chain rule runs
 * for those only (their gradients go to compact slots of the workspace, no
 * full gradient buffer is written), and one streaming kernel applies Adam
 * with the moments of *opt to every parameter, with zero gradient for the
 * unmarked Gaussians.  Every parameter is updated, also those whose gradient
 * is zero, so the result equals fgs_rasterize_backward followed by
 * fgs_adam_step over the six groups (with bfloat16 SH, the SH gradient is
 * rounded to bfloat16 first, as a stored gradient would be).  The parameter
 * planes *g points to are updated in place and must be writable; sh_rest must
 * hold all 45 planes (planes beyond sh_degree get a zero gradient).  Other
 * arguments as for fgs_rasterize_backward and fgs_adam_step. */
fgs_status fgs_rasterize_backward_adam(const fgs_gaussians* g, const fgs_camera* cam,
                                       const fgs_settings* st, void* workspace, size_t workspace_bytes,
                                       int64_t instance_capacity, const float* image,
                                       const uint32_t* last, const float* dl_dimage,
                                       const fgs_adam_moments* opt, int64_t step, double beta1,
                                       double beta2, double eps, void* stream);

/* Fused Adam over several parameter groups in one launch (Sec. 3.3
 * "Parameter Updates"; hyperparameters App. A): for every element,
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   p <- p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps),
 * including elements whose gradient is zero.  groups: host array of
 * n_groups (1..16) descriptors; step t >= 1.  The hyperparameters are taken
 * in double so that 1 - beta and the bias corrections are formed before
 * rounding to float32, as PyTorch does. */
fgs_status fgs_adam_step(const fgs_adam_group* groups, int32_t n_groups, int64_t step,
                         double beta1, double beta2, double eps, void* stream);

/* fgs_adam_step with the step count on the device, for a step captured into
 * a graph and replayed: d_state is a device buffer of at least 256 bytes,
 * 8-byte aligned, whose first int64 is the step counter t (zero it before
 * the first step); each call increments it, forms the bias corrections of
 * the new t on the device (in double, as fgs_adam_step does on the host) and
 * applies Adam.  The rest of the buffer is the call's scratch. */
fgs_status fgs_adam_step_device(const fgs_adam_group* groups, int32_t n_groups, void* d_state, double beta1,
                                double beta2, double eps, void* stream);

/* L1 loss term of Sec. 2.1 / App. A: dl_dimage[i] = sign(image[i] - target[i]) / n
 * (sign(0) = 0) for i < n; when loss (device double, nullable) is given, it
 * receives mean |image - target| reduced in float64. */
fgs_status fgs_l1_loss_backward(const float* image, const float* target, int64_t n,
                                float* dl_dimage, double* loss, void* stream);

/* Z-order layout (Sec. 3.3 "Locality-preserving Densification"): re-sorting
 * the Gaussians in Morton order of their means places Gaussians that are
 * close in 3D close in memory, which the gathers of the rasterizer and the
 * scattered updates of the fused backward + Adam benefit from; the paper
 * applies it every few thousand iterations.  Conventions: bounding cube of
 * the means with side the largest per-axis extent; 10 bits per axis,
 * q = min(1023, floor((x - min) * (1024 / side))) in float32; codes interleave
 * the bits with x in bit 0; ties keep the index order (stable).
 * fgs_zorder_workspace_size: device scratch bytes for n Gaussians (host *bytes);
 *   n < 2^30.
 * fgs_zorder_permutation: perm[k] (device uint32[n]) = index of the Gaussian at
 *   position k; means float32 [3][n] (finite); workspace 256-byte aligned. */
fgs_status fgs_zorder_workspace_size(int64_t n, size_t* bytes);
fgs_status fgs_zorder_permutation(const float* means, int64_t n, void* workspace, size_t workspace_bytes,
                                  uint32_t* perm, void* stream);
/* Gather of `planes` planes of n elements of elem_bytes (2 or 4) bytes:
 * dst[p][k] = src[p][perm[k]] (apply a z-order permutation to parameters and
 * optimizer moments alike).  src and dst must not overlap. */
fgs_status fgs_permute_planes(const void* src, void* dst, int64_t n, int32_t planes, int32_t elem_bytes,
                              const uint32_t* perm, void* stream);

/* Stable radix sort of (key, value) pairs, the device sort the forward runs
 * by depth (32-bit keys) and by tile (16- or 32-bit keys) (Sec. 3.2
 * "Sorting"): afterwards the pairs are ordered by the value of key bits
 * [0, key_bits), and pairs with equal such bits keep their input order; bits
 * at and above key_bits are carried along unsorted.  keys: device array of
 * n keys of key_bytes (2 or 4) bytes; vals: device uint32[n]; both sorted in
 * place; n < 2^30.  key_bits: 0..8*key_bytes (0 leaves the arrays as they
 * are).
 * workspace: device, 256-byte aligned, at least fgs_sort_workspace_size bytes
 * (host *bytes); its contents are scratch.  Errors: FGS_ERR_INVALID_ARGUMENT
 * for a bad size, width, pointer or workspace; nothing is launched then. */
fgs_status fgs_sort_workspace_size(int64_t n, int32_t key_bytes, size_t* bytes);
fgs_status fgs_sort_pairs(void* keys, uint32_t* vals, int64_t n, int32_t key_bytes, int32_t key_bits,
                          void* workspace, size_t workspace_bytes, void* stream);

/* fgs_sort_pairs without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as fgs_sort_pairs, minus
 * the workspace: the scratch is a static device array of
 * FGS_SORT_NOALLOC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends, so n is limited to
 * FGS_SORT_NOALLOC_MAX_PAIRS (a larger n returns FGS_ERR_INVALID_ARGUMENT
 * and launches nothing).  The call allocates nothing; its first call on a
 * device looks up the array's address there (the device must be current and
 * `stream`, when not NULL, must belong to it).  Every call on a device shares
 * that device's array: calls that overlap on one device (other threads,
 * other streams) race and give wrong results; serialise them.  Nothing in the
 * array has to start at a particular value. */
#define FGS_SORT_NOALLOC_MAX_PAIRS (1 << 20)
#define FGS_SORT_NOALLOC_SCRATCH_BYTES ((size_t)17 << 19) /* 8.5 MiB */
fgs_status fgs_sort_pairs_noalloc(void* keys, uint32_t* vals, int64_t n, int32_t key_bytes, int32_t key_bits,
                                  void* stream);

/* Batched views (several cameras, or timesteps of a dynamic scene, rendered
 * and differentiated in one pass; the paper renders image batches per
 * iteration for its 4D extension, Sec. 3.4).  Up to FGS_MAX_VIEWS cameras
 * cams[0..n_views) (host array); times[v] (host, nullable = all 0) is the time
 * of view v for dynamic Gaussians.  Every (view, Gaussian) pair is
 * preprocessed; all pairs share one depth sort, instances are keyed by a
 * global tile id (the tiles of view 0, then view 1, ...) and one stable tile
 * sort, and one launch blends every tile of every view.  images: the views'
 * [3][H_v][W_v] blocks one after another; t_finals (nullable) and lasts the
 * views' [H_v][W_v] planes one after another.  The per-view results equal
 * those of single-view calls; the backward sums each Gaussian's gradient
 * over the views (and, for dynamic Gaussians, writes dL/dvelocity =
 * sum_v t_v dL/dmean_v and dL/daccel = sum_v t_v^2 dL/dmean_v).
 * mode FGS_FORWARD_NO_SYNC: the forward call never synchronises the stream,
 * so the whole step can be captured into a graph; every launch is sized by
 * the capacities and reads the counts from the workspace counters, *stats is
 * not filled (n_visible = n_instances = depth_key_bits = -1), and an instance
 * count above the capacity sets bit 0 of counters[7] (the image is then
 * incomplete: grow the capacity, re-capture and run again).  Without it the
 * call behaves like fgs_rasterize_forward (one synchronisation,
 * FGS_ERR_CAPACITY).
 * The depth sort orders the visible keys minus the smallest (same order and
 * ties: keys are the bits of positive floats); the host-synchronised call
 * sorts the bits of max - min only.
 * mode | FGS_FORWARD_DEPTH_BITS(b), 1 <= b <= 31, only with
 * FGS_FORWARD_NO_SYNC: max - min is taken to fit in b bits (the
 * depth_key_bits a synchronised call reported) and the depth sort covers
 * those (without it all 31, up to one more radix pass; trailing passes whose
 * digit is the same in every key find that on the device and do no work, at
 * the cost of their launches).  A wider span sets bit 1 of counters[7]: the
 * depth order, and so the image, is then wrong; run a synchronised call,
 * re-capture with its depth_key_bits and run again. */
#define FGS_MAX_VIEWS 16
#define FGS_FORWARD_NO_SYNC 1u
#define FGS_FORWARD_DEPTH_BITS(b) ((uint32_t)(b) << 8)
fgs_status fgs_batch_workspace_size(int64_t n, const fgs_camera* cams, int32_t n_views, const fgs_settings* st,
                                    int64_t instance_capacity, size_t* bytes);
fgs_status fgs_batch_workspace_layout(int64_t n, const fgs_camera* cams, int32_t n_views, const fgs_settings* st,
                                      int64_t instance_capacity, fgs_layout* out);
fgs_status fgs_rasterize_forward_batch(const fgs_gaussians* g, const fgs_camera* cams, const float* times,
                                       int32_t n_views, const fgs_settings* st, void* workspace,
                                       size_t workspace_bytes, int64_t instance_capacity, float* images,
                                       float* t_finals, uint32_t* lasts, uint32_t mode, fgs_forward_stats* stats,
                                       void* stream);
fgs_status fgs_rasterize_backward_batch(const fgs_gaussians* g, const fgs_camera* cams, const float* times,
                                        int32_t n_views, const fgs_settings* st, void* workspace,
                                        size_t workspace_bytes, int64_t instance_capacity, const float* images,
                                        const uint32_t* lasts, const float* dl_dimages,
                                        const fgs_gaussian_grads* grads, void* stream);

/* Timing hook for measurement: arms a one-shot timer on the calling thread.
 * The next time this thread's library calls run `step`, start_event is
 * recorded on the call's stream just before it and stop_event just after it
 * (hipEvent_t handles created by the caller); the hook is then disarmed.
 * Steps (one kernel each unless noted): "preprocess", "duplicate",
 * "tile_sort" (all passes of the tile radix sort), "blend_forward",
 * "blend_backward", "preprocess_backward", and for
 * fgs_rasterize_backward_adam "touched_gradients" (marks, list and chain rule
 * of the Gaussians with a gradient: three launches) and "adam_sparse" (the
 * Adam step of every parameter), "adam".  step = NULL
 * disarms.  An unknown name returns FGS_ERR_INVALID_ARGUMENT. */
fgs_status fgs_time_next_launch(const char* step, void* start_event, void* stop_event);

#ifdef __cplusplus
}
#endif
#endif /* FASTERGS_H */
