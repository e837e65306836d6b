// Internal declarations shared by the HIP translation units of libfastergs.
// Device helpers here are header-only so that every kernel that needs the same
// decision (the tile test) runs the identical instruction sequence.
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>

#include "../../include/fastergs.h"

namespace fgs {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWave = 64;
// items per thread in the 32-bit-key radix kernels (a build-time tuning constant)
#ifndef FGS_SORT32_ITEMS
#define FGS_SORT32_ITEMS 16
#endif
constexpr int kScanItems = FGS_SORT32_ITEMS;
constexpr int kSortItemsLarge = 32;  // pairs per thread of a sort's large blocks (8192 pairs)
// pairs per thread of the 16-bit-key sort (a build-time tuning constant)
#ifndef FGS_SORT16_ITEMS
#define FGS_SORT16_ITEMS 16
#endif
constexpr int64_t kMaxSortPairs = int64_t(1) << 30;  // a device sort takes fewer pairs
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kNumXcd = 8;           // MI355X: 8 XCDs, workgroups dealt round-robin

// Camera as the kernels see it.
struct CamDev {
  float w[12];        // rows 0..2 of the world-to-camera matrix, row-major 3x4
  float campos[3];    // camera centre in world space, -W3^T t
  float fx, fy, cx, cy;
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  float near_z;
  float bg[3];
};

// Up to kMaxViews cameras rendered in one pass (batched views, or timesteps of
// a dynamic scene).  Passed by value as a kernel argument, so a captured graph
// carries it.  A single view is n_views = 1.
constexpr int kMaxViews = 16;
struct ViewSet {
  CamDev cam[kMaxViews];
  float time[kMaxViews];                // t of each view (dynamic means; 0 otherwise)
  uint32_t tile_base[kMaxViews + 1];    // first global tile of each view; [n_views] = total tiles
  uint64_t pix_base[kMaxViews + 1];     // first pixel of each view in the concatenated images
  uint32_t n_views;
};

// View of global tile t (tile_base is increasing).
__device__ __forceinline__ uint32_t view_of_tile(const ViewSet& vs, uint32_t t) {
  uint32_t v = 0;
#pragma unroll 1
  while (v + 1 < vs.n_views && t >= vs.tile_base[v + 1]) ++v;
  return v;
}

struct SetDev {
  float alpha_min, alpha_max, t_min, dilation, quat_min, det_min;
  int32_t fp64_conic;  // determinant and 2x2 inverse in float64 (precision form)
};

// SH planes hold float32 or bfloat16 elements (sh_bf16); kernels that touch
// them are instantiated for both.
struct GaussDev {
  const float* means;
  const float* velocity;  // dynamic scenes: mean(t) = means + velocity t + accel t^2 (NULL: static)
  const float* accel;
  const float* log_scales;
  const float* quats;
  const float* logits;
  const void* sh_dc;
  const void* sh_rest;
  // conditional 4D Gaussians (NULL: 3D): time of the mean, temporal
  // log-scale, right-isoclinic quaternion [4][n] (quats is the left one)
  const float* mean_t;
  const float* log_scale_t;
  const float* quats_r;
  uint32_t n;
  int32_t sh_coeffs;  // (degree + 1)^2
  int32_t sh_bf16;
};

struct GradDev {
  float* means;
  float* velocity;  // written when the Gaussians are dynamic
  float* accel;
  float* log_scales;
  float* quats;
  float* logits;
  void* sh_dc;  // element type of the SH parameters
  void* sh_rest;
  float* mean_t;  // written for conditional 4D Gaussians
  float* log_scale_t;
  float* quats_r;
};

// bfloat16 <-> float32.  Widening is exact; narrowing rounds to nearest, ties
// to even (add 0x7fff plus the lowest kept bit, then truncate), NaN stays NaN.
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
template <bool BF16>
__device__ __forceinline__ float sh_load(const void* p, size_t idx) {
  if constexpr (BF16) return bf16_to_f32(static_cast<const uint16_t*>(p)[idx]);
  else return static_cast<const float*>(p)[idx];
}
template <bool BF16>
__device__ __forceinline__ void sh_store(void* p, size_t idx, float v) {
  if constexpr (BF16) static_cast<uint16_t*>(p)[idx] = f32_to_bf16(v);
  else static_cast<float*>(p)[idx] = v;
}
// The value a float32 takes once stored in the SH element type.
template <bool BF16>
__device__ __forceinline__ float sh_round(float v) {
  if constexpr (BF16) return bf16_to_f32(f32_to_bf16(v));
  else return v;
}

// One Adam element in torch.optim.Adam's float32 order (Sec. 3.3 "Parameter
// Updates"):  m += (1 - b1)(g - m);  v = b2 v + (1 - b2) g^2;
//             p -= step_size * m / (sqrt(v) / sqrt(1 - b2^t) + eps),
// with step_size = lr / (1 - b1^t).  Shared by the optimizer kernel and the
// fused backward + optimizer kernel so both give identical results.
struct AdamCoef {
  float one_minus_b1, beta2, one_minus_b2, inv_sqrt_bc2, eps;
};
__device__ __forceinline__ void adam_elem(float& p, float g, float& m, float& v, const AdamCoef& a, float step) {
#pragma clang fp contract(on)
  m = fmaf(a.one_minus_b1, g - m, m);
  v = fmaf(a.one_minus_b2, g * g, v * a.beta2);
  const float denom = sqrtf(v) * a.inv_sqrt_bc2 + a.eps;
  p = p - step * (m / denom);
}
// Host side: coefficients from double hyperparameters (1 - beta and the bias
// corrections are formed in double before rounding, as PyTorch does).
AdamCoef adam_coef(int64_t step, double beta1, double beta2, double eps, double* bias1);

// ----------------------------------------------------------------------------
// Workgroup -> tile mapping.  Workgroups are dealt to the 8 XCDs round-robin
// (workgroup b runs on XCD b % 8).  Giving each XCD a contiguous band of
// tiles keeps the splat records that neighbouring tiles share in one L2.
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb) {
  const uint32_t xcd = b % kNumXcd;
  const uint32_t local = b / kNumXcd;
  const uint32_t base = nb / kNumXcd, rem = nb % kNumXcd;
  // XCD x owns tiles [start(x), start(x) + base + (x < rem)).
  const uint32_t start = xcd * base + (xcd < rem ? xcd : rem);
  return start + local;
}

// ----------------------------------------------------------------------------
// Exact tile test (FP32, fixed operation order, no contraction).
// Keeps a tile when the minimum of d^T [[a,b],[b,c]] d over the tile's
// pixel-centre hull (clipped to the image) is <= thr = 2 ln(o / alpha_min).
// ----------------------------------------------------------------------------
// The minimiser along an edge is -(b d) / c (vertical edge) or -(b d) / a
// (horizontal), taken as -(b d) * (1/c) with the reciprocal rounded once per
// Gaussian (ra = 1/a, rc = 1/c).
__device__ __forceinline__ float edge_min_q(float a, float b, float c, float ra, float rc, float dfix,
                                            float m_other, float lo, float hi, bool fix_is_x) {
#pragma clang fp contract(off)
  float t = fix_is_x ? (-(b * dfix)) * rc : (-(b * dfix)) * ra;
  float p = fminf(fmaxf(m_other + t, lo), hi);
  float dvar = p - m_other;
  float dx = fix_is_x ? dfix : dvar;
  float dy = fix_is_x ? dvar : dfix;
  return ((a * dx) * dx + ((b + b) * dx) * dy) + (c * dy) * dy;
}

// The hull is [x0, x1] x [y0, y1] in pixel centres: x0 = tx*tile + 0.5 and
// x1 = min(x0 + tile - 1, width - 0.5), likewise in y (integers + 0.5, exact
// in FP32).
__device__ __forceinline__ bool tile_keep(float mx, float my, float a, float b, float c, float ra, float rc,
                                          float thr, float x0, float x1, float y0, float y1) {
#pragma clang fp contract(off)
  const bool left = mx < x0, right = mx > x1, top = my < y0, bottom = my > y1;
  // At most one vertical and one horizontal edge face the centre (left and
  // right exclude each other, as do top and bottom): the minimum over the hull
  // is the smaller of those two edge minima, and 0 inside the hull.  Both are
  // evaluated and selected without divergent branches.
  const bool out_x = left || right, out_y = top || bottom;
  const float qX = edge_min_q(a, b, c, ra, rc, (left ? x0 : x1) - mx, my, y0, y1, true);
  const float qY = edge_min_q(a, b, c, ra, rc, (top ? y0 : y1) - my, mx, x0, x1, false);
  const float inf = __builtin_huge_valf();
  const float q = fminf(out_x ? qX : inf, out_y ? qY : inf);
  return !(out_x || out_y) || q <= thr;
}

// Conditional 4D Gaussian at time t (Sec. 3.4 "Extension to Dynamic
// Scenes").  The 4D rotation maps (x, y, z, t), read as the quaternion
// t + xi + yj + zk, to ql v qr with both quaternions normalised: in (w, x,
// y, z) coordinates the product L(ql) R(qr) of the left- and
// right-multiplication matrices, then reordered to (x, y, z, t).
// Sigma4 = M M^T with M = R diag(exp(ls4)); the conditional mean is
// mu + Sigma_xyz,t (t - mean_t) / Sigma_tt, the covariance the Schur
// complement Sigma_xyz,xyz - Sigma_xyz,t Sigma_t,xyz / Sigma_tt, and the
// opacity factor exp(-(t - mean_t)^2 / (2 Sigma_tt)).
//
// Evaluated in a projection form: with m the time row of M (Sigma_tt =
// |m|^2) and u = m / |m|, h = M_xyz u and e = (t - mean_t) / |m|, the mean
// shift is h e, the factor exp(-e^2 / 2) and the covariance N N^T with
// N = M_xyz - h u^T (M_xyz projected off u).  The Schur complement would
// subtract two products of size |M_xyz|^2 and lose that much absolute
// accuracy; N carries an error of order |M_xyz| only, so for a Gaussian
// elongated along a direction that mixes space and time the conditional
// covariance keeps about the square root of the relative error.  One
// rounding per operation (contraction off).  S holds the covariance entries
// 00, 01, 02, 11, 12, 22; qn is the smaller quaternion norm (the degenerate
// guard takes both).
struct Cond4 {
  float mu[3];
  float S[6];
  float p;
  float qn;
};

__device__ __forceinline__ void unit_quat(const float* q, float* u, float& qn) {
#pragma clang fp contract(off)
  qn = sqrtf(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  u[0] = q[0] / qn;
  u[1] = q[1] / qn;
  u[2] = q[2] / qn;
  u[3] = q[3] / qn;
}

// L(a) and R(b) of quaternion products a v = L(a) v and v b = R(b) v, (w, x, y, z).
__device__ __forceinline__ void quat_lr(const float* a, const float* b, float (&L)[4][4], float (&R)[4][4]) {
  L[0][0] = a[0]; L[0][1] = -a[1]; L[0][2] = -a[2]; L[0][3] = -a[3];
  L[1][0] = a[1]; L[1][1] = a[0];  L[1][2] = -a[3]; L[1][3] = a[2];
  L[2][0] = a[2]; L[2][1] = a[3];  L[2][2] = a[0];  L[2][3] = -a[1];
  L[3][0] = a[3]; L[3][1] = -a[2]; L[3][2] = a[1];  L[3][3] = a[0];
  R[0][0] = b[0]; R[0][1] = -b[1]; R[0][2] = -b[2]; R[0][3] = -b[3];
  R[1][0] = b[1]; R[1][1] = b[0];  R[1][2] = b[3];  R[1][3] = -b[2];
  R[2][0] = b[2]; R[2][1] = -b[3]; R[2][2] = b[0];  R[2][3] = b[1];
  R[3][0] = b[3]; R[3][1] = b[2];  R[3][2] = -b[1]; R[3][3] = b[0];
}

// 4D rotation in (x, y, z, t) order from unit quaternions a (left), b (right).
__device__ __forceinline__ void rotation4(const float* a, const float* b, float (&R4)[4][4]) {
#pragma clang fp contract(off)
  float L[4][4], Rq[4][4];
  quat_lr(a, b, L, Rq);
  constexpr int pm[4] = {1, 2, 3, 0};  // x, y, z, t -> w, x, y, z index
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = pm[r], j = pm[c];
      R4[r][c] = ((L[i][0] * Rq[0][j] + L[i][1] * Rq[1][j]) + L[i][2] * Rq[2][j]) + L[i][3] * Rq[3][j];
    }
}

// Projection-form conditioning of M (rows x, y, z, t) at dt = t - mean_t:
// h, e and the covariance entries as described above.
__device__ __forceinline__ void condition_m(const float (&M)[4][4], float dt, float (&h)[3], float& e,
                                            float (&S)[6]) {
#pragma clang fp contract(off)
  const float nt = sqrtf(((M[3][0] * M[3][0] + M[3][1] * M[3][1]) + M[3][2] * M[3][2]) + M[3][3] * M[3][3]);
  const float inv = 1.0f / nt;
  const float u[4] = {M[3][0] * inv, M[3][1] * inv, M[3][2] * inv, M[3][3] * inv};
  e = dt * inv;
  float N[3][4];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    h[r] = ((M[r][0] * u[0] + M[r][1] * u[1]) + M[r][2] * u[2]) + M[r][3] * u[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) N[r][k] = M[r][k] - h[r] * u[k];
  }
  auto nn = [&](int r, int q) {
    return ((N[r][0] * N[q][0] + N[r][1] * N[q][1]) + N[r][2] * N[q][2]) + N[r][3] * N[q][3];
  };
  S[0] = nn(0, 0);
  S[1] = nn(0, 1);
  S[2] = nn(0, 2);
  S[3] = nn(1, 1);
  S[4] = nn(1, 2);
  S[5] = nn(2, 2);
}

__device__ __forceinline__ Cond4 condition4d(const float* ql, const float* qr, const float* ls4, float mean_t,
                                             float t, float mu0, float mu1, float mu2) {
#pragma clang fp contract(off)
  Cond4 c;
  float a[4], b[4], qna, qnb;
  unit_quat(ql, a, qna);
  unit_quat(qr, b, qnb);
  float R4[4][4];
  rotation4(a, b, R4);
  const float s[4] = {expf(ls4[0]), expf(ls4[1]), expf(ls4[2]), expf(ls4[3])};
  float M[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) M[r][k] = R4[r][k] * s[k];
  float h[3], e;
  condition_m(M, t - mean_t, h, e, c.S);
  c.mu[0] = mu0 + h[0] * e;
  c.mu[1] = mu1 + h[1] * e;
  c.mu[2] = mu2 + h[2] * e;
  c.p = expf(-(0.5f * (e * e)));
  c.qn = fminf(qna, qnb);
  return c;
}

// Decode the packed tile rectangle.
__device__ __forceinline__ void unpack_rect(uint2 r, int& tx0, int& ty0, int& tx1, int& ty1) {
  tx0 = (int)(r.x & 0xffffu);
  ty0 = (int)(r.x >> 16);
  tx1 = (int)(r.y & 0xffffu);
  ty1 = (int)(r.y >> 16);
}

// ----------------------------------------------------------------------------
// Wave / block primitives (wave64, 256-thread blocks).
// ----------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t y = __shfl_up(v, d, kWave);
    if (lane >= d) v += y;
  }
  return v;
}

// Exclusive scan across the 256 threads of a block; *total gets the block sum.
// `lds` must hold kBlock / kWave words.  Contains two barriers.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  uint32_t inc = wave_inclusive_scan(v, lane);
  if (lane == kWave - 1) lds[wave] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    uint32_t s = lds[w];
    pre += (w < wave) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

__device__ __forceinline__ uint32_t block_reduce_sum(uint32_t v, uint32_t* lds) {
  uint32_t t;
  block_exclusive_scan(v, lds, &t);
  return t;
}

// ----------------------------------------------------------------------------
// Load-balanced walk over candidate tiles (wave64).  Each lane holds one
// Gaussian and its candidate tiles (the tile rectangle, row-major).  The wave
// visits all candidates of its 64 Gaussians 64 at a time, in (lane, tile)
// order, so every lane tests one candidate per step whatever the rectangle
// sizes.  Every step calls emit(owner_lane, rank, tx, ty, keep) in all lanes
// (uniform control flow, so emit may use cross-lane shuffles); for a kept tile
// rank is its index among all kept tiles of the wave in that order, so the
// wave's kept tiles map to one contiguous run of output slots.
// ----------------------------------------------------------------------------
struct CandLane {
  float mx, my, a, b, c, thr;
  int tx0, ty0, w;  // rectangle origin and width in tiles
  uint32_t cand;    // candidate tiles (0: none)
  int width, height;  // image of this Gaussian's view
};

// floor(r / w) for r < 2^31 from m = floor((2^32 - 1) / w): the high word of
// r m is floor(r / w) or one less, and one step corrects it.  Tile
// coordinates are 16-bit, so the quotient and w fit the 24-bit multiplier.
__device__ __forceinline__ uint32_t div_magic(uint32_t w) { return 0xffffffffu / w; }
__device__ __forceinline__ uint32_t udiv_magic(uint32_t r, uint32_t w, uint32_t m) {
  const uint32_t q = __umulhi(r, m);
  return __umul24(q + 1u, w) <= r ? q + 1u : q;
}

// What a lane needs of the Gaussian that owns its candidate: staged in LDS
// once per walk and read with three 16-byte loads per step (instead of a
// cross-lane shuffle per field).
struct alignas(16) OwnerRec {
  float mx, my, a, b;
  float c, thr, ra, rc;    // ra = 1/a, rc = 1/c (the tile test's reciprocals)
  float x0b, y0b;          // pixel-centre origin of the rectangle: tx0*tile + 0.5, ty0*tile + 0.5
  float xmax, ymax;        // last pixel centres of the view: width - 0.5, height - 0.5
  int w;                   // rectangle width in tiles
  uint32_t cstart;         // first candidate's position in the wave's candidate list
  uint32_t wmagic;         // div_magic(w)
  uint32_t txy0;           // tx0 | ty0 << 16
};

// LDS of one wave's walk.
struct WalkLds {
  OwnerRec own[kWave];
  uint32_t owner_at[kWave];
};

// A volatile pointer into LDS that keeps its address space: through a plain
// volatile pointer the compiler emits flat (system-coherent) loads and stores
// and waits on them like on memory.
typedef __attribute__((address_space(3))) volatile uint32_t lds_volatile_u32;
template <typename T>
__device__ __forceinline__ lds_volatile_u32* lds_volatile(T* p) {
  return (lds_volatile_u32*)(p);
}

// Orders a wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One step of a load-balanced walk over a wave's list of items, where lane l
// owns the run [start, start + len) of the list (runs in lane order): the
// lane owning position c0 + lane.  The owner of each run that starts in (or
// runs into) the step claims the run's first position in owner_at with the
// step's tag; position q belongs to the last claim at or below q.  claims /
// first: whether this lane's run meets the step, and its first position in
// the step.  owner_at must hold no tag of this step beforehand (tags grow by
// 0x100 per step and owner_at starts at 0xffffffff).
__device__ __forceinline__ int wave_run_owner(uint32_t start, uint32_t len, uint32_t c0, uint32_t tag,
                                              lds_volatile_u32* owner_at, uint64_t upto, bool& claims,
                                              uint32_t& first) {
  const int lane = threadIdx.x & (kWave - 1);
  claims = len > 0 && start < c0 + kWave && start + len > c0;
  first = start > c0 ? start - c0 : 0u;
  if (claims) owner_at[first] = tag | (uint32_t)lane;
  const uint32_t mine = owner_at[lane];
  const uint64_t claimed = __ballot((mine & ~0xffu) == tag);
  const uint64_t m = claimed & upto;
  const int src_slot = m ? 63 - __clzll(m) : 0;
  return (int)(owner_at[src_slot] & 0xffu);
}

// emit(owner, const OwnerRec&, rank among the wave's kept tiles, tx, ty, keep)
// is called by every lane at every step (uniform control flow); LDS the
// caller wrote before the call is visible to all lanes inside emit.
// RANKS = true: returns the number of kept tiles of the whole wave (the same
// in every lane).  RANKS = false (a walk that only counts): the ranks passed
// to emit are 0 and each lane gets the kept tiles of its own Gaussian.
template <bool RANKS, typename Emit>
__device__ __forceinline__ uint32_t wave_tile_walk(const CandLane& me, WalkLds& L, int tile, Emit emit) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t incl = wave_inclusive_scan(me.cand, lane);
  const uint32_t cstart = incl - me.cand;
  const uint32_t total = __shfl(incl, kWave - 1, kWave);
  const uint64_t upto = ((lane == 0) ? 0ull : (~0ull >> (64 - lane))) | (1ull << lane);
  const float ftile = (float)tile, ftile1 = (float)(tile - 1);
  // RANKS: wave-uniform count of the kept candidates of the earlier steps;
  // else this lane's Gaussian's kept tiles so far
  uint32_t running = 0;
  uint32_t tag = 0;
  {
#pragma clang fp contract(off)
    const float ra = me.cand ? 1.0f / me.a : 0.0f, rc = me.cand ? 1.0f / me.c : 0.0f;
    const int sh = __builtin_ctz((unsigned)tile);
    L.own[lane] = OwnerRec{me.mx, me.my, me.a, me.b, me.c, me.thr, ra, rc,
                           (float)(me.tx0 << sh) + 0.5f, (float)(me.ty0 << sh) + 0.5f,
                           (float)(me.width - 1) + 0.5f, (float)(me.height - 1) + 0.5f,
                           me.w, cstart, div_magic((uint32_t)max(me.w, 1)),
                           (uint32_t)me.tx0 | ((uint32_t)me.ty0 << 16)};
  }
  lds_volatile_u32* owner_at = lds_volatile(L.owner_at);
  owner_at[lane] = 0xffffffffu;  // no step tag matches
  wave_lds_sync();
  for (uint32_t c0 = 0; c0 < total; c0 += kWave, tag += 0x100u) {
    bool claims;
    uint32_t slot;
    const int owner = wave_run_owner(cstart, me.cand, c0, tag, owner_at, upto, claims, slot);
    const uint32_t pos = c0 + (uint32_t)lane;
    const bool valid = pos < total;
    const OwnerRec o = L.own[owner];
    const uint32_t r = pos - o.cstart;
    const uint32_t ry = udiv_magic(r, (uint32_t)o.w, o.wmagic);
    const uint32_t rx = r - __umul24(ry, (uint32_t)o.w);
    const float x0 = fmaf((float)rx, ftile, o.x0b), y0 = fmaf((float)ry, ftile, o.y0b);
    const float x1 = fminf(x0 + ftile1, o.xmax), y1 = fminf(y0 + ftile1, o.ymax);
    const int tx = (int)(o.txy0 & 0xffffu) + (int)rx;
    const int ty = (int)(o.txy0 >> 16) + (int)ry;
    const bool keep = tile_keep(o.mx, o.my, o.a, o.b, o.c, o.ra, o.rc, o.thr, x0, x1, y0, y1) & valid;
    if (!RANKS) {
      // the claiming lane adds the kept tiles of its Gaussian's segment of
      // this step (an LDS atomic per kept tile serialises on the owner's
      // counter and was slower)
      const uint64_t kb = __ballot(keep);
      if (claims) {
        const uint32_t hi = min(cstart + me.cand - c0, (uint32_t)kWave);  // exclusive
        const uint64_t seg = (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull)) & ~((slot == 0) ? 0ull : ((1ull << slot) - 1ull));
        running += (uint32_t)__popcll(kb & seg);
      }
      emit(owner, o, 0u, tx, ty, keep);
      continue;
    }
    const uint64_t kb = __ballot(keep);
    const uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(kb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)kb, 0u));
    emit(owner, o, running + before, tx, ty, keep);  // uniform call
    running += (uint32_t)__popcll(kb);
  }
  return running;
}

// Records the calling thread's error message (fgs_last_error) and returns s.
fgs_status fail(fgs_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }
// a word count rounded up to a multiple of 64 words (256 bytes)
inline uint64_t round_up64(uint64_t w) { return (w + 63) & ~uint64_t(63); }

// ----------------------------------------------------------------------------
// Host-side launchers (each .hip file owns its kernels).
// ----------------------------------------------------------------------------
// p[0..n) = v (a kernel, so captured graphs contain no memset nodes); the
// same launch also sets *word = word_v when word is given.
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s, uint32_t* word = nullptr,
                           uint32_t word_v = 0u);

// The backward's gradient accumulator and marks are known to be zero when
// the counter pair [kStatAccumClean, +1] reads {kAccumClean, the layout's
// tag}; the blend backward breaks the pair before it adds, and the backwards
// that zero every row they read restore it at their end.
constexpr uint32_t kAccumClean = 0x5a3c0f81u;
// p[0..n) = 0 (p 16-byte aligned) unless flag[0..2) = {kAccumClean, tag}.
hipError_t launch_clear_unless(uint32_t* p, uint64_t n, const uint32_t* flag, uint32_t tag, hipStream_t s);

// Scratch words needed by scan_u32 for n items.
size_t scan_scratch_words(uint64_t n);
// Exclusive scan of in[0..n) into out (which may alias in); writes the grand
// total to *d_total when d_total != NULL.
hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* d_total, uint32_t* scratch,
                    hipStream_t s);

size_t radix_scratch_words(uint64_t n);
// Stable LSD radix sort of (key, value) pairs on bits [begin_bit, end_bit).
// Items: n (host, < 2^30) or *d_count (device, <= n) when d_count != NULL.
// Data starts in keys[0]/vals[0]; returns (in *final_buf) the buffer holding
// the result.  d_range (device, optional): {min, max} of the keys; the
// trailing passes whose digit is the same in every key are then skipped, and
// the buffer holding the result is written to the device word final_word
// (required then; *final_buf is -1).  keep_keys = false: the last pass writes
// the values only (the sorted keys are not needed).
// large_blocks: blocks of kBlock * kSortItemsLarge pairs instead of the
// default shape (longer digit runs per block, fewer waves per SIMD).
hipError_t radix_sort_pairs(uint32_t* keys[2], uint32_t* vals[2], uint32_t n, const uint32_t* d_count,
                            int begin_bit, int end_bit, uint32_t* scratch, int* final_buf, hipStream_t s,
                            const uint32_t* d_range = nullptr, bool keep_keys = true,
                            uint32_t* final_word = nullptr, bool large_blocks = false);
// The same for 16-bit keys (begin_bit < end_bit <= 16).
hipError_t radix_sort_pairs16(uint16_t* keys[2], uint32_t* vals[2], uint32_t n, const uint32_t* d_count,
                              int begin_bit, int end_bit, uint32_t* scratch, int* final_buf, hipStream_t s,
                              bool large_blocks = false);

// Per-Gaussian splat record: four float4 (64 bytes, so a gather of any three
// of them touches one cache line):
//   [0] {mu2D.x, mu2D.y, opacity, 2 ln(opacity / alpha_min)}
//   [1] {conic a, b, c, camera z}
//   [2] {r, g, b, flags (colour clamp bits 0-2, bit 3 set)}
//   [3] {tile rectangle (tx0 | ty0 << 16, tx1 | ty1 << 16), instance count, 0}
constexpr int kRecWords = 4;
// Grid (Gaussian blocks, views); outputs at j = v n + i.  Also writes one
// uint4 {visible, instances, min key, max key} per (view, 256-thread block)
// into partials[n_views * ceil(n / 256)].
hipError_t launch_preprocess(const GaussDev& g, const ViewSet& vs, const SetDev& st, int tile,
                             float4* rec, uint32_t* n_tiles, uint32_t* depth_key, uint4* partials,
                             hipStream_t s);
// Slots of the workspace counters (uint32 words).
constexpr int kStatVisible = 0;    // visible Gaussians
constexpr int kStatKeyMin = 1;     // smallest visible depth key
constexpr int kStatKeyMax = 2;     // largest visible depth key
constexpr int kStatDepthBuf = 3;   // ping-pong buffer holding the depth-sorted visible ids
constexpr int kStatInstances = 4;  // instance count I, uint64 at words 4-5
constexpr int kStatSortCount = 6;  // min(I, instance capacity): instances written and sorted
constexpr int kStatOverflow = 7;   // 1 when I exceeds the instance capacity
constexpr int kStatTouched = 8;    // fused backward: Gaussians that received a gradient
constexpr int kStatKeySpan = 10;   // {0, max - min key}: the range of the compacted depth keys (words 10-11)
constexpr int kStatAccumClean = 12;  // {kAccumClean, layout tag} while accum and marks are all zero (words 12-13)
// Z-order: scratch bytes for n Gaussians; perm[k] = index of the Gaussian at
// position k of the Morton order of the means [3][n]; gather of `planes`
// planes of n elements of 2 or 4 bytes: dst[p][k] = src[p][perm[k]].
size_t zorder_scratch_bytes(uint64_t n);
hipError_t launch_zorder(const float* means, uint32_t n, void* scratch, uint32_t* perm, hipStream_t s);
hipError_t launch_permute(const void* src, void* dst, uint32_t n, int planes, int elem_bytes,
                          const uint32_t* perm, hipStream_t s);
// Reduces the preprocess's per-block partials {visible, instances, key min,
// key max} into the counters, including min(I, cap), the span {0, max key -
// min key} of the compacted (offset) depth keys and the overflow flags (bit
// 0: I > cap; bit 1: the span needs more than depth_bits bits, never set for
// depth_bits = 32), and replaces each block's visible count by its exclusive
// prefix (the block's first compacted position).
// partials sits at the start of a scratch of stats_scratch_words(nb) words.
hipError_t launch_stats(uint4* partials, uint32_t nb, uint64_t cap, int depth_bits, uint32_t* counters,
                        hipStream_t s);
size_t stats_scratch_words(uint32_t nb);
// n: Gaussians per view; entries j = v n + i of n_views views; partials as
// left by launch_stats (nb = n_views * ceil(n / 256)).  The compacted keys
// are the depth keys minus *key_min (device: the smallest visible key).
// Also zeroes clear[0 .. clear_words) and clear2[0 .. clear2_words) (the
// duplication's look-back words and the tile ranges).
hipError_t launch_compact_visible(const uint32_t* n_tiles, const uint32_t* depth_key, uint32_t n, uint32_t n_views,
                                  uint4* partials, const uint32_t* key_min, uint32_t* vis_keys, uint32_t* vis_ids,
                                  uint32_t* clear, size_t clear_words, uint32_t* clear2, size_t clear2_words,
                                  hipStream_t s);
// Tile keys are written as uint16 (key_bytes 2: every global tile id and the
// out-of-range id `tiles` fit) or uint32 (key_bytes 4).  Each visible entry's
// first slot is found by the kernel (decoupled look-back over its workgroups
// in dup_scan, dup_scan_words(n) words zeroed beforehand; a workgroup whose
// wait runs out sums the earlier counts itself and adds 1 to *slow;
// no_wait: every workgroup after the first takes that path, for tests).
size_t dup_scan_words(uint64_t n);
// The depth-sorted entries are vis_ids[*which_ids] (vis_ids[0] when
// which_ids is NULL).
hipError_t launch_duplicate(const uint32_t* const vis_ids[2], const uint32_t* which_ids, const uint32_t* d_nvis,
                            uint32_t n, uint32_t* dup_scan, uint32_t* slow, bool no_wait, const float4* rec,
                            const ViewSet& vs, uint32_t n_gauss, int tile, uint32_t cap, void* keys, int key_bytes,
                            uint32_t* vals, hipStream_t s);
// Ranges of the first min(*d_count, n) (or n) sorted keys.
hipError_t launch_tile_ranges(const void* keys, int key_bytes, uint32_t n, const uint32_t* d_count, uint32_t tiles,
                              uint2* ranges, hipStream_t s);
// Tile queues of the persistent blend: one counter per XCD, kQueueStride
// words (128 bytes) apart, in a region of kQueueWords words.
constexpr uint32_t kQueueStride = 32;
constexpr uint32_t kQueueWords = kQueueStride * kNumXcd;
// One wave per global tile of all views (tile size 8, 16 or 32); images,
// t_finals, lasts and dl_dimages hold the views one after another.  queues
// (kQueueWords device words, or NULL): persistent waves take the tiles from
// per-XCD queues instead of one workgroup per tile (the launch zeroes them).
hipError_t launch_blend_forward(const uint2* ranges, const uint32_t* vals, const float4* rec, const ViewSet& vs,
                                const SetDev& st, int tile, float* images, float* t_finals, uint32_t* lasts,
                                uint32_t* queues, hipStream_t s);
// Adds each fragment's nine gradient sums to its entry's accumulator row and
// sets the entry's byte in `marks` when it adds a nonzero value; accum and
// marks start at zero.  reset_word (optional) and *dirty_word are set to 0
// by the launch; queues as in the forward.
hipError_t launch_blend_backward(const uint2* ranges, const uint32_t* vals, const float4* rec, const ViewSet& vs,
                                 const SetDev& st, int tile, const float* images, const uint32_t* lasts,
                                 const float* dl_dimages, float* accum, uint8_t* marks, uint32_t* reset_word,
                                 uint32_t* dirty_word, uint32_t n, uint32_t* queues, hipStream_t s);
hipError_t launch_preprocess_backward(const GaussDev& g, const CamDev& cam, const float4* rec, const float* accum,
                                      const GradDev& gr, hipStream_t s);
// Several views / timesteps: gradients summed over the views (accum is
// [n_views n][9]); dynamic Gaussians also get dL/dvelocity and dL/daccel.
// marks: the blend backward's byte per entry (nonzero: the entry's
// accumulator row received a value); only marked entries are chained, and
// with rezero their marks and rows are cleared (accum and marks are all zero
// after).
hipError_t launch_preprocess_backward_views(const GaussDev& g, const ViewSet& vs, const float4* rec, float* accum,
                                            uint8_t* marks, const GradDev& gr, bool rezero, hipStream_t s);
// Fused backward + Adam, first part: marks the Gaussians with a gradient in
// `touched` (4 bits per byte), lists them (count in *counter, cleared here),
// gives Gaussian list[s] slot s (slot_of) and writes its 59 raw-parameter
// gradients to grads[p][s] (grads: float [59][n]); with rezero the marks and
// rows it reads are cleared (accum and marks are all zero after).
// *counter must be 0 on entry (the blend backward's reset_word).
hipError_t launch_touched_gradients(const GaussDev& g, const CamDev& cam, const float4* rec, float* accum,
                                    uint8_t* marks, uint8_t* touched, uint32_t* counter, uint32_t* list,
                                    uint32_t* slot_of, float* grads, bool rezero, hipStream_t s);
// Second part: Adam on every parameter of the six groups (means, log_scales,
// quats, logits, sh_dc, sh_rest; planes of length n), with the gradient of
// the marked Gaussians from their slots and zero for all others.  With
// state_word (8-byte aligned), the pair {kAccumClean, state_tag} is written
// there (the accumulator state after a chain rule that cleared what it read).
hipError_t launch_adam_sparse(void* const params[6], float* const exp_avg[6], float* const exp_avg_sq[6],
                              const float lr[6], bool sh_bf16, uint64_t n, const uint8_t* touched,
                              const uint32_t* slot_of, const float* grads, int64_t step, double beta1, double beta2,
                              double eps, uint32_t* state_word, uint32_t state_tag, hipStream_t s);
// step >= 1: host step count; step == 0: advance the device step counter in
// dev_state (256 bytes, first an int64 t) and use it.
hipError_t launch_adam(const fgs_adam_group* groups, int n_groups, int64_t step, double beta1, double beta2,
                       double eps, void* dev_state, hipStream_t s);
hipError_t launch_l1_backward(const float* image, const float* target, uint32_t n, float* dl,
                              double* loss, hipStream_t s);

}  // namespace fgs
