// Per-tile front-to-back blending and its backward pass (Sec. 2.1 Eq. (3)-(4);
// App. B.1: alpha cap 0.99, stop once T < 1e-4, front-to-back gradients;
// Sec. 3.2 "Per-Gaussian Backward" / App. B.3 on reducing gradient atomics).
//
// One wave64 per 16x16 tile; lane l owns the four pixels (l % 16, l / 16 + 4r),
// r = 0..3.  The tile's list is read in batches of 64 entries: lane i gathers
// entry i's 48-byte splat record with vector loads (the next batch is in flight
// in registers while the current one is used); the current batch sits in LDS,
// from where every lane reads fragment k at the same address (a broadcast).  The x-terms of the quadratic
// are shared by a lane's four pixels and the conic is pre-scaled so that alpha
// takes one v_exp_f32.  A wave stops as soon as its 256 pixels are done.
//
// Backward: the wave replays the walk up to the tile's last blended fragment.
// Per fragment, each lane sums the nine gradient terms of its four pixels,
// the wave sums them over its 64 lanes on the VALU with a transpose butterfly
// (16 cross-lane steps for 9 values: DPP within rows, gfx950 permlane swaps
// across rows), and nine lanes issue one float atomic each per (Gaussian, tile).
#include "fgs_internal.h"

namespace fgs {

// A tile of TILE x TILE pixels is one wave64: lane l owns column l % TILE
// and rows l / TILE + (64 / TILE) r, for TILE * TILE / 64 values of r
// (1 pixel per lane at 8x8, 4 at 16x16, 16 at 32x32).
template <int TILE>
struct TileShape {
  static_assert(TILE == 8 || TILE == 16 || TILE == 32, "tile size");
  static constexpr int kRows = TILE * TILE / kWave;  // pixels per lane
  static constexpr int kStep = kWave / TILE;         // rows between a lane's pixels
};

// The view of a block's global tile and that view's tile, camera and outputs.
struct TileView {
  uint32_t view, tile;
  uint64_t pix0;  // first pixel of the view in the concatenated images
};
__device__ __forceinline__ TileView tile_view(const ViewSet& vs, uint32_t gt) {
  const uint32_t v = view_of_tile(vs, gt);
  return TileView{v, gt - vs.tile_base[v], vs.pix_base[v]};
}

// A batch of up to 64 consecutive list entries: lane i holds entry base + i.
// The record words are native 4-vectors: with the HIP float4 wrapper the
// prefetched batch was kept in scratch memory (the wrapper's union defeats
// the promotion of the struct to registers).
typedef float rec4 __attribute__((ext_vector_type(4)));
struct Batch {
  uint32_t gid;
  rec4 r0, r1, r2;  // splat record: {mu2D, o, -}, {a, b, c, -}, {r, g, b, flags}
};

__device__ __forceinline__ void load_batch(const uint32_t* __restrict__ vals, const float4* __restrict__ rec,
                                           uint32_t base, uint32_t end, int lane, Batch& b) {
  const uint32_t j = base + (uint32_t)lane;
  if (j < end) {
    b.gid = vals[j];
    const rec4* r = reinterpret_cast<const rec4*>(rec) + kRecWords * (size_t)b.gid;
    b.r0 = r[0];
    b.r1 = r[1];
    b.r2 = r[2];
  }
}

// The batch being blended, staged in LDS so that every lane reads entry k
// with the same address (a broadcast read, no bank conflict) instead of a
// v_readlane per field, and so that only the prefetched batch occupies
// registers.
// q: the conic pre-scaled once per entry when the batch is staged (not once
// per fragment in every lane), so that
// alpha = min(alpha_max, o * 2^(a2 dx^2 + b2 dx dy + c2 dy^2)).
struct BatchLds {
  float4 r0[kWave], r1[kWave], r2[kWave], q[kWave];
  uint32_t gid[kWave];
};
constexpr float kHalfLog2e = 0.72134752044448170368f;  // log2(e) / 2

__device__ __forceinline__ void stage_batch(const Batch& b, BatchLds& L, int lane) {
  L.r0[lane] = make_float4(b.r0.x, b.r0.y, b.r0.z, b.r0.w);
  L.r1[lane] = make_float4(b.r1.x, b.r1.y, b.r1.z, b.r1.w);
  L.r2[lane] = make_float4(b.r2.x, b.r2.y, b.r2.z, b.r2.w);
  L.q[lane] = make_float4(-kHalfLog2e * b.r1.x, -2.0f * kHalfLog2e * b.r1.y, -kHalfLog2e * b.r1.z, 0.0f);
  L.gid[lane] = b.gid;
}

// Splat k of a batch, broadcast to the wave.
struct Splat {
  float mx, my, o, a, b, c, a2, b2, c2;
};

__device__ __forceinline__ Splat splat_of(const BatchLds& L, int k) {
  const float4 r0 = L.r0[k], r1 = L.r1[k], q = L.q[k];
  Splat s;
  s.mx = r0.x;
  s.my = r0.y;
  s.o = r0.z;
  s.a = r1.x;
  s.b = r1.y;
  s.c = r1.z;
  s.a2 = q.x;
  s.b2 = q.y;
  s.c2 = q.z;
  return s;
}

// Alpha of Eq. (3) for one pixel, given the terms of the lane's column:
// ax = a2 dx^2 and bx = b2 dx.  The forward and the backward call exactly
// this sequence, so they take identical skip decisions.
__device__ __forceinline__ float pixel_alpha(const Splat& s, float ax, float bx, float dy, float alpha_max,
                                             float& G) {
  G = __builtin_amdgcn_exp2f(fmaf(fmaf(s.c2, dy, bx), dy, ax));
  // min(alpha_max, o G) for o G >= 0, as a median (one instruction; fminf
  // would re-canonicalise alpha_max at every fragment)
  return __builtin_amdgcn_fmed3f(s.o * G, 0.0f, alpha_max);
}

// Global tile gt of all views, by one wave.  images: the views' [3][H][W]
// blocks one after another; t_finals and lasts likewise with one plane.
template <int TILE>
__device__ __forceinline__ void blend_fwd_tile(uint32_t gt, const uint2* __restrict__ ranges,
                                               const uint32_t* __restrict__ vals, const float4* __restrict__ rec,
                                               const ViewSet& vs, const SetDev& st, float* __restrict__ images,
                                               float* __restrict__ t_finals, uint32_t* __restrict__ lasts) {
  constexpr int kRows = TileShape<TILE>::kRows, kStep = TileShape<TILE>::kStep;
  const TileView tv = tile_view(vs, gt);
  const CamDev& cam = vs.cam[tv.view];
  float* __restrict__ image = images + 3 * tv.pix0;
  float* __restrict__ t_final = t_finals ? t_finals + tv.pix0 : nullptr;
  uint32_t* __restrict__ last = lasts + tv.pix0;
  const uint32_t tile = tv.tile;
  const int tx = (int)(tile % (uint32_t)cam.tiles_x), ty = (int)(tile / (uint32_t)cam.tiles_x);
  const int lane = threadIdx.x;
  const int px = tx * TILE + (lane % TILE);
  const float fx = (float)px + 0.5f;
  float fy[kRows], T[kRows], C0[kRows], C1[kRows], C2[kRows];
  uint32_t lpos[kRows];
  bool live[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int py = ty * TILE + lane / TILE + kStep * r;
    fy[r] = (float)py + 0.5f;
    T[r] = 1.0f; C0[r] = C1[r] = C2[r] = 0.0f;
    lpos[r] = 0;
    live[r] = px < cam.width && py < cam.height;
  }
  const uint2 range = ranges[gt];
  const uint32_t beg = __builtin_amdgcn_readfirstlane(range.x);
  const uint32_t end = __builtin_amdgcn_readfirstlane(range.y);
  __shared__ BatchLds s_batch;
  Batch nxt = {};
  load_batch(vals, rec, beg, end, lane, nxt);
  bool running = beg < end;
  for (uint32_t base = beg; running && base < end; base += kWave) {
    __syncthreads();  // (one wave) the previous batch's reads are done
    stage_batch(nxt, s_batch, lane);
    __syncthreads();
    if (base + kWave < end) load_batch(vals, rec, base + kWave, end, lane, nxt);
    const int cnt = (int)min((uint32_t)kWave, end - base);
    for (int k = 0; k < cnt; ++k) {
      const Splat sp = splat_of(s_batch, k);
      const float dx = fx - sp.mx;
      const float ax = sp.a2 * dx * dx, bx = sp.b2 * dx;
      const float4 r2 = s_batch.r2[k];
      const float cr = r2.x, cg = r2.y, cb = r2.z;
      bool any = false;
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        float G;
        const float alpha = pixel_alpha(sp, ax, bx, fy[r] - sp.my, st.alpha_max, G);
        const bool blend = live[r] && alpha >= st.alpha_min;
        const float a = blend ? alpha : 0.0f;  // branch-free: a skipped fragment has alpha 0
        const float wgt = a * T[r];
        C0[r] = fmaf(wgt, cr, C0[r]);
        C1[r] = fmaf(wgt, cg, C1[r]);
        C2[r] = fmaf(wgt, cb, C2[r]);
        T[r] -= wgt;  // T (1 - alpha)
        lpos[r] = blend ? base - beg + (uint32_t)k + 1u : lpos[r];
        live[r] = live[r] && !(T[r] < st.t_min);
        any |= live[r];
      }
      if (__ballot(any) == 0ull) {
        running = false;
        break;
      }
    }
  }
  const size_t hw = (size_t)cam.width * cam.height;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int py = ty * TILE + lane / TILE + kStep * r;
    if (px < cam.width && py < cam.height) {
      const size_t pix = (size_t)py * cam.width + px;
      image[pix] = fmaf(T[r], cam.bg[0], C0[r]);
      image[hw + pix] = fmaf(T[r], cam.bg[1], C1[r]);
      image[2 * hw + pix] = fmaf(T[r], cam.bg[2], C2[r]);
      if (t_final) t_final[pix] = T[r];
      last[pix] = lpos[r];
    }
  }
}

// Tile queues (persistent waves): XCD x owns the same band of tiles as in
// xcd_tile, and the waves running on it take the band's tiles in order from
// counter x (one 128-byte line each, zero before the launch), so a wave that
// finishes a short tile takes the next one instead of the hardware
// dispatcher starting a new workgroup.  Every wave stops at the first
// number past its band: no wave waits on another.
__device__ __forceinline__ void xcd_band(uint32_t xcd, uint32_t nb, uint32_t& start, uint32_t& count) {
  const uint32_t base = nb / kNumXcd, rem = nb % kNumXcd;
  start = xcd * base + (xcd < rem ? xcd : rem);
  count = base + (xcd < rem ? 1u : 0u);
}
__device__ __forceinline__ uint32_t queue_take(uint32_t* q) {
  uint32_t t = 0;
  if (threadIdx.x == 0) t = atomicAdd(q, 1u);
  return (uint32_t)__shfl((int)t, 0, kWave);
}

// Grid: one wave per global tile of all views (XCD-banded order).
template <int TILE>
__global__ __launch_bounds__(kWave) void k_blend_fwd(const uint2* __restrict__ ranges,
                                                     const uint32_t* __restrict__ vals,
                                                     const float4* __restrict__ rec, ViewSet vs, SetDev st,
                                                     float* __restrict__ images, float* __restrict__ t_finals,
                                                     uint32_t* __restrict__ lasts) {
  blend_fwd_tile<TILE>(xcd_tile(blockIdx.x, gridDim.x), ranges, vals, rec, vs, st, images, t_finals, lasts);
}

// Persistent waves over the tile queues (a multiple of 8 workgroups).
template <int TILE>
__global__ __launch_bounds__(kWave) void k_blend_fwd_queue(const uint2* __restrict__ ranges,
                                                           const uint32_t* __restrict__ vals,
                                                           const float4* __restrict__ rec, ViewSet vs, SetDev st,
                                                           float* __restrict__ images, float* __restrict__ t_finals,
                                                           uint32_t* __restrict__ lasts, uint32_t* __restrict__ queues) {
  const uint32_t xcd = blockIdx.x % kNumXcd;
  uint32_t start, count;
  xcd_band(xcd, vs.tile_base[vs.n_views], start, count);
  for (uint32_t t = queue_take(queues + kQueueStride * xcd); t < count; t = queue_take(queues + kQueueStride * xcd))
    blend_fwd_tile<TILE>(start + t, ranges, vals, rec, vs, st, images, t_finals, lasts);
}

// Workgroups of a persistent launch of `kernel` (one wave each): as many as
// the chip holds at once, a multiple of the XCD count, at most `tiles`
// rounded up to it.
template <typename K>
static uint32_t queue_grid(K kernel, uint32_t tiles) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess || cus <= 0 ||
      per_cu <= 0)
    return 0;
  const uint64_t want = std::min<uint64_t>((uint64_t)cus * (uint64_t)per_cu, (uint64_t)tiles + kNumXcd - 1);
  return (uint32_t)std::max<uint64_t>(kNumXcd, want / kNumXcd * kNumXcd);
}

template <int TILE>
static hipError_t blend_forward_t(const uint2* ranges, const uint32_t* vals, const float4* rec, const ViewSet& vs,
                                  const SetDev& st, float* images, float* t_finals, uint32_t* lasts,
                                  uint32_t* queues, uint32_t tiles, hipStream_t s) {
  if (queues == nullptr) {
    k_blend_fwd<TILE><<<tiles, kWave, 0, s>>>(ranges, vals, rec, vs, st, images, t_finals, lasts);
    return hipGetLastError();
  }
  const uint32_t grid = queue_grid(k_blend_fwd_queue<TILE>, tiles);
  if (grid == 0) return hipErrorInvalidConfiguration;
  hipError_t e = launch_fill_u32(queues, 0u, kQueueWords, s);
  if (e != hipSuccess) return e;
  k_blend_fwd_queue<TILE><<<grid, kWave, 0, s>>>(ranges, vals, rec, vs, st, images, t_finals, lasts, queues);
  return hipGetLastError();
}

hipError_t launch_blend_forward(const uint2* ranges, const uint32_t* vals, const float4* rec, const ViewSet& vs,
                                const SetDev& st, int tile, float* images, float* t_finals, uint32_t* lasts,
                                uint32_t* queues, hipStream_t s) {
  const uint32_t tiles = vs.tile_base[vs.n_views];
  if (tiles == 0) return hipSuccess;
  if (tile == 8) return blend_forward_t<8>(ranges, vals, rec, vs, st, images, t_finals, lasts, queues, tiles, s);
  if (tile == 32) return blend_forward_t<32>(ranges, vals, rec, vs, st, images, t_finals, lasts, queues, tiles, s);
  return blend_forward_t<16>(ranges, vals, rec, vs, st, images, t_finals, lasts, queues, tiles, s);
}

// ---------------------------------------------------------------------------
// Cross-lane sums on the VALU (no LDS round trip): DPP quad_perm / row_ror /
// row_shr within 16-lane rows, and the gfx950 permlane swaps across rows
// (called with the same register twice, the two outputs hold a lane's value
// and its partner's, so their sum is the pair sum).
template <int CTRL, bool BOUND_ZERO = false>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, BOUND_ZERO));
}
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kRowRor4 = 0x124;
constexpr int kRowRor8 = 0x128;   // within a 16-lane row: lane l <- l ^ 8
constexpr int kRowShr4 = 0x114;   // lane l <- l - 4 (0 for the first 4 lanes of a row)

__device__ __forceinline__ float pair16(float x) {
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}
__device__ __forceinline__ float pair32(float x) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

// Sum of v[0..7] over the 64 lanes by a transpose butterfly: each exchange
// halves the values a lane carries.  On return, lanes with bit 2 set (l % 8 >= 4)
// hold the total of value 4*b0 + 2*b1 + b3 (b = bits of the lane index).
__device__ __forceinline__ float wave_reduce8(const float* v, int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b3 = lane & 8;
  float r4[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float send = b0 ? v[j] : v[j + 4];
    const float keep = b0 ? v[j + 4] : v[j];
    r4[j] = keep + dpp<kQuadXor1>(send);
  }
  float r2[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float send = b1 ? r4[j] : r4[j + 2];
    const float keep = b1 ? r4[j + 2] : r4[j];
    r2[j] = keep + dpp<kQuadXor2>(send);
  }
  float r1 = (b3 ? r2[1] : r2[0]) + dpp<kRowRor8>(b3 ? r2[0] : r2[1]);
  r1 += dpp<kRowShr4, true>(r1);  // complete in lanes with bit 2 set
  r1 = pair16(r1);
  return pair32(r1);
}

__device__ __forceinline__ float wave_reduce1(float x) {
  x += dpp<kQuadXor1>(x);
  x += dpp<kQuadXor2>(x);
  x += dpp<kRowRor4>(x);
  x += dpp<kRowRor8>(x);
  x = pair16(x);
  return pair32(x);
}

constexpr int kGrad = 9;  // dL/d(mu2D.x, mu2D.y, a, b, c, opacity, r, g, b)

// Global tile gt, by one wave.  accum: [n][9] with n the (view, Gaussian)
// index range of the record.
template <int TILE>
__device__ __forceinline__ void blend_bwd_tile(uint32_t gt, const uint2* __restrict__ ranges,
                                               const uint32_t* __restrict__ vals, const float4* __restrict__ rec,
                                               const ViewSet& vs, const SetDev& st, const float* __restrict__ images,
                                               const uint32_t* __restrict__ lasts,
                                               const float* __restrict__ dl_dimages, float* __restrict__ accum,
                                               uint8_t* __restrict__ marks) {
  constexpr int kRows = TileShape<TILE>::kRows, kStep = TileShape<TILE>::kStep;
  const TileView tv = tile_view(vs, gt);
  const CamDev& cam = vs.cam[tv.view];
  const float* __restrict__ image = images + 3 * tv.pix0;
  const float* __restrict__ dl_dimage = dl_dimages + 3 * tv.pix0;
  const uint32_t* __restrict__ last = lasts + tv.pix0;
  const uint32_t tile = tv.tile;
  const int tx = (int)(tile % (uint32_t)cam.tiles_x), ty = (int)(tile / (uint32_t)cam.tiles_x);
  const int lane = threadIdx.x;
  const int px = tx * TILE + (lane % TILE);
  const float fx = (float)px + 0.5f;
  const size_t hw = (size_t)cam.width * cam.height;
  float fy[kRows], gc0[kRows], gc1[kRows], gc2[kRows];
  // R = g . (C - S_i): the upstream gradient dotted with the part of the final
  // colour C (background included) not yet blended after fragment i
  float T[kRows], R[kRows];
  uint32_t my_last[kRows];
  uint32_t walk = 0;
  // the pixels' inputs are loaded all at once: a pixel outside the image
  // reads the nearest one inside (always a valid address) and is zeroed
  // (loads under a per-lane guard would go out one row at a time)
  float img[kRows][3];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int py = ty * TILE + lane / TILE + kStep * r;
    const size_t pix = (size_t)min(py, cam.height - 1) * cam.width + min(px, cam.width - 1);
    my_last[r] = last[pix];
    gc0[r] = dl_dimage[pix]; gc1[r] = dl_dimage[hw + pix]; gc2[r] = dl_dimage[2 * hw + pix];
    img[r][0] = image[pix]; img[r][1] = image[hw + pix]; img[r][2] = image[2 * hw + pix];
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int py = ty * TILE + lane / TILE + kStep * r;
    fy[r] = (float)py + 0.5f;
    T[r] = 1.0f;
    if (px < cam.width && py < cam.height) {
      R[r] = gc0[r] * img[r][0] + gc1[r] * img[r][1] + gc2[r] * img[r][2];
    } else {
      my_last[r] = 0;
      gc0[r] = gc1[r] = gc2[r] = 0.0f;
      R[r] = 0.0f;
    }
    walk = max(walk, my_last[r]);
  }
  // longest walk of the tile (wave max)
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) walk = max(walk, (uint32_t)__shfl_xor((int)walk, d, kWave));
  const uint32_t beg = __builtin_amdgcn_readfirstlane(ranges[gt].x);
  const uint32_t lim = __builtin_amdgcn_readfirstlane(ranges[gt].y);
  const uint32_t end = min(beg + __builtin_amdgcn_readfirstlane(walk), lim);
  // lanes that publish the wave sums: l % 8 >= 4 of the first row hold value 4*b0 + 2*b1 + b3
  const bool writer = lane < 16 && (lane & 4);
  const int wq = ((lane & 1) << 2) | (lane & 2) | ((lane >> 3) & 1);

  __shared__ BatchLds s_batch;
  Batch nxt = {};
  load_batch(vals, rec, beg, end, lane, nxt);
  for (uint32_t base = beg; base < end; base += kWave) {
    __syncthreads();  // (one wave) the previous batch's reads are done
    stage_batch(nxt, s_batch, lane);
    __syncthreads();
    if (base + kWave < end) load_batch(vals, rec, base + kWave, end, lane, nxt);
    const int cnt = (int)min((uint32_t)kWave, end - base);
    for (int k = 0; k < cnt; ++k) {
      const uint32_t pos = base - beg + (uint32_t)k;
      const Splat sp = splat_of(s_batch, k);
      const float4 r2 = s_batch.r2[k];
      const float cr = r2.x, cg = r2.y, cb = r2.z;
      const float dx = fx - sp.mx;
      const float ax = sp.a2 * dx * dx, bx = sp.b2 * dx;
      // Per lane, over its pixels: dG = dL/dalpha * G for the blended,
      // uncapped ones (dL/do = sum dG; dL/dpower = o dG with power =
      // -(a dx^2 + 2 b dx dy + c dy^2) / 2), its dy and dy^2 moments (dx is the
      // lane's own constant, so the dx moments follow from sO), and the colour
      // weights.
      float sO = 0.f, sQ = 0.f, sYY = 0.f, w0 = 0.f, w1 = 0.f, w2 = 0.f;
      bool any = false;
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        const float dy = fy[r] - sp.my;
        float G;
        const float alpha = pixel_alpha(sp, ax, bx, dy, st.alpha_max, G);
        const bool blend = pos < my_last[r] && alpha >= st.alpha_min;
        // a strip of the tile that no pixel of blends the fragment keeps its
        // state unchanged: skip it (a wave-uniform branch)
        if (__ballot(blend) == 0ull) continue;
        any = true;
        const float a = blend ? alpha : 0.0f;
        const float wgt = a * T[r];
        w0 = fmaf(wgt, gc0[r], w0);
        w1 = fmaf(wgt, gc1[r], w1);
        w2 = fmaf(wgt, gc2[r], w2);
        const float gcol = gc0[r] * cr + gc1[r] * cg + gc2[r] * cb;
        R[r] = fmaf(-wgt, gcol, R[r]);
        // dC/dalpha_i . g = T_i (g . c_i) - g . (C - S_i) / (1 - alpha_i)
        const float dalpha = fmaf(-R[r], __builtin_amdgcn_rcpf(1.0f - alpha), T[r] * gcol);
        T[r] -= wgt;
        // a capped alpha carries no gradient to o or G
        const float dG = (blend && !(sp.o * G > st.alpha_max)) ? dalpha * G : 0.0f;
        sO += dG;
        const float dyG = dG * dy;
        sQ += dyG;
        sYY = fmaf(dyG, dy, sYY);
      }
      if (!any) continue;  // no pixel of the tile blends this fragment
      // the lane's nine terms, the opacity factor of the first five applied
      // after the wave sum
      const float dxO = dx * sO;
      float v[kGrad];
      v[0] = fmaf(sp.a, dxO, sp.b * sQ);  // dL/dmu2D.x / o
      v[1] = fmaf(sp.b, dxO, sp.c * sQ);  // dL/dmu2D.y / o
      v[2] = -0.5f * dx * dxO;            // dL/da / o
      v[3] = -dx * sQ;                    // dL/db / o
      v[4] = -0.5f * sYY;                 // dL/dc / o
      v[5] = sO;                          // dL/do
      v[6] = w0; v[7] = w1; v[8] = w2;
      const float r8 = wave_reduce8(v, lane) * (wq < 5 ? sp.o : 1.0f);
      const float r1 = wave_reduce1(v[8]);
      const uint32_t gid = s_batch.gid[k];
      // one atomic instruction for the nine sums: they are adjacent in the
      // Gaussian's [9] accumulator row
      const float val = writer ? r8 : r1;
      if ((writer || lane == 0) && val != 0.0f) {
        unsafeAtomicAdd(accum + (size_t)gid * kGrad + (writer ? wq : 8), val);
        marks[gid] = 1u;  // the same byte from every lane that adds: no atomic needed
      }
    }
  }
}

// Grid: one wave per global tile (XCD-banded order); the first workgroup
// also zeroes *reset_word when given, and *dirty_word (the accumulator is no
// longer known to be zero).
template <int TILE>
__global__ __launch_bounds__(kWave) void k_blend_bwd(const uint2* __restrict__ ranges,
                                                     const uint32_t* __restrict__ vals,
                                                     const float4* __restrict__ rec, ViewSet vs, SetDev st,
                                                     const float* __restrict__ images,
                                                     const uint32_t* __restrict__ lasts,
                                                     const float* __restrict__ dl_dimages,
                                                     float* __restrict__ accum, uint8_t* __restrict__ marks,
                                                     uint32_t* __restrict__ reset_word,
                                                     uint32_t* __restrict__ dirty_word) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (reset_word != nullptr) *reset_word = 0u;
    *dirty_word = 0u;
  }
  blend_bwd_tile<TILE>(xcd_tile(blockIdx.x, gridDim.x), ranges, vals, rec, vs, st, images, lasts, dl_dimages,
                       accum, marks);
}

// Persistent waves over the tile queues.
template <int TILE>
__global__ __launch_bounds__(kWave) void k_blend_bwd_queue(const uint2* __restrict__ ranges,
                                                           const uint32_t* __restrict__ vals,
                                                           const float4* __restrict__ rec, ViewSet vs, SetDev st,
                                                           const float* __restrict__ images,
                                                           const uint32_t* __restrict__ lasts,
                                                           const float* __restrict__ dl_dimages,
                                                           float* __restrict__ accum, uint8_t* __restrict__ marks,
                                                           uint32_t* __restrict__ reset_word,
                                                           uint32_t* __restrict__ dirty_word,
                                                           uint32_t* __restrict__ queues) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (reset_word != nullptr) *reset_word = 0u;
    *dirty_word = 0u;
  }
  const uint32_t xcd = blockIdx.x % kNumXcd;
  uint32_t start, count;
  xcd_band(xcd, vs.tile_base[vs.n_views], start, count);
  for (uint32_t t = queue_take(queues + kQueueStride * xcd); t < count; t = queue_take(queues + kQueueStride * xcd))
    blend_bwd_tile<TILE>(start + t, ranges, vals, rec, vs, st, images, lasts, dl_dimages, accum, marks);
}

template <int TILE>
static hipError_t blend_backward_t(const uint2* ranges, const uint32_t* vals, const float4* rec, const ViewSet& vs,
                                   const SetDev& st, const float* images, const uint32_t* lasts,
                                   const float* dl_dimages, float* accum, uint8_t* marks, uint32_t* reset_word,
                                   uint32_t* dirty_word, uint32_t* queues, uint32_t tiles, hipStream_t s) {
  if (queues == nullptr) {
    k_blend_bwd<TILE><<<tiles, kWave, 0, s>>>(ranges, vals, rec, vs, st, images, lasts, dl_dimages, accum, marks,
                                              reset_word, dirty_word);
    return hipGetLastError();
  }
  const uint32_t grid = queue_grid(k_blend_bwd_queue<TILE>, tiles);
  if (grid == 0) return hipErrorInvalidConfiguration;
  hipError_t e = launch_fill_u32(queues, 0u, kQueueWords, s);
  if (e != hipSuccess) return e;
  k_blend_bwd_queue<TILE><<<grid, kWave, 0, s>>>(ranges, vals, rec, vs, st, images, lasts, dl_dimages, accum,
                                                 marks, reset_word, dirty_word, queues);
  return hipGetLastError();
}

hipError_t launch_blend_backward(const uint2* ranges, const uint32_t* vals, const float4* rec, const ViewSet& vs,
                                 const SetDev& st, int tile, const float* images, const uint32_t* lasts,
                                 const float* dl_dimages, float* accum, uint8_t* marks, uint32_t* reset_word,
                                 uint32_t* dirty_word, uint32_t n, uint32_t* queues, hipStream_t s) {
  const uint32_t tiles = vs.tile_base[vs.n_views];
  if (tiles == 0 || n == 0) return hipSuccess;
  if (tile == 8)
    return blend_backward_t<8>(ranges, vals, rec, vs, st, images, lasts, dl_dimages, accum, marks, reset_word,
                               dirty_word, queues, tiles, s);
  if (tile == 32)
    return blend_backward_t<32>(ranges, vals, rec, vs, st, images, lasts, dl_dimages, accum, marks, reset_word,
                                dirty_word, queues, tiles, s);
  return blend_backward_t<16>(ranges, vals, rec, vs, st, images, lasts, dl_dimages, accum, marks, reset_word,
                              dirty_word, queues, tiles, s);
}

}  // namespace fgs
