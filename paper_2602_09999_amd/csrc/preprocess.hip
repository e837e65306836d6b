// Per-Gaussian preprocess, visible compaction, instance duplication and tile
// ranges (Sec. 2.1 Eq. (1)-(2) and activations; Sec. 3.2 "Splat Bounding",
// "Tile-based Culling", "Sorting"; App. B.1 degenerate-Gaussian guard; App. B.2
// compaction of visible indices only -- the per-Gaussian record stays in
// Gaussian order so the backward pass needs no indirection).
//
// One thread per Gaussian; every plane is read with unit stride across the
// wavefront (structure-of-arrays).  The key-deciding arithmetic (projection,
// conic, threshold, rectangle, tile test) is evaluated in FP32 one operation
// at a time in a fixed order with contraction disabled, so the instance keys
// are reproducible bit for bit.
#include "fgs_internal.h"

namespace fgs {

// Degree-3 real SH basis along unit direction (x, y, z) (Sec. 2.1).
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = 0.28209479177387814f;
  Y[1] = -0.4886025119029199f * y;
  Y[2] = 0.4886025119029199f * z;
  Y[3] = -0.4886025119029199f * x;
  Y[4] = 1.0925484305920792f * (x * y);
  Y[5] = -1.0925484305920792f * (y * z);
  Y[6] = 0.31539156525252005f * (2.0f * zz - xx - yy);
  Y[7] = -1.0925484305920792f * (x * z);
  Y[8] = 0.5462742152960396f * (xx - yy);
  Y[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
  Y[10] = 2.890611442640554f * (x * y) * z;
  Y[11] = -0.4570457994644658f * y * (4.0f * zz - xx - yy);
  Y[12] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -0.4570457994644658f * x * (4.0f * zz - xx - yy);
  Y[14] = 1.445305721320277f * z * (xx - yy);
  Y[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
}

// View-dependent colour: sum_k coeff_k Y_k(dir) + 0.5, clipped at 0 per channel.
// Returns the clip flags (bit c set when channel c was clipped).
template <bool SHB>
__device__ __forceinline__ uint32_t sh_colour(const GaussDev& g, uint32_t i, float px, float py, float pz,
                                              const CamDev& cam, float* rgb) {
  float dx = px - cam.campos[0], dy = py - cam.campos[1], dz = pz - cam.campos[2];
  const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  dx *= inv; dy *= inv; dz *= inv;
  float Y[16];
  sh_basis(dx, dy, dz, Y);
  const size_t n = g.n;
  const int K = g.sh_coeffs;  // 1, 4, 9 or 16
  // every coefficient is loaded before the first is used (a loop over the
  // run-time count waits for each one's loads in turn)
  float dc[3], rest[45];
#pragma unroll
  for (int q = 0; q < 3; ++q) dc[q] = sh_load<SHB>(g.sh_dc, (size_t)q * n + i);
  if (K == 16) {  // uniform; degree 3: no per-load guard (a guarded load is waited for inside its guard)
#pragma unroll
    for (int q = 0; q < 45; ++q) rest[q] = sh_load<SHB>(g.sh_rest, (size_t)q * n + i);
  } else {
#pragma unroll
    for (int q = 0; q < 45; ++q) rest[q] = (q < 3 * (K - 1)) ? sh_load<SHB>(g.sh_rest, (size_t)q * n + i) : 0.0f;
  }
  float c0 = Y[0] * dc[0], c1 = Y[0] * dc[1], c2 = Y[0] * dc[2];
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    if (k < K) {  // uniform
      c0 = fmaf(Y[k], rest[3 * (k - 1)], c0);
      c1 = fmaf(Y[k], rest[3 * (k - 1) + 1], c1);
      c2 = fmaf(Y[k], rest[3 * (k - 1) + 2], c2);
    }
  }
  c0 += 0.5f; c1 += 0.5f; c2 += 0.5f;
  uint32_t flags = (c0 < 0.0f ? 1u : 0u) | (c1 < 0.0f ? 2u : 0u) | (c2 < 0.0f ? 4u : 0u);
  rgb[0] = fmaxf(c0, 0.0f);
  rgb[1] = fmaxf(c1, 0.0f);
  rgb[2] = fmaxf(c2, 0.0f);
  return flags;
}

// Grid: (Gaussian blocks, views).  Outputs of (view v, Gaussian i) sit at
// index j = v n + i.
template <bool SHB>
__global__ __launch_bounds__(kBlock) void k_preprocess(GaussDev g, ViewSet vs, SetDev st, int tile,
                                                       float4* __restrict__ rec, uint32_t* __restrict__ n_tiles,
                                                       uint4* __restrict__ partials,
                                                       uint32_t* __restrict__ depth_key, uint32_t chunks) {
#pragma clang fp contract(off)
  __shared__ WalkLds s_walk[kBlock / kWave];
  // Workgroup b takes chunk (b mod 8) + 8 (b div 8 n_views) of the Gaussians
  // in view (b div 8) mod n_views: workgroups are dealt to the eight XCDs in
  // turn, so the views of one chunk run on one XCD one after another and
  // read its parameters from that XCD's L2 (one view: chunk b).
  const uint32_t b = blockIdx.x, nv = vs.n_views;
  const uint32_t view = (b / kNumXcd) % nv;
  const uint32_t chunk = b % kNumXcd + kNumXcd * (b / (kNumXcd * nv));
  if (chunk >= chunks) return;  // the last group's missing chunks (uniform)
  const CamDev& cam = vs.cam[view];
  const uint32_t i0 = chunk * kBlock + threadIdx.x;
  const bool in_range = i0 < g.n;
  const uint32_t i = in_range ? i0 : g.n - 1;  // lanes past the end mirror the last Gaussian, then drop it
  const size_t n = g.n;
  const size_t j = (size_t)view * n + i;
  const float* W = cam.w;

  // every parameter load goes out before the first store (the depth key),
  // which they could otherwise not pass
  float mu0 = g.means[i], mu1 = g.means[n + i], mu2 = g.means[2 * n + i];
  const float qw0 = g.quats[i], qx0 = g.quats[n + i], qy0 = g.quats[2 * n + i], qz0 = g.quats[3 * n + i];
  const float ls0 = g.log_scales[i], ls1 = g.log_scales[n + i], ls2 = g.log_scales[2 * n + i];
  const float logit = g.logits[i];
  if (g.velocity) {  // dynamic scene: mean at the view's time, (mu + v t) + a t^2
    const float t = vs.time[view], tt = t * t;
    mu0 = (mu0 + g.velocity[i] * t) + g.accel[i] * tt;
    mu1 = (mu1 + g.velocity[n + i] * t) + g.accel[n + i] * tt;
    mu2 = (mu2 + g.velocity[2 * n + i] * t) + g.accel[2 * n + i] * tt;
  }
  // conditional 4D Gaussians (uniform): the mean, covariance and opacity
  // factor of the conditional 3D Gaussian at the view's time
  const bool cond4 = g.quats_r != nullptr;
  Cond4 c4;
  if (cond4) {
    const float ql[4] = {qw0, qx0, qy0, qz0};
    const float qr[4] = {g.quats_r[i], g.quats_r[n + i], g.quats_r[2 * n + i], g.quats_r[3 * n + i]};
    const float ls4[4] = {ls0, ls1, ls2, g.log_scale_t[i]};
    c4 = condition4d(ql, qr, ls4, g.mean_t[i], vs.time[view], mu0, mu1, mu2);
    mu0 = c4.mu[0];
    mu1 = c4.mu[1];
    mu2 = c4.mu[2];
  }
  const float X = ((W[0] * mu0 + W[1] * mu1) + W[2] * mu2) + W[3];
  const float Yc = ((W[4] * mu0 + W[5] * mu1) + W[6] * mu2) + W[7];
  const float Z = ((W[8] * mu0 + W[9] * mu1) + W[10] * mu2) + W[11];
  if (in_range) depth_key[j] = __float_as_uint(Z);

  // activations: normalised quaternion, exp scales, sigmoid opacity
  float qn, S00, S01, S02, S11, S12, S22;
  if (cond4) {
    qn = c4.qn;
    S00 = c4.S[0]; S01 = c4.S[1]; S02 = c4.S[2]; S11 = c4.S[3]; S12 = c4.S[4]; S22 = c4.S[5];
  } else {
    const float n2 = ((qw0 * qw0 + qx0 * qx0) + qy0 * qy0) + qz0 * qz0;
    qn = sqrtf(n2);
    const float w = qw0 / qn, x = qx0 / qn, y = qy0 / qn, z = qz0 / qn;
    const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    const float wx = w * x, wy = w * y, wz = w * z;
    const float r00 = 1.0f - 2.0f * (yy + zz), r01 = 2.0f * (xy - wz), r02 = 2.0f * (xz + wy);
    const float r10 = 2.0f * (xy + wz), r11 = 1.0f - 2.0f * (xx + zz), r12 = 2.0f * (yz - wx);
    const float r20 = 2.0f * (xz - wy), r21 = 2.0f * (yz + wx), r22 = 1.0f - 2.0f * (xx + yy);
    const float s0 = expf(ls0), s1 = expf(ls1), s2 = expf(ls2);
    const float m00 = r00 * s0, m01 = r01 * s1, m02 = r02 * s2;
    const float m10 = r10 * s0, m11 = r11 * s1, m12 = r12 * s2;
    const float m20 = r20 * s0, m21 = r21 * s1, m22 = r22 * s2;
    // Sigma = M M^T
    S00 = (m00 * m00 + m01 * m01) + m02 * m02;
    S01 = (m00 * m10 + m01 * m11) + m02 * m12;
    S02 = (m00 * m20 + m01 * m21) + m02 * m22;
    S11 = (m10 * m10 + m11 * m11) + m12 * m12;
    S12 = (m10 * m20 + m11 * m21) + m12 * m22;
    S22 = (m20 * m20 + m21 * m21) + m22 * m22;
  }

  // Eq. (1): mean projection with the intrinsics
  const float iz = 1.0f / Z;
  const float u = X * iz, v = Yc * iz;
  const float mx = cam.fx * u + cam.cx;
  const float my = cam.fy * v + cam.cy;
  // Eq. (2): T = J W3, Sigma2D = T Sigma T^T
  const float j00 = cam.fx * iz, j11 = cam.fy * iz;
  const float j02 = -(j00 * u), j12 = -(j11 * v);
  const float T00 = j00 * W[0] + j02 * W[8], T01 = j00 * W[1] + j02 * W[9], T02 = j00 * W[2] + j02 * W[10];
  const float T10 = j11 * W[4] + j12 * W[8], T11 = j11 * W[5] + j12 * W[9], T12 = j11 * W[6] + j12 * W[10];
  const float U00 = (T00 * S00 + T01 * S01) + T02 * S02;
  const float U01 = (T00 * S01 + T01 * S11) + T02 * S12;
  const float U02 = (T00 * S02 + T01 * S12) + T02 * S22;
  const float U10 = (T10 * S00 + T11 * S01) + T12 * S02;
  const float U11 = (T10 * S01 + T11 * S11) + T12 * S12;
  const float U12 = (T10 * S02 + T11 * S12) + T12 * S22;
  const float c00 = (U00 * T00 + U01 * T01) + U02 * T02;
  const float c01 = (U00 * T10 + U01 * T11) + U02 * T12;
  const float c11 = (U10 * T10 + U11 * T11) + U12 * T12;
  // dilation (2D low-pass filter) and conic; the precision form takes the
  // near-degenerate determinant and inverse in float64 (exact products, one
  // rounding per subtraction and per division, conic rounded to float32)
  const float h00 = c00 + st.dilation, h11 = c11 + st.dilation, h01 = c01;
  float ca, cb, cc;
  bool det_ok;
  if (st.fp64_conic) {
    const double det = (double)c00 * (double)c11 - (double)c01 * (double)c01;
    const double deth = (double)h00 * (double)h11 - (double)h01 * (double)h01;
    ca = (float)((double)h11 / deth);
    cb = (float)(-(double)h01 / deth);
    cc = (float)((double)h00 / deth);
    det_ok = det >= (double)st.det_min;
  } else {
    const float det = c00 * c11 - c01 * c01;
    const float deth = h00 * h11 - h01 * h01;
    ca = h11 / deth;
    cb = -h01 / deth;
    cc = h00 / deth;
    det_ok = det >= st.det_min;
  }
  float o = 1.0f / (1.0f + expf(-logit));
  if (cond4) o = o * c4.p;  // the marginal factor of the time

  bool ok = (qn >= st.quat_min) && (Z >= cam.near_z) && det_ok && (o > st.alpha_min);
  // opacity-aware extent: alpha reaches alpha_min out to d^T Sigma^-1 d = 2 ln(o / alpha_min)
  const float thr = 2.0f * logf(o / st.alpha_min);
  const float ext_x = sqrtf(thr * h00), ext_y = sqrtf(thr * h11);
  ok = ok && (ext_x >= 0.0f) && (ext_y >= 0.0f) && isfinite(mx) && isfinite(my) && isfinite(ca) &&
       isfinite(cb) && isfinite(cc);

  // rectangle in pixel-centre indices, then tiles
  const float lx = (mx - ext_x) - 0.5f, hx = (mx + ext_x) - 0.5f;
  const float ly = (my - ext_y) - 0.5f, hy = (my + ext_y) - 0.5f;
  const float wm1 = (float)(cam.width - 1), hm1 = (float)(cam.height - 1);
  bool nonempty = in_range && ok && (hx >= 0.0f) && (lx <= wm1) && (hy >= 0.0f) && (ly <= hm1);
  CandLane me = {mx, my, ca, cb, cc, thr, 0, 0, 1, 0u, cam.width, cam.height};
  uint32_t rect_lo = 0, rect_hi = 0;
  if (nonempty) {
    const int i0x = (lx <= 0.0f) ? 0 : (int)ceilf(lx);
    const int i1x = (hx >= wm1) ? cam.width - 1 : (int)floorf(hx);
    const int k0 = (ly <= 0.0f) ? 0 : (int)ceilf(ly);
    const int k1 = (hy >= hm1) ? cam.height - 1 : (int)floorf(hy);
    if (i0x <= i1x && k0 <= k1) {
      const int tx0 = i0x / tile, tx1 = i1x / tile, ty0 = k0 / tile, ty1 = k1 / tile;
      me.tx0 = tx0;
      me.ty0 = ty0;
      me.w = tx1 - tx0 + 1;
      me.cand = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
      rect_lo = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
      rect_hi = (uint32_t)tx1 | ((uint32_t)ty1 << 16);
    }
  }
  // exact per-tile test of every candidate tile, load-balanced over the wave
  const uint32_t count = wave_tile_walk<false>(me, s_walk[threadIdx.x / kWave], tile,
                                               [](int, const OwnerRec&, uint32_t, int, int, bool) {});
  const bool vis = in_range && count > 0;
  if (in_range) n_tiles[j] = count;
  if (vis) {
    float rgb[3];
    const uint32_t clip = sh_colour<SHB>(g, i, mu0, mu1, mu2, cam, rgb);
    rec[kRecWords * j + 0] = make_float4(mx, my, o, thr);
    rec[kRecWords * j + 1] = make_float4(ca, cb, cc, Z);
    rec[kRecWords * j + 2] = make_float4(rgb[0], rgb[1], rgb[2], __uint_as_float(clip | 8u));
    rec[kRecWords * j + 3] = make_float4(__uint_as_float(rect_lo), __uint_as_float(rect_hi),
                                         __uint_as_float(count), 0.0f);
  }
  // this block's share of the statistics the host reads after the preprocess
  // (visible count, instance count, smallest and largest visible depth key),
  // reduced last so that no wave waits on another before its own work is done
  uint32_t b_vis = vis ? 1u : 0u, b_sum = vis ? count : 0u;
  uint32_t b_min = vis ? __float_as_uint(Z) : 0xffffffffu, b_max = vis ? __float_as_uint(Z) : 0u;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    b_vis += __shfl_xor(b_vis, d, kWave);
    b_sum += __shfl_xor(b_sum, d, kWave);
    b_min = min(b_min, (uint32_t)__shfl_xor((int)b_min, d, kWave));
    b_max = max(b_max, (uint32_t)__shfl_xor((int)b_max, d, kWave));
  }
  __shared__ uint4 s_part[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) s_part[wave] = make_uint4(b_vis, b_sum, b_min, b_max);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint4 t = s_part[0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) {
      const uint4 u = s_part[w];
      t = make_uint4(t.x + u.x, t.y + u.y, min(t.z, u.z), max(t.w, u.w));
    }
    partials[(size_t)view * chunks + chunk] = t;
  }
}

hipError_t launch_preprocess(const GaussDev& g, const ViewSet& vs, const SetDev& st, int tile, float4* rec,
                             uint32_t* n_tiles, uint32_t* depth_key, uint4* partials, hipStream_t s) {
  if (g.n == 0 || vs.n_views == 0) return hipSuccess;
  // chunks of kBlock Gaussians; groups of kNumXcd chunks times the views
  const uint32_t chunks = ceil_div(g.n, kBlock);
  const uint32_t grid = ceil_div(chunks, kNumXcd) * kNumXcd * vs.n_views;
  if (g.sh_bf16)
    k_preprocess<true><<<grid, kBlock, 0, s>>>(g, vs, st, tile, rec, n_tiles, partials, depth_key, chunks);
  else
    k_preprocess<false><<<grid, kBlock, 0, s>>>(g, vs, st, tile, rec, n_tiles, partials, depth_key, chunks);
  return hipGetLastError();
}

// Statistics the host needs to size the rest of the pass -- visible count,
// instance count I (the sum of the per-Gaussian counts, independent of the
// depth order) and the range of the visible depth keys -- from the
// preprocess blocks' partials.  One workgroup; writes every counter word.
// Statistics read after the preprocess (visible count, instance count,
// smallest and largest visible depth key, sort count and overflow flag) and
// each preprocess block's first position in the compacted list, in two
// launches.  k_stats_group: workgroup g takes partials [256 g, 256 g + 256)
// (coalesced), replaces each block's visible count by its exclusive prefix
// within the group and writes the group's totals.  k_stats_final: one
// workgroup over the groups: the counters, and each group's first position.
struct StatsGroup {
  uint32_t vis, kmin, kmax, pad;
  unsigned long long sum;
};

__global__ __launch_bounds__(kBlock) void k_stats_group(uint4* __restrict__ partials, uint32_t nb,
                                                        StatsGroup* __restrict__ groups) {
  __shared__ uint32_t s_lds[kBlock / kWave];
  __shared__ uint32_t s_min[kBlock / kWave], s_max[kBlock / kWave];
  __shared__ unsigned long long s_sum[kBlock / kWave];
  const uint32_t b = blockIdx.x * kBlock + threadIdx.x;
  const uint4 t = b < nb ? partials[b] : make_uint4(0u, 0u, 0xffffffffu, 0u);
  uint32_t total;
  const uint32_t ex = block_exclusive_scan(t.x, s_lds, &total);
  if (b < nb) partials[b].x = ex;
  unsigned long long sum = t.y;
  uint32_t kmin = t.z, kmax = t.w;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    sum += __shfl_xor(sum, d, kWave);
    kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, d, kWave));
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, d, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) {
    s_min[wave] = kmin; s_max[wave] = kmax; s_sum[wave] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) {
      sum += s_sum[w]; kmin = min(kmin, s_min[w]); kmax = max(kmax, s_max[w]);
    }
    groups[blockIdx.x] = StatsGroup{total, kmin, kmax, 0u, sum};
  }
}

__global__ __launch_bounds__(kBlock) void k_stats_final(const StatsGroup* __restrict__ groups, uint32_t ng,
                                                        uint64_t cap, int depth_bits, uint32_t* __restrict__ c,
                                                        uint32_t* __restrict__ group_start) {
  __shared__ uint32_t s_lds[kBlock / kWave];
  __shared__ uint32_t s_min[kBlock / kWave], s_max[kBlock / kWave];
  __shared__ unsigned long long s_sum[kBlock / kWave];
  uint32_t carry = 0, kmin = 0xffffffffu, kmax = 0u;
  unsigned long long sum = 0;
  for (uint32_t g0 = 0; g0 < ng; g0 += kBlock) {
    const uint32_t g = g0 + threadIdx.x;
    const StatsGroup t = g < ng ? groups[g] : StatsGroup{0u, 0xffffffffu, 0u, 0u, 0ull};
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(t.vis, s_lds, &tot);
    if (g < ng) group_start[g] = carry + ex;
    carry += tot;
    sum += t.sum;
    kmin = min(kmin, t.kmin);
    kmax = max(kmax, t.kmax);
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    sum += __shfl_xor(sum, d, kWave);
    kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, d, kWave));
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, d, kWave));
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) {
    s_min[wave] = kmin; s_max[wave] = kmax; s_sum[wave] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) {
      sum += s_sum[w]; kmin = min(kmin, s_min[w]); kmax = max(kmax, s_max[w]);
    }
    c[kStatVisible] = carry;
    c[kStatKeyMin] = kmin;
    c[kStatKeyMax] = kmax;
    c[kStatDepthBuf] = 0u;
    reinterpret_cast<unsigned long long*>(c + kStatInstances)[0] = sum;
    c[kStatSortCount] = (uint32_t)(sum < cap ? sum : cap);
    // the compacted keys are offset by the smallest: they span [0, kmax - kmin]
    const uint32_t span = carry > 0 ? kmax - kmin : 0u;
    c[kStatKeySpan] = 0u;
    c[kStatKeySpan + 1] = span;
    const bool depth_over = depth_bits < 32 && (span >> depth_bits) != 0u;
    c[kStatOverflow] = (sum > cap ? 1u : 0u) | (depth_over ? 2u : 0u);
  }
}

size_t stats_scratch_words(uint32_t nb) {
  const size_t ng = (nb + kBlock - 1) / kBlock;
  return 4 * (size_t)nb + round_up64(sizeof(StatsGroup) / 4 * ng) + round_up64(ng);
}

// The group records and group starts follow the nb partials in the same scratch.
static StatsGroup* stats_groups(uint4* partials, uint32_t nb) {
  return reinterpret_cast<StatsGroup*>(reinterpret_cast<uint32_t*>(partials) + 4 * (size_t)nb);
}
static uint32_t* stats_group_start(uint4* partials, uint32_t nb) {
  const size_t ng = (nb + kBlock - 1) / kBlock;
  return reinterpret_cast<uint32_t*>(partials) + 4 * (size_t)nb + round_up64(sizeof(StatsGroup) / 4 * ng);
}

hipError_t launch_stats(uint4* partials, uint32_t nb, uint64_t cap, int depth_bits, uint32_t* counters,
                        hipStream_t s) {
  const uint32_t ng = ceil_div(nb, kBlock);
  k_stats_group<<<ng, kBlock, 0, s>>>(partials, nb, stats_groups(partials, nb));
  k_stats_final<<<1, kBlock, 0, s>>>(stats_groups(partials, nb), ng, cap, depth_bits, counters,
                                     stats_group_start(partials, nb));
  return hipGetLastError();
}

// Writes (depth key - smallest visible key, entry index) of every entry with
// at least one instance, in index order (which the stable depth sort turns
// into the (depth, index) tie-break).  The keys are the bits of positive
// floats, which order like the floats, so subtracting the smallest keeps the
// order and the ties, and leaves keys in [0, max - min]: depths crossing a
// power of two differ in exponent bits up to bit 30, but rarely in more than
// 24 bits of offset, which the sort then takes in three passes instead of
// four.  Same grid as the preprocess: block (b, v), preprocess block q = v *
// gridDim.x + b, takes entries v n + [256 b, 256 b + 256), starts at its
// group's start plus its prefix within the group, and ranks its visible
// entries with ballots.
__global__ __launch_bounds__(kBlock) void k_compact(const uint32_t* __restrict__ n_tiles,
                                                    const uint32_t* __restrict__ depth_key, uint32_t n,
                                                    const uint4* __restrict__ partials,
                                                    const uint32_t* __restrict__ group_start,
                                                    const uint32_t* __restrict__ key_min,
                                                    uint32_t* __restrict__ vis_keys,
                                                    uint32_t* __restrict__ vis_ids,
                                                    uint32_t* __restrict__ clear, size_t clear_words,
                                                    uint32_t* __restrict__ clear2, size_t clear2_words) {
  __shared__ uint32_t s_w[kBlock / kWave];
  {  // also clears the duplication's look-back words (and flag) and the tile ranges for this forward
    const size_t nthreads = (size_t)gridDim.x * gridDim.y * kBlock;
    const size_t t0 = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kBlock + threadIdx.x;
    for (size_t w = t0; w < clear_words; w += nthreads) clear[w] = 0u;
    for (size_t w = t0; w < clear2_words; w += nthreads) clear2[w] = 0u;
  }
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  const size_t j = (size_t)blockIdx.y * n + i;
  const bool vis = i < n && n_tiles[j] != 0u;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint64_t m = __ballot(vis);
  const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  if (lane == 0) s_w[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t pre = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) pre += (w < wave) ? s_w[w] : 0u;
  if (vis) {
    const size_t q = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    const uint32_t p = group_start[q / kBlock] + partials[q].x + pre + below;
    vis_keys[p] = depth_key[j] - *key_min;
    vis_ids[p] = (uint32_t)j;
  }
}

hipError_t launch_compact_visible(const uint32_t* n_tiles, const uint32_t* depth_key, uint32_t n, uint32_t n_views,
                                  uint4* partials, const uint32_t* key_min, uint32_t* vis_keys, uint32_t* vis_ids,
                                  uint32_t* clear, size_t clear_words, uint32_t* clear2, size_t clear2_words,
                                  hipStream_t s) {
  if (n == 0 || n_views == 0) return hipSuccess;
  const dim3 grid(ceil_div(n, kBlock), n_views);
  const uint32_t nb = grid.x * n_views;
  k_compact<<<grid, kBlock, 0, s>>>(n_tiles, depth_key, n, partials, stats_group_start(partials, nb), key_min,
                                    vis_keys, vis_ids, clear, clear_words, clear2, clear2_words);
  return hipGetLastError();
}

// Duplication with its own offsets.  Each visible Gaussian, in depth order,
// writes its kept tiles starting at the sum of the counts of the Gaussians
// before it; the counts come from the records the kernel reads anyway (no
// separate scan gathering them in depth order).  Workgroup b sums its 256
// counts, publishes the sum, then adds the sums of workgroups 0..b-1 by
// decoupled look-back and publishes its inclusive prefix.  A workgroup only
// waits for workgroups with smaller indices, which the dispatcher starts
// first and which never wait for it.  The results do not rest on that order:
// every wait is bounded, and a wait that runs out sums the counts of all
// earlier entries directly (slow, exact) and counts itself in `slow`.
//
// A wave handles 64 consecutive Gaussians and spreads their candidate tiles
// over its lanes (load-balanced walk), so the wave's kept tiles are written as
// one contiguous, coalesced run.  Writes stay inside the wave's run of slots
// and below `cap`.  Entries are (view, Gaussian) indices j = v n_gauss + i; the key of
// an instance is its global tile id tile_base[v] + ty tiles_x(v) + tx.
//
// dup_scan: word 0 the slow-path count, then at word 64 one 64-bit status per
// workgroup: 0 (not published), kDupAggregate | sum, kDupInclusive | prefix;
// cleared by the compaction.
constexpr uint64_t kDupAggregate = 1ull << 32, kDupInclusive = 2ull << 32;
constexpr uint32_t kDupSpinLimit = 1u << 14;
constexpr uint32_t kDupStatusWord = 64;

size_t dup_scan_words(uint64_t n) { return kDupStatusWord + 2 * ((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ uint64_t dup_status_load(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dup_status_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The count of entry q: the last word of its record's fourth float4.
__device__ __forceinline__ uint32_t dup_count(const uint32_t* __restrict__ vis_ids, const float4* __restrict__ rec,
                                              uint32_t q) {
  return __float_as_uint(rec[kRecWords * (size_t)vis_ids[q] + 3].z);
}

// Wave 0 of workgroup blk > 0: the sum of the counts of workgroups 0..blk-1.
// Lane l looks at workgroup top - l of a 64-wide window (indices below 0 read
// as an inclusive prefix of 0); once every workgroup nearer than the window's
// nearest inclusive prefix has published its sum, the sums down to that
// prefix are added and the look-back ends, or moves on to the next window if
// the window holds no inclusive prefix.  (Windows of several statuses per
// lane cost registers, and so occupancy in the walk that follows, for no
// gain.)  After spin_limit polls of a window (kDupSpinLimit; 0 to test the
// fallback) the wave adds up the counts of entries 0..blk*256-1 itself.
__device__ __forceinline__ uint64_t dup_lookback(uint64_t* status, uint32_t blk, const uint32_t* __restrict__ vis_ids,
                                                 const float4* __restrict__ rec, uint32_t* slow, uint32_t spin_limit) {
  const int lane = threadIdx.x & (kWave - 1);
  uint64_t acc = 0;
  for (int64_t top = (int64_t)blk - 1;; top -= kWave) {
    const int64_t j = top - lane;
    uint64_t st = 0, incl = 0, needed = 0;
    bool ready = false;
    for (uint32_t spin = 0; spin < spin_limit && !ready; ++spin) {
      st = j >= 0 ? dup_status_load(status + j) : kDupInclusive;
      const uint32_t flag = (uint32_t)(st >> 32);
      incl = __ballot(flag == 2u);
      const int last = incl ? __ffsll((long long)incl) - 1 : kWave - 1;  // lanes 0..last are needed
      needed = last >= kWave - 1 ? ~0ull : ((2ull << last) - 1ull);
      ready = (__ballot(flag == 0u) & needed) == 0ull;
      if (!ready) __builtin_amdgcn_s_sleep(1);
    }
    if (!ready) {
      uint64_t v = 0;
      for (uint32_t q = (uint32_t)lane; q < blk * kBlock; q += kWave) v += dup_count(vis_ids, rec, q);
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
      if (lane == 0) atomicAdd(slow, 1u);
      return v;
    }
    uint64_t v = (needed >> lane) & 1ull ? (uint64_t)(uint32_t)st : 0ull;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
    acc += v;
    if (incl) return acc;
  }
}

template <typename KT>
__global__ __launch_bounds__(kBlock) void k_duplicate(const uint32_t* __restrict__ vis_ids0,
                                                      const uint32_t* __restrict__ vis_ids1,
                                                      const uint32_t* __restrict__ which_ids,
                                                      const uint32_t* __restrict__ d_nvis, uint32_t n,
                                                      uint32_t* __restrict__ dup_scan, uint32_t* __restrict__ slow,
                                                      uint32_t spin_limit,
                                                      const float4* __restrict__ rec, ViewSet vs,
                                                      uint32_t n_gauss, int tile, uint32_t cap,
                                                      KT* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ WalkLds s_walk[kBlock / kWave];
  __shared__ uint2 s_dup[kBlock / kWave][kWave];
  __shared__ uint32_t s_scan[kBlock / kWave];
  __shared__ uint32_t s_base;
  const uint32_t blk = blockIdx.x;
  const uint32_t nv = min(*d_nvis, n);
  if (blk * kBlock >= nv) return;  // uniform; no later workgroup has entries either
  // the depth sort leaves its result in either buffer (noted on the device)
  const uint32_t* __restrict__ vis_ids = (which_ids != nullptr && *which_ids != 0u) ? vis_ids1 : vis_ids0;
  uint64_t* status = reinterpret_cast<uint64_t*>(dup_scan + kDupStatusWord);
  const uint32_t p = blk * kBlock + threadIdx.x;
  CandLane me = {};
  uint32_t gid = 0, count = 0, kbase = 0, tiles_x = 0;
  if (p < nv) {
    gid = vis_ids[p];
    const uint32_t v = vs.n_views > 1 ? gid / n_gauss : 0u;
    kbase = vs.tile_base[v];
    tiles_x = (uint32_t)vs.cam[v].tiles_x;
    me.width = vs.cam[v].width;
    me.height = vs.cam[v].height;
    // three float4 of one 64-byte record: one cache line per Gaussian
    const float4 r0 = rec[kRecWords * (size_t)gid + 0];
    const float4 r1 = rec[kRecWords * (size_t)gid + 1];
    const float4 r3 = rec[kRecWords * (size_t)gid + 3];
    count = __float_as_uint(r3.z);  // the same word dup_count reads
    int tx0, ty0, tx1, ty1;
    unpack_rect(make_uint2(__float_as_uint(r3.x), __float_as_uint(r3.y)), tx0, ty0, tx1, ty1);
    me = CandLane{r0.x, r0.y, r1.x, r1.y, r1.z, r0.w, tx0, ty0, tx1 - tx0 + 1,
                  count ? (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1)) : 0u, me.width, me.height};
  }
  // this workgroup's offsets: its own exclusive prefix plus the look-back sum
  uint32_t btotal;
  const uint32_t excl = block_exclusive_scan(count, s_scan, &btotal);
  if (threadIdx.x == 0) dup_status_store(status + blk, (blk == 0 ? kDupInclusive : kDupAggregate) | btotal);
  if (threadIdx.x < kWave) {
    const uint64_t prefix = blk > 0 ? dup_lookback(status, blk, vis_ids, rec, slow, spin_limit) : 0ull;
    if (threadIdx.x == 0) {
      if (blk > 0) dup_status_store(status + blk, kDupInclusive | (uint32_t)(prefix + btotal));
      s_base = (uint32_t)prefix;
    }
  }
  __syncthreads();
  if ((blk * kBlock + (threadIdx.x & ~(kWave - 1u))) >= nv) return;  // whole wave past the end
  const uint32_t off = s_base + excl;
  const uint32_t tiles = vs.tile_base[vs.n_views];
  // The wave's Gaussians own one contiguous run of slots (their offsets are
  // consecutive) and the walk visits their candidates in the same order, so a
  // kept tile's slot is the run's start plus its rank among the wave's kept
  // tiles.  Lanes past nv have count 0, so lane 63's off + count ends the run.
  const uint32_t run_start = __shfl(off, 0, kWave);
  const uint32_t run_end = __shfl(off + count, kWave - 1, kWave);
  const uint32_t lim = min(run_end, cap);
  // the owner's Gaussian and key base, read by owner in emit; with 16-bit
  // keys the base and the view's tiles_x both fit in 16 bits and share a word
  const int tile_shift = __builtin_ctz((unsigned)tile);
  s_dup[threadIdx.x / kWave][threadIdx.x & (kWave - 1)] =
      make_uint2(gid, sizeof(KT) == 2 ? (kbase | (tiles_x << 16)) : kbase);
  const uint32_t written = wave_tile_walk<true>(
      me, s_walk[threadIdx.x / kWave], tile,
      [&](int owner, const OwnerRec& o, uint32_t rank, int tx, int ty, bool keep) {
        const uint32_t slot = run_start + rank;
        if (keep && slot < lim) {
          const uint2 d = s_dup[threadIdx.x / kWave][owner];
          // tile coordinates and tiles_x stay below 2^16, so __umul24 is exact
          uint32_t key;
          if (sizeof(KT) == 2) {
            key = (d.y & 0xffffu) + __umul24((uint32_t)ty, d.y >> 16) + (uint32_t)tx;
          } else {  // tiles_x of the owner's view (xmax = width - 0.5)
            const uint32_t row = ((uint32_t)(o.xmax + 0.5f) + (uint32_t)tile - 1u) >> tile_shift;
            key = d.y + __umul24((uint32_t)ty, row) + (uint32_t)tx;
          }
          keys[slot] = (KT)key;
          vals[slot] = d.x;
        }
      });
  // The walk repeats the preprocess count on the same stored values, so the
  // totals agree and this never runs; should they ever disagree, the wave's
  // whole run is filled with an out-of-range tile id (ignored by the range
  // kernel) so that no slot is left undefined.
  if (written != run_end - run_start) {  // wave-uniform
    const uint32_t g0 = __shfl(gid, 0, kWave);
    for (uint32_t slot = run_start + (threadIdx.x & (kWave - 1)); slot < lim; slot += kWave) {
      keys[slot] = (KT)tiles;
      vals[slot] = g0;
    }
  }
}

hipError_t launch_duplicate(const uint32_t* const vis_ids[2], const uint32_t* which_ids, const uint32_t* d_nvis,
                            uint32_t n, uint32_t* dup_scan, uint32_t* slow, bool no_wait, const float4* rec,
                            const ViewSet& vs, uint32_t n_gauss, int tile, uint32_t cap, void* keys, int key_bytes,
                            uint32_t* vals, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t spin_limit = no_wait ? 0u : kDupSpinLimit;
  const uint32_t grid = ceil_div(n, kBlock);
  if (key_bytes == 2)
    k_duplicate<uint16_t><<<grid, kBlock, 0, s>>>(vis_ids[0], vis_ids[1], which_ids, d_nvis, n, dup_scan, slow,
                                                  spin_limit, rec, vs, n_gauss, tile, cap,
                                                  static_cast<uint16_t*>(keys), vals);
  else
    k_duplicate<uint32_t><<<grid, kBlock, 0, s>>>(vis_ids[0], vis_ids[1], which_ids, d_nvis, n, dup_scan, slow,
                                                  spin_limit, rec, vs, n_gauss, tile, cap,
                                                  static_cast<uint32_t*>(keys), vals);
  return hipGetLastError();
}

// Start and end of each tile's run in the sorted keys; a run boundary is where
// a key differs from its neighbour.  Each thread takes V consecutive keys (64
// bytes, four 16-byte loads; the key buffer is 256-byte aligned); the keys
// just before and after its V come from the neighbouring lanes by shuffle,
// and only the wave's first and last lane read them from memory.
template <typename KT>
__global__ __launch_bounds__(kBlock) void k_tile_ranges(const KT* __restrict__ keys, uint32_t n,
                                                        const uint32_t* __restrict__ d_count, uint32_t tiles,
                                                        uint2* __restrict__ ranges) {
  constexpr int H = 16 / (int)sizeof(KT);  // keys per 16-byte load
  constexpr int kLoads = 4;
  constexpr int V = kLoads * H;
  constexpr uint32_t kNone = 0xffffffffu;  // differs from every key
  const uint32_t count = d_count ? min(*d_count, n) : n;
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t i0 = (blockIdx.x * kBlock + threadIdx.x) * (uint32_t)V;
  if ((blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1u))) * (uint32_t)V >= count) return;  // whole wave
  uint32_t k[V];
  if (i0 + V <= count) {
    struct alignas(16) Vec { KT k[H]; };
    Vec a[kLoads];
#pragma unroll
    for (int l = 0; l < kLoads; ++l) a[l] = reinterpret_cast<const Vec*>(keys + i0)[l];
#pragma unroll
    for (int l = 0; l < kLoads; ++l)
#pragma unroll
      for (int j = 0; j < H; ++j) k[l * H + j] = a[l].k[j];
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) k[j] = (i0 + j < count) ? (uint32_t)keys[i0 + j] : kNone;
  }
  uint32_t prev = (uint32_t)__shfl((int)k[V - 1], (lane + kWave - 1) & (kWave - 1), kWave);
  uint32_t next = (uint32_t)__shfl((int)k[0], (lane + 1) & (kWave - 1), kWave);
  if (lane == 0) prev = (i0 == 0) ? kNone : (uint32_t)keys[i0 - 1];
  if (lane == kWave - 1) next = (i0 + V < count) ? (uint32_t)keys[i0 + V] : kNone;
  if (i0 >= count) return;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const uint32_t kj = k[j];
    if (kj >= tiles) continue;
    const uint32_t before = j ? k[j - 1] : prev;
    const uint32_t after = j < V - 1 ? k[j + 1] : next;
    if (before != kj) ranges[kj].x = i0 + j;
    if (after != kj) ranges[kj].y = i0 + j + 1;
  }
}

hipError_t launch_tile_ranges(const void* keys, int key_bytes, uint32_t n, const uint32_t* d_count, uint32_t tiles,
                              uint2* ranges, hipStream_t s) {
  if (n == 0) return hipSuccess;
  // 64 bytes of keys per thread
  if (key_bytes == 2)
    k_tile_ranges<uint16_t><<<ceil_div(ceil_div(n, 32), kBlock), kBlock, 0, s>>>(
        static_cast<const uint16_t*>(keys), n, d_count, tiles, ranges);
  else
    k_tile_ranges<uint32_t><<<ceil_div(ceil_div(n, 16), kBlock), kBlock, 0, s>>>(
        static_cast<const uint32_t*>(keys), n, d_count, tiles, ranges);
  return hipGetLastError();
}

}  // namespace fgs
