// Per-tile front-to-back blending and its backward pass (Sec. 2.1 Eq. (3)-(4);
// App. B.1: alpha cap 0.99, stop once T < 1e-4, front-to-back gradients;
// Sec. 3.2 "Per-Gaussian Backward" / App. B.3 on reducing gradient atomics).
//
// One workgroup of 256 threads per 16x16 tile, one pixel per thread.  Splat
// records of the tile's list are gathered 256 at a time into LDS and then
// read by every pixel of the tile (LDS broadcast, no bank conflicts).
//
// Backward: every pixel replays its own walk in the same order up to its last
// blended fragment.  Per fragment, the nine per-pixel gradient terms are
// summed over the 64 pixels of a wavefront with a transpose butterfly (16
// cross-lane steps for 9 values instead of 54), the four wavefront partials
// are combined through LDS, and one float atomic per value per (Gaussian,
// tile) goes to the accumulators.
#include "fgs_internal.h"

namespace fgs {

constexpr int kTile = 16;

__global__ __launch_bounds__(kBlock) void k_blend_fwd(const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ vals,
                                                      const float4* __restrict__ rec, CamDev cam, SetDev st,
                                                      float* __restrict__ image, float* __restrict__ t_final,
                                                      uint32_t* __restrict__ last) {
  __shared__ float4 s_geo[kBlock];  // mu2D.x, mu2D.y, opacity
  __shared__ float4 s_con[kBlock];  // conic a, b, c
  __shared__ float4 s_col[kBlock];  // r, g, b
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = (int)(tile % (uint32_t)cam.tiles_x), ty = (int)(tile / (uint32_t)cam.tiles_x);
  const int px = tx * kTile + (int)(threadIdx.x % kTile);
  const int py = ty * kTile + (int)(threadIdx.x / kTile);
  const bool inside = px < cam.width && py < cam.height;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const uint2 range = ranges[tile];

  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t last_pos = 0;
  bool done = !inside;
  for (uint32_t start = range.x; start < range.y; start += kBlock) {
    if (__syncthreads_count(done ? 1 : 0) == kBlock) break;  // also guards LDS reuse
    const uint32_t j = start + threadIdx.x;
    if (j < range.y) {
      const uint32_t gid = vals[j];
      const float4 r0 = rec[3 * (size_t)gid + 0];
      const float4 r1 = rec[3 * (size_t)gid + 1];
      const float4 r2 = rec[3 * (size_t)gid + 2];
      s_geo[threadIdx.x] = r0;
      s_con[threadIdx.x] = r1;
      s_col[threadIdx.x] = r2;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBlock, range.y - start);
    if (!done) {
      for (int k = 0; k < cnt; ++k) {
        const float4 geo = s_geo[k];
        const float4 con = s_con[k];
        float g;
        const float alpha = splat_alpha(fx - geo.x, fy - geo.y, con.x, con.y, con.z, geo.z, st.alpha_max, g);
        if (alpha < st.alpha_min) continue;
        const float4 col = s_col[k];
        const float wgt = alpha * T;
        C0 = fmaf(wgt, col.x, C0);
        C1 = fmaf(wgt, col.y, C1);
        C2 = fmaf(wgt, col.z, C2);
        T = T * (1.0f - alpha);
        last_pos = start - range.x + (uint32_t)k + 1u;
        if (T < st.t_min) {
          done = true;
          break;
        }
      }
    }
  }
  if (inside) {
    const size_t hw = (size_t)cam.width * cam.height;
    const size_t pix = (size_t)py * cam.width + px;
    image[pix] = fmaf(T, cam.bg[0], C0);
    image[hw + pix] = fmaf(T, cam.bg[1], C1);
    image[2 * hw + pix] = fmaf(T, cam.bg[2], C2);
    if (t_final) t_final[pix] = T;
    last[pix] = last_pos;
  }
}

hipError_t launch_blend_forward(const uint2* ranges, const uint32_t* vals, const float4* rec, const CamDev& cam,
                                const SetDev& st, float* image, float* t_final, uint32_t* last, hipStream_t s) {
  const uint32_t tiles = (uint32_t)cam.tiles_x * (uint32_t)cam.tiles_y;
  if (tiles == 0) return hipSuccess;
  k_blend_fwd<<<tiles, kBlock, 0, s>>>(ranges, vals, rec, cam, st, image, t_final, last);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sum of v[0..7] over the 64 lanes: on return, lane l holds the total of value
// 4*b0 + 2*b1 + b2 where b0, b1, b2 are the low bits of l.
__device__ __forceinline__ float wave_reduce8(const float* v, int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
  float r4[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float send = b0 ? v[j] : v[j + 4];
    const float keep = b0 ? v[j + 4] : v[j];
    r4[j] = keep + __shfl_xor(send, 1, kWave);
  }
  float r2[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float send = b1 ? r4[j] : r4[j + 2];
    const float keep = b1 ? r4[j + 2] : r4[j];
    r2[j] = keep + __shfl_xor(send, 2, kWave);
  }
  float r1 = (b2 ? r2[1] : r2[0]) + __shfl_xor(b2 ? r2[0] : r2[1], 4, kWave);
  r1 += __shfl_xor(r1, 8, kWave);
  r1 += __shfl_xor(r1, 16, kWave);
  r1 += __shfl_xor(r1, 32, kWave);
  return r1;
}

__device__ __forceinline__ float wave_reduce1(float v) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

constexpr int kGrad = 9;  // dL/d(mu2D.x, mu2D.y, a, b, c, opacity, r, g, b)

__global__ __launch_bounds__(kBlock) void k_blend_bwd(const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ vals,
                                                      const float4* __restrict__ rec, CamDev cam, SetDev st,
                                                      const float* __restrict__ image,
                                                      const uint32_t* __restrict__ last,
                                                      const float* __restrict__ dl_dimage,
                                                      float* __restrict__ accum, uint32_t n) {
  constexpr int kWaves = kBlock / kWave;
  __shared__ float4 s_geo[kBlock];
  __shared__ float4 s_con[kBlock];
  __shared__ float4 s_col[kBlock];
  __shared__ uint32_t s_id[kBlock];
  __shared__ float s_red[kWaves][kBlock][kGrad];
  __shared__ uint32_t s_max[kWaves];

  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = (int)(tile % (uint32_t)cam.tiles_x), ty = (int)(tile / (uint32_t)cam.tiles_x);
  const int px = tx * kTile + (int)(threadIdx.x % kTile);
  const int py = ty * kTile + (int)(threadIdx.x / kTile);
  const bool inside = px < cam.width && py < cam.height;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint2 range = ranges[tile];

  const size_t hw = (size_t)cam.width * cam.height;
  const size_t pix = inside ? (size_t)py * cam.width + px : 0;
  const uint32_t my_last = inside ? last[pix] : 0u;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, F0 = 0.f, F1 = 0.f, F2 = 0.f;
  if (inside) {
    g0 = dl_dimage[pix]; g1 = dl_dimage[hw + pix]; g2 = dl_dimage[2 * hw + pix];
    F0 = image[pix]; F1 = image[hw + pix]; F2 = image[2 * hw + pix];
  }
  // longest walk in the tile
  uint32_t m = my_last;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, kWave));
  if (lane == 0) s_max[wave] = m;
  __syncthreads();
  uint32_t walk = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) walk = max(walk, s_max[w]);
  const uint32_t end = min(range.x + walk, range.y);

  float T = 1.0f, S0 = 0.f, S1 = 0.f, S2 = 0.f;
  for (uint32_t start = range.x; start < end; start += kBlock) {
    __syncthreads();  // the previous batch's LDS is no longer read
    const uint32_t j = start + threadIdx.x;
    if (j < end) {
      const uint32_t gid = vals[j];
      s_id[threadIdx.x] = gid;
      s_geo[threadIdx.x] = rec[3 * (size_t)gid + 0];
      s_con[threadIdx.x] = rec[3 * (size_t)gid + 1];
      s_col[threadIdx.x] = rec[3 * (size_t)gid + 2];
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBlock, end - start);
    for (int k = 0; k < cnt; ++k) {
      const uint32_t pos = start - range.x + (uint32_t)k;
      const float4 geo = s_geo[k];
      const float4 con = s_con[k];
      const float dx = fx - geo.x, dy = fy - geo.y;
      float G;
      const float alpha = splat_alpha(dx, dy, con.x, con.y, con.z, geo.z, st.alpha_max, G);
      const bool contrib = (pos < my_last) && (alpha >= st.alpha_min);
      float v[kGrad];
#pragma unroll
      for (int q = 0; q < kGrad; ++q) v[q] = 0.0f;
      if (contrib) {
        const float4 col = s_col[k];
        const float wgt = alpha * T;
        v[6] = wgt * g0;
        v[7] = wgt * g1;
        v[8] = wgt * g2;
        S0 = fmaf(wgt, col.x, S0);
        S1 = fmaf(wgt, col.y, S1);
        S2 = fmaf(wgt, col.z, S2);
        const float inv1m = 1.0f / (1.0f - alpha);
        // dC/dalpha_i = T_i c_i - (C - S_i) / (1 - alpha_i), C including T_final * bg
        const float dalpha = g0 * (T * col.x - (F0 - S0) * inv1m) + g1 * (T * col.y - (F1 - S1) * inv1m) +
                             g2 * (T * col.z - (F2 - S2) * inv1m);
        T = T * (1.0f - alpha);
        const bool capped = geo.z * G > st.alpha_max;
        const float dG = capped ? 0.0f : dalpha * geo.z;
        v[5] = capped ? 0.0f : dalpha * G;
        const float dpow = dG * G;  // power = -(a dx^2 + 2 b dx dy + c dy^2) / 2
        v[0] = dpow * (con.x * dx + con.y * dy);
        v[1] = dpow * (con.y * dx + con.z * dy);
        v[2] = -0.5f * dpow * dx * dx;
        v[3] = -dpow * dx * dy;
        v[4] = -0.5f * dpow * dy * dy;
      }
      if (__ballot(contrib) != 0ull) {
        const float r8 = wave_reduce8(v, lane);
        const float r1 = wave_reduce1(v[8]);
        if (lane < 8) s_red[wave][k][((lane & 1) << 2) | (lane & 2) | ((lane >> 2) & 1)] = r8;
        if (lane == 0) s_red[wave][k][8] = r1;
      } else if (lane < kGrad) {
        s_red[wave][k][lane] = 0.0f;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const uint32_t gid = s_id[threadIdx.x];
      float acc[kGrad];
      bool any = false;
#pragma unroll
      for (int q = 0; q < kGrad; ++q) {
        float a = 0.0f;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) a += s_red[w][threadIdx.x][q];
        acc[q] = a;
        any |= (a != 0.0f);
      }
      if (any) {
#pragma unroll
        for (int q = 0; q < kGrad; ++q)
          if (acc[q] != 0.0f) unsafeAtomicAdd(accum + (size_t)q * n + gid, acc[q]);
      }
    }
  }
}

hipError_t launch_blend_backward(const uint2* ranges, const uint32_t* vals, const float4* rec, const CamDev& cam,
                                 const SetDev& st, const float* image, const uint32_t* last, const float* dl_dimage,
                                 float* accum, uint32_t n, hipStream_t s) {
  const uint32_t tiles = (uint32_t)cam.tiles_x * (uint32_t)cam.tiles_y;
  if (tiles == 0 || n == 0) return hipSuccess;
  k_blend_bwd<<<tiles, kBlock, 0, s>>>(ranges, vals, rec, cam, st, image, last, dl_dimage, accum, n);
  return hipGetLastError();
}

}  // namespace fgs
