// Z-order (Morton order) layout of the Gaussians (Sec. 3.3 "Locality-
// preserving Densification"): Gaussians close in 3D are placed close in the
// parameter buffers, so the gathers of the rasterizer (records by tile list,
// the parameters of the Gaussians that receive a gradient) touch fewer cache
// lines.  Applied now and then during training, not every step.
//
// Conventions (the paper names the technique only): bounding cube with side
// the largest per-axis extent of the means, 10 bits per axis quantised in
// FP32 as min(1023, floor((x - lo) * (1024 / side))), bit interleave with x
// in bit 0, stable order (ties keep the index order).
#include "fgs_internal.h"

namespace fgs {

// per-block {min x, min y, min z, max x, max y, max z}
__global__ __launch_bounds__(kBlock) void k_bbox_partial(const float* __restrict__ means, uint32_t n,
                                                         float* __restrict__ part) {
  __shared__ float s_v[kBlock / kWave][6];
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  float v[6];
  if (i < n) {
    for (int a = 0; a < 3; ++a) v[a] = v[3 + a] = means[(size_t)a * n + i];
  } else {
    for (int a = 0; a < 3; ++a) {
      v[a] = __builtin_huge_valf();
      v[3 + a] = -__builtin_huge_valf();
    }
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v[a] = fminf(v[a], __shfl_xor(v[a], d, kWave));
      v[3 + a] = fmaxf(v[3 + a], __shfl_xor(v[3 + a], d, kWave));
    }
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0)
    for (int a = 0; a < 6; ++a) s_v[wave][a] = v[a];
  __syncthreads();
  if (threadIdx.x < 6) {
    float r = s_v[0][threadIdx.x];
    for (int w = 1; w < kBlock / kWave; ++w)
      r = threadIdx.x < 3 ? fminf(r, s_v[w][threadIdx.x]) : fmaxf(r, s_v[w][threadIdx.x]);
    part[(size_t)blockIdx.x * 6 + threadIdx.x] = r;
  }
}

// box = {lo x, lo y, lo z, scale = 1024 / side (0 when side == 0)}
__global__ __launch_bounds__(kBlock) void k_bbox_final(const float* __restrict__ part, uint32_t nb,
                                                       float* __restrict__ box) {
  __shared__ float s_v[kBlock / kWave][6];
  float v[6];
  for (int a = 0; a < 3; ++a) {
    v[a] = __builtin_huge_valf();
    v[3 + a] = -__builtin_huge_valf();
  }
  for (uint32_t b = threadIdx.x; b < nb; b += kBlock)
    for (int a = 0; a < 3; ++a) {
      v[a] = fminf(v[a], part[(size_t)b * 6 + a]);
      v[3 + a] = fmaxf(v[3 + a], part[(size_t)b * 6 + 3 + a]);
    }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v[a] = fminf(v[a], __shfl_xor(v[a], d, kWave));
      v[3 + a] = fmaxf(v[3 + a], __shfl_xor(v[3 + a], d, kWave));
    }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0)
    for (int a = 0; a < 6; ++a) s_v[wave][a] = v[a];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w)
      for (int a = 0; a < 3; ++a) {
        v[a] = fminf(v[a], s_v[w][a]);
        v[3 + a] = fmaxf(v[3 + a], s_v[w][3 + a]);
      }
    const float side = fmaxf(fmaxf(v[3] - v[0], v[4] - v[1]), v[5] - v[2]);
    box[0] = v[0];
    box[1] = v[1];
    box[2] = v[2];
    box[3] = side > 0.0f ? 1024.0f / side : 0.0f;
  }
}

// 10-bit value -> bits at positions 0, 3, 6, ..., 27 (shift-and-mask spreading)
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__global__ __launch_bounds__(kBlock) void k_morton(const float* __restrict__ means, uint32_t n,
                                                   const float* __restrict__ box, uint32_t* __restrict__ codes,
                                                   uint32_t* __restrict__ idx) {
#pragma clang fp contract(off)
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float s = box[3];
  uint32_t q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float t = (means[(size_t)a * n + i] - box[a]) * s;
    q[a] = s > 0.0f ? min(1023u, (uint32_t)t) : 0u;
  }
  codes[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  idx[i] = i;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_permute(const T* __restrict__ src, T* __restrict__ dst, uint32_t n,
                                                    const uint32_t* __restrict__ perm) {
  const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const size_t p = (size_t)blockIdx.y * n;
  dst[p + k] = src[p + perm[k]];
}

size_t zorder_scratch_bytes(uint64_t n) {
  const uint64_t nb = (n + kBlock - 1) / kBlock;
  const uint64_t words = 3 * round_up64(n) + round_up64(6 * nb) + 64 + round_up64(radix_scratch_words(n));
  return words * 4;
}

// scratch: codes[2][n], idx[n] (the second value buffer is `perm`), bbox
// partials, box, radix scratch.
hipError_t launch_zorder(const float* means, uint32_t n, void* scratch, uint32_t* perm, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint32_t* w = static_cast<uint32_t*>(scratch);
  uint32_t* codes0 = w;
  uint32_t* codes1 = codes0 + round_up64(n);
  uint32_t* idx1 = codes1 + round_up64(n);
  const uint32_t nb = ceil_div(n, kBlock);
  float* part = reinterpret_cast<float*>(idx1 + round_up64(n));
  float* box = part + round_up64(6 * (uint64_t)nb);
  uint32_t* rscratch = reinterpret_cast<uint32_t*>(box + 64);
  k_bbox_partial<<<nb, kBlock, 0, s>>>(means, n, part);
  k_bbox_final<<<1, kBlock, 0, s>>>(part, nb, box);
  k_morton<<<nb, kBlock, 0, s>>>(means, n, box, codes0, perm);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint32_t* keys[2] = {codes0, codes1};
  uint32_t* vals[2] = {perm, idx1};
  int fin = 0;
  e = radix_sort_pairs(keys, vals, n, nullptr, 0, 30, rscratch, &fin, s, nullptr, false);
  if (e != hipSuccess) return e;
  if (fin != 0) return hipMemcpyAsync(perm, vals[fin], (size_t)n * 4, hipMemcpyDeviceToDevice, s);
  return hipSuccess;
}

hipError_t launch_permute(const void* src, void* dst, uint32_t n, int planes, int elem_bytes,
                          const uint32_t* perm, hipStream_t s) {
  if (n == 0 || planes == 0) return hipSuccess;
  const dim3 grid(ceil_div(n, kBlock), (uint32_t)planes);
  if (elem_bytes == 2)
    k_permute<uint16_t><<<grid, kBlock, 0, s>>>(static_cast<const uint16_t*>(src), static_cast<uint16_t*>(dst), n,
                                                perm);
  else
    k_permute<uint32_t><<<grid, kBlock, 0, s>>>(static_cast<const uint32_t*>(src), static_cast<uint32_t*>(dst), n,
                                                perm);
  return hipGetLastError();
}

}  // namespace fgs
