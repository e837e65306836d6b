// Fused multi-group Adam (Sec. 3.3 "Parameter Updates": one fused kernel that
// matches PyTorch's Adam; every element is updated, also with a zero gradient)
// and the L1 loss gradient (Sec. 2.1, App. A loss).
//
// Adam streams p, g, m, v once (16 B read + 12 B written per element) with
// 16-byte vector accesses; one launch covers all parameter groups, each with
// its own learning rate.  The update follows torch.optim.Adam's float32 order:
//   m += (1 - b1) (g - m);  v = b2 v + (1 - b2) g^2;
//   p -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps).
#include "fgs_internal.h"

namespace fgs {

constexpr int kMaxGroups = 16;

struct AdamGroupDev {
  float* p;
  const float* g;
  float* m;
  float* v;
  uint64_t numel;
  uint64_t vec_begin;  // first float4 slot of this group in the flattened launch
  float step_size;     // lr / (1 - b1^t)
  int32_t vec4;        // all four pointers 16-byte aligned
};

struct AdamArgs {
  AdamGroupDev grp[kMaxGroups];
  int32_t n_groups;
  float one_minus_b1, beta2, one_minus_b2, inv_sqrt_bc2, eps;
};

__device__ __forceinline__ void adam_elem(float& p, float g, float& m, float& v, const AdamArgs& a, float step) {
  m = fmaf(a.one_minus_b1, g - m, m);
  v = fmaf(a.one_minus_b2, g * g, v * a.beta2);
  const float denom = sqrtf(v) * a.inv_sqrt_bc2 + a.eps;
  p = p - step * (m / denom);
}

constexpr int kAdamSlots = 2;  // float4 slots per thread (more loads in flight)

typedef float vf4 __attribute__((ext_vector_type(4)));
// Streaming load of a gradient that is read exactly once.
__device__ __forceinline__ float4 load_once4(const float* p) {
  const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ int adam_group(const AdamArgs& a, uint64_t slot) {
  int gi = 0;
#pragma unroll 1
  while (gi + 1 < a.n_groups && slot >= a.grp[gi + 1].vec_begin) ++gi;
  return gi;
}

// Each workgroup covers kAdamSlots * 256 consecutive float4 slots; thread t
// takes slots t and t + 256 so that every load instruction is coalesced.
__global__ __launch_bounds__(kBlock) void k_adam(AdamArgs a, uint64_t total_vec) {
  const uint64_t base = (uint64_t)blockIdx.x * (kBlock * kAdamSlots) + threadIdx.x;
  float4 p[kAdamSlots], g[kAdamSlots], m[kAdamSlots], v[kAdamSlots];
  int gi[kAdamSlots];
  bool vec[kAdamSlots];
#pragma unroll
  for (int u = 0; u < kAdamSlots; ++u) {
    const uint64_t slot = base + (uint64_t)u * kBlock;
    vec[u] = false;
    gi[u] = 0;
    if (slot >= total_vec) continue;
    gi[u] = adam_group(a, slot);
    const AdamGroupDev& G = a.grp[gi[u]];
    const uint64_t e0 = (slot - G.vec_begin) * 4;
    vec[u] = G.vec4 && e0 + 4 <= G.numel;
    if (vec[u]) {
      p[u] = *reinterpret_cast<const float4*>(G.p + e0);
      g[u] = load_once4(G.g + e0);
      m[u] = *reinterpret_cast<const float4*>(G.m + e0);
      v[u] = *reinterpret_cast<const float4*>(G.v + e0);
    }
  }
#pragma unroll
  for (int u = 0; u < kAdamSlots; ++u) {
    const uint64_t slot = base + (uint64_t)u * kBlock;
    if (slot >= total_vec) continue;
    const AdamGroupDev& G = a.grp[gi[u]];
    const uint64_t e0 = (slot - G.vec_begin) * 4;
    if (vec[u]) {
      adam_elem(p[u].x, g[u].x, m[u].x, v[u].x, a, G.step_size);
      adam_elem(p[u].y, g[u].y, m[u].y, v[u].y, a, G.step_size);
      adam_elem(p[u].z, g[u].z, m[u].z, v[u].z, a, G.step_size);
      adam_elem(p[u].w, g[u].w, m[u].w, v[u].w, a, G.step_size);
      *reinterpret_cast<float4*>(G.p + e0) = p[u];
      *reinterpret_cast<float4*>(G.m + e0) = m[u];
      *reinterpret_cast<float4*>(G.v + e0) = v[u];
    } else {
      for (uint64_t e = e0; e < e0 + 4 && e < G.numel; ++e) {
        float pe = G.p[e], me = G.m[e], ve = G.v[e];
        adam_elem(pe, G.g[e], me, ve, a, G.step_size);
        G.p[e] = pe;
        G.m[e] = me;
        G.v[e] = ve;
      }
    }
  }
}

hipError_t launch_adam(const fgs_adam_group* groups, int n_groups, int64_t step, double beta1, double beta2,
                       double eps, hipStream_t s) {
  AdamArgs a = {};
  a.n_groups = n_groups;
  const double bc1 = 1.0 - std::pow(beta1, (double)step);
  const double bc2 = 1.0 - std::pow(beta2, (double)step);
  a.one_minus_b1 = (float)(1.0 - beta1);
  a.beta2 = (float)beta2;
  a.one_minus_b2 = (float)(1.0 - beta2);
  a.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
  a.eps = (float)eps;
  uint64_t vec = 0;
  for (int k = 0; k < n_groups; ++k) {
    AdamGroupDev& G = a.grp[k];
    G.p = groups[k].param;
    G.g = groups[k].grad;
    G.m = groups[k].exp_avg;
    G.v = groups[k].exp_avg_sq;
    G.numel = (uint64_t)groups[k].numel;
    G.vec_begin = vec;
    G.step_size = (float)((double)groups[k].lr / bc1);
    const uintptr_t bits = (uintptr_t)G.p | (uintptr_t)G.g | (uintptr_t)G.m | (uintptr_t)G.v;
    G.vec4 = (bits & 15u) == 0 ? 1 : 0;
    vec += (G.numel + 3) / 4;
  }
  if (vec == 0) return hipSuccess;
  const uint64_t per_block = (uint64_t)kBlock * kAdamSlots;
  k_adam<<<(uint32_t)((vec + per_block - 1) / per_block), kBlock, 0, s>>>(a, vec);
  return hipGetLastError();
}

// dL/dC = sign(C - target) / n; optional float64 sum of |C - target| / n.
__global__ __launch_bounds__(kBlock) void k_l1(const float* __restrict__ img, const float* __restrict__ tgt,
                                               uint32_t n, float inv_n, double inv_n64, float* __restrict__ dl,
                                               double* __restrict__ loss) {
  __shared__ double part[kBlock / kWave];
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  double a = 0.0;
  if (i < n) {
    const float d = img[i] - tgt[i];
    dl[i] = d > 0.0f ? inv_n : (d < 0.0f ? -inv_n : 0.0f);
    a = fabs((double)img[i] - (double)tgt[i]);
  }
  if (loss == nullptr) return;
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) a += __shfl_xor(a, m, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    unsafeAtomicAdd(loss, t * inv_n64);
  }
}

hipError_t launch_l1_backward(const float* image, const float* target, uint32_t n, float* dl, double* loss,
                              hipStream_t s) {
  if (loss) {
    hipError_t e = hipMemsetAsync(loss, 0, sizeof(double), s);
    if (e != hipSuccess) return e;
  }
  if (n == 0) return hipSuccess;
  k_l1<<<ceil_div(n, kBlock), kBlock, 0, s>>>(image, target, n, (float)(1.0 / (double)n), 1.0 / (double)n, dl,
                                              loss);
  return hipGetLastError();
}

}  // namespace fgs
