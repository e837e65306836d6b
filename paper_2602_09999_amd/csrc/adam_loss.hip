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

#include <cmath>

namespace fgs {

constexpr int kMaxGroups = 16;

struct AdamGroupDev {
  void* p;        // float32 or bfloat16 (bf16), like the gradient
  const void* g;
  float* m;
  float* v;
  uint64_t numel;
  uint64_t vec_begin;  // first 4-element slot of this group in the flattened launch
  float step_size;     // lr / (1 - b1^t)
  int32_t vec4;        // pointers aligned for 4-element vector accesses
  int32_t bf16;
};

// Optimizer state on the device, for steps whose count must advance inside a
// replayed graph: the step counter t and the scalars of step t.
struct AdamDevState {
  int64_t step;
  AdamCoef c;
  float step_size[kMaxGroups];  // lr_g / (1 - b1^t)
};
static_assert(sizeof(AdamDevState) <= 256, "state fits the caller's 256 bytes");

struct AdamArgs {
  AdamGroupDev grp[kMaxGroups];
  int32_t n_groups;
  AdamCoef c;
  const AdamDevState* dev;  // non-NULL: take c and the step sizes from here
};

struct LrList {
  float lr[kMaxGroups];
};

// One thread: t <- t + 1, then the scalars of step t in double, rounded once.
__global__ void k_adam_scalars(AdamDevState* __restrict__ st, double beta1, double beta2, double eps, LrList lrs,
                               int32_t n_groups) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t t = st->step + 1;
  st->step = t;
  const double bc1 = 1.0 - pow(beta1, (double)t);
  const double bc2 = 1.0 - pow(beta2, (double)t);
  st->c.one_minus_b1 = (float)(1.0 - beta1);
  st->c.beta2 = (float)beta2;
  st->c.one_minus_b2 = (float)(1.0 - beta2);
  st->c.inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
  st->c.eps = (float)eps;
  for (int k = 0; k < n_groups; ++k) st->step_size[k] = (float)((double)lrs.lr[k] / bc1);
}

AdamCoef adam_coef(int64_t step, double beta1, double beta2, double eps, double* bias1) {
  const double bc1 = 1.0 - std::pow(beta1, (double)step);
  const double bc2 = 1.0 - std::pow(beta2, (double)step);
  AdamCoef c;
  c.one_minus_b1 = (float)(1.0 - beta1);
  c.beta2 = (float)beta2;
  c.one_minus_b2 = (float)(1.0 - beta2);
  c.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(bc2));
  c.eps = (float)eps;
  if (bias1) *bias1 = bc1;
  return c;
}

constexpr int kAdamSlots = 2;  // 4-element slots per thread (more loads in flight)

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef unsigned int vu2 __attribute__((ext_vector_type(2)));
// Streaming loads of a gradient that is read exactly once.
__device__ __forceinline__ float4 load_once4(const void* p) {
  const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float4 load_once_bf16x4(const void* p) {
  const vu2 v = __builtin_nontemporal_load(reinterpret_cast<const vu2*>(p));
  return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                     __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
}
__device__ __forceinline__ void store_once4(float* p, float4 f) {
  const vf4 v = {f.x, f.y, f.z, f.w};
  __builtin_nontemporal_store(v, reinterpret_cast<vf4*>(p));
}
__device__ __forceinline__ void store_bf16x4(void* p, float4 f) {
  const vu2 v = {(uint32_t)f32_to_bf16(f.x) | ((uint32_t)f32_to_bf16(f.y) << 16),
                 (uint32_t)f32_to_bf16(f.z) | ((uint32_t)f32_to_bf16(f.w) << 16)};
  __builtin_nontemporal_store(v, reinterpret_cast<vu2*>(p));
}

__device__ __forceinline__ int adam_group(const AdamArgs& a, uint64_t slot) {
  int gi = 0;
#pragma unroll 1
  while (gi + 1 < a.n_groups && slot >= a.grp[gi + 1].vec_begin) ++gi;
  return gi;
}

__device__ __forceinline__ void adam4(float4& p, const float4& g, float4& m, float4& v, const AdamCoef& c,
                                      float step) {
  adam_elem(p.x, g.x, m.x, v.x, c, step);
  adam_elem(p.y, g.y, m.y, v.y, c, step);
  adam_elem(p.z, g.z, m.z, v.z, c, step);
  adam_elem(p.w, g.w, m.w, v.w, c, step);
}

// Each workgroup covers kAdamSlots * 256 consecutive 4-element slots; thread t
// takes slots t and t + 256 so that every load instruction is coalesced.
// bfloat16 parameters are widened, updated in float32 against float32
// moments and rounded back to nearest-even.
__global__ __launch_bounds__(kBlock) void k_adam(AdamArgs a, uint64_t total_vec) {
  // the scalars of this step: from the arguments, or from the device state
  const AdamCoef c = a.dev ? a.dev->c : a.c;
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
      // every stream is read once and written once: non-temporal accesses
      if (G.bf16) {
        p[u] = load_once_bf16x4(static_cast<const uint16_t*>(G.p) + e0);
        g[u] = load_once_bf16x4(static_cast<const uint16_t*>(G.g) + e0);
      } else {
        p[u] = load_once4(static_cast<const float*>(G.p) + e0);
        g[u] = load_once4(static_cast<const float*>(G.g) + e0);
      }
      m[u] = load_once4(G.m + e0);
      v[u] = load_once4(G.v + e0);
    }
  }
#pragma unroll
  for (int u = 0; u < kAdamSlots; ++u) {
    const uint64_t slot = base + (uint64_t)u * kBlock;
    if (slot >= total_vec) continue;
    const AdamGroupDev& G = a.grp[gi[u]];
    const uint64_t e0 = (slot - G.vec_begin) * 4;
    if (vec[u]) {
      adam4(p[u], g[u], m[u], v[u], c, a.dev ? a.dev->step_size[gi[u]] : G.step_size);
      if (G.bf16) store_bf16x4(static_cast<uint16_t*>(G.p) + e0, p[u]);
      else store_once4(static_cast<float*>(G.p) + e0, p[u]);
      store_once4(G.m + e0, m[u]);
      store_once4(G.v + e0, v[u]);
    } else if (G.bf16) {
      for (uint64_t e = e0; e < e0 + 4 && e < G.numel; ++e) {
        float pe = sh_load<true>(G.p, e), me = G.m[e], ve = G.v[e];
        adam_elem(pe, sh_load<true>(G.g, e), me, ve, c, a.dev ? a.dev->step_size[gi[u]] : G.step_size);
        sh_store<true>(G.p, e, pe);
        G.m[e] = me;
        G.v[e] = ve;
      }
    } else {
      for (uint64_t e = e0; e < e0 + 4 && e < G.numel; ++e) {
        float pe = sh_load<false>(G.p, e), me = G.m[e], ve = G.v[e];
        adam_elem(pe, sh_load<false>(G.g, e), me, ve, c, a.dev ? a.dev->step_size[gi[u]] : G.step_size);
        sh_store<false>(G.p, e, pe);
        G.m[e] = me;
        G.v[e] = ve;
      }
    }
  }
}

// step >= 1: host step count; step == 0: advance and use the device counter
// of dev_state (an AdamDevState).
hipError_t launch_adam(const fgs_adam_group* groups, int n_groups, int64_t step, double beta1, double beta2,
                       double eps, void* dev_state, hipStream_t s) {
  AdamArgs a = {};
  a.n_groups = n_groups;
  double bc1 = 1.0;
  a.c = adam_coef(step > 0 ? step : 1, beta1, beta2, eps, &bc1);
  a.dev = step > 0 ? nullptr : static_cast<const AdamDevState*>(dev_state);
  LrList lrs = {};
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
    lrs.lr[k] = groups[k].lr;
    G.bf16 = groups[k].dtype == FGS_BF16 ? 1 : 0;
    const uintptr_t pg = (uintptr_t)G.p | (uintptr_t)G.g, mv = (uintptr_t)G.m | (uintptr_t)G.v;
    G.vec4 = ((pg & (G.bf16 ? 7u : 15u)) == 0 && (mv & 15u) == 0) ? 1 : 0;
    vec += (G.numel + 3) / 4;
  }
  if (a.dev) {
    k_adam_scalars<<<1, kWave, 0, s>>>(static_cast<AdamDevState*>(dev_state), beta1, beta2, eps, lrs, n_groups);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (vec == 0) return hipSuccess;
  const uint64_t per_block = (uint64_t)kBlock * kAdamSlots;
  k_adam<<<(uint32_t)((vec + per_block - 1) / per_block), kBlock, 0, s>>>(a, vec);
  return hipGetLastError();
}

// Adam step over the six parameter groups of the Gaussians with sparse
// gradients: a Gaussian whose bit is set in `touched` takes its gradient of
// plane p from grads[p][slot_of[i]] (written by the fused backward), every
// other one a zero gradient; every parameter is updated.  Grid: (chunks of
// 4 * 256 Gaussians, the 59 planes): a thread takes four consecutive Gaussians
// of one plane, so the Gaussian index and the mark byte need no division, and
// every stream access is a 16-byte (8-byte for bfloat16) non-temporal one.
// Per float32 element 12 bytes are read and 12 written, plus the marks and,
// for marked Gaussians only, the slot and the gradient.
struct SparseAdamArgs {
  void* p[6];
  float* m[6];
  float* v[6];
  float step_size[6];
  AdamCoef c;
  uint32_t n;
  int32_t sh_bf16;
  int32_t vec;  // n % 4 == 0 and every plane 16-byte (8-byte for bfloat16) aligned
};

__device__ __forceinline__ int plane_group(int p) {
  return p < 3 ? 0 : p < 6 ? 1 : p < 10 ? 2 : p < 11 ? 3 : p < 14 ? 4 : 5;
}
__device__ __forceinline__ int group_first_plane(int g) {
  return g == 0 ? 0 : g == 1 ? 3 : g == 2 ? 6 : g == 3 ? 10 : g == 4 ? 11 : 14;
}

__global__ __launch_bounds__(kBlock) void k_adam_sparse(SparseAdamArgs a, const uint8_t* __restrict__ touched,
                                                        const uint32_t* __restrict__ slot_of,
                                                        const float* __restrict__ grads,
                                                        uint32_t* __restrict__ state_word, uint32_t state_tag) {
  // the chain rule before this launch left the accumulators zero: record it
  if (state_word != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
    *reinterpret_cast<uint2*>(state_word) = make_uint2(kAccumClean, state_tag);
  const int plane = blockIdx.y;
  const int gi = plane_group(plane);
  const size_t n = a.n;
  const size_t off = (size_t)(plane - group_first_plane(gi)) * n;
  const uint32_t q = blockIdx.x * kBlock + threadIdx.x;  // four Gaussians 4q .. 4q+3
  const uint32_t i0 = q * 4u;
  if (i0 >= a.n) return;
  const uint32_t mark = touched[q];
  float g4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (mark) {
    const float* gp = grads + (size_t)plane * n;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (mark >> e & 1u) g4[e] = gp[slot_of[i0 + e]];
  }
  const bool bf = a.sh_bf16 && gi >= 4;
  const float st = a.step_size[gi];
  float* M = a.m[gi] + off;
  float* V = a.v[gi] + off;
  if (a.vec && i0 + 4 <= a.n) {
    float4 pp;
    if (bf) {
      const vu2 u = __builtin_nontemporal_load(reinterpret_cast<const vu2*>(static_cast<uint16_t*>(a.p[gi]) + off + i0));
      pp = make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
    } else {
      const vf4 u = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(static_cast<float*>(a.p[gi]) + off + i0));
      pp = make_float4(u.x, u.y, u.z, u.w);
    }
    vf4 mm = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(M + i0));
    vf4 vv = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(V + i0));
    float m4[4] = {mm.x, mm.y, mm.z, mm.w}, v4[4] = {vv.x, vv.y, vv.z, vv.w};
    float p4[4] = {pp.x, pp.y, pp.z, pp.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) adam_elem(p4[e], g4[e], m4[e], v4[e], a.c, st);
    if (bf) {
      const vu2 u = {(uint32_t)f32_to_bf16(p4[0]) | ((uint32_t)f32_to_bf16(p4[1]) << 16),
                     (uint32_t)f32_to_bf16(p4[2]) | ((uint32_t)f32_to_bf16(p4[3]) << 16)};
      __builtin_nontemporal_store(u, reinterpret_cast<vu2*>(static_cast<uint16_t*>(a.p[gi]) + off + i0));
    } else {
      const vf4 u = {p4[0], p4[1], p4[2], p4[3]};
      __builtin_nontemporal_store(u, reinterpret_cast<vf4*>(static_cast<float*>(a.p[gi]) + off + i0));
    }
    const vf4 mo = {m4[0], m4[1], m4[2], m4[3]}, vo = {v4[0], v4[1], v4[2], v4[3]};
    __builtin_nontemporal_store(mo, reinterpret_cast<vf4*>(M + i0));
    __builtin_nontemporal_store(vo, reinterpret_cast<vf4*>(V + i0));
  } else {
    for (uint32_t e = 0; e < 4 && i0 + e < a.n; ++e) {
      const size_t k = off + i0 + e;
      float pe = bf ? sh_load<true>(a.p[gi], k) : sh_load<false>(a.p[gi], k);
      float me = a.m[gi][k], ve = a.v[gi][k];
      adam_elem(pe, g4[e], me, ve, a.c, st);
      if (bf) sh_store<true>(a.p[gi], k, pe);
      else sh_store<false>(a.p[gi], k, pe);
      a.m[gi][k] = me;
      a.v[gi][k] = ve;
    }
  }
}

hipError_t launch_adam_sparse(void* const params[6], float* const exp_avg[6], float* const exp_avg_sq[6],
                              const float lr[6], bool sh_bf16, uint64_t n, const uint8_t* touched,
                              const uint32_t* slot_of, const float* grads, int64_t step, double beta1, double beta2,
                              double eps, uint32_t* state_word, uint32_t state_tag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if ((uintptr_t)state_word % 8) return hipErrorInvalidValue;
  SparseAdamArgs a = {};
  double bc1 = 1.0;
  a.c = adam_coef(step, beta1, beta2, eps, &bc1);
  a.n = (uint32_t)n;
  a.sh_bf16 = sh_bf16 ? 1 : 0;
  bool vec = n % 4 == 0;
  for (int k = 0; k < 6; ++k) {
    a.p[k] = params[k];
    a.m[k] = exp_avg[k];
    a.v[k] = exp_avg_sq[k];
    a.step_size[k] = (float)((double)lr[k] / bc1);
    const uintptr_t need = (sh_bf16 && k >= 4) ? 7u : 15u;
    vec = vec && ((uintptr_t)params[k] & need) == 0 && ((uintptr_t)exp_avg[k] & 15u) == 0 &&
          ((uintptr_t)exp_avg_sq[k] & 15u) == 0;
  }
  a.vec = vec ? 1 : 0;
  const dim3 grid(ceil_div(ceil_div(n, 4), kBlock), 59);
  k_adam_sparse<<<grid, kBlock, 0, s>>>(a, touched, slot_of, grads, state_word, state_tag);
  return hipGetLastError();
}

// dL/dC = sign(C - target) / n; optional float64 sum of |C - target| / n.
// A thread takes four consecutive pixels values (16-byte accesses) when the
// buffers are 16-byte aligned, else one.
template <int V>
__global__ __launch_bounds__(kBlock) void k_l1(const float* __restrict__ img, const float* __restrict__ tgt,
                                               uint32_t n, float inv_n, double inv_n64, float* __restrict__ dl,
                                               double* __restrict__ loss) {
  __shared__ double part[kBlock / kWave];
  const uint32_t i0 = (blockIdx.x * kBlock + threadIdx.x) * (uint32_t)V;
  double a = 0.0;
  if (V == 4 && i0 + 4 <= n) {
    const float4 c = *reinterpret_cast<const float4*>(img + i0);
    const float4 t = *reinterpret_cast<const float4*>(tgt + i0);
    const float cv[4] = {c.x, c.y, c.z, c.w}, tv[4] = {t.x, t.y, t.z, t.w};
    float o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float d = cv[e] - tv[e];
      o[e] = d > 0.0f ? inv_n : (d < 0.0f ? -inv_n : 0.0f);
      if (loss) a += fabs((double)cv[e] - (double)tv[e]);
    }
    *reinterpret_cast<float4*>(dl + i0) = make_float4(o[0], o[1], o[2], o[3]);
  } else {
    for (uint32_t i = i0; i < i0 + V && i < n; ++i) {
      const float d = img[i] - tgt[i];
      dl[i] = d > 0.0f ? inv_n : (d < 0.0f ? -inv_n : 0.0f);
      a += fabs((double)img[i] - (double)tgt[i]);
    }
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
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(loss), 0u, 2, s);  // +0.0
    if (e != hipSuccess) return e;
  }
  if (n == 0) return hipSuccess;
  const float inv_n = (float)(1.0 / (double)n);
  const double inv_n64 = 1.0 / (double)n;
  if ((((uintptr_t)image | (uintptr_t)target | (uintptr_t)dl) & 15u) == 0)
    k_l1<4><<<ceil_div(ceil_div(n, 4), kBlock), kBlock, 0, s>>>(image, target, n, inv_n, inv_n64, dl, loss);
  else
    k_l1<1><<<ceil_div(n, kBlock), kBlock, 0, s>>>(image, target, n, inv_n, inv_n64, dl, loss);
  return hipGetLastError();
}

}  // namespace fgs
