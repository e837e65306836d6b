// Backward of the per-Gaussian preprocess: from the accumulated gradients of
// the 2D splat (mu2D, conic, opacity, colour) to the raw parameters, with the
// activation gradients fused in (Sec. 3.2 "Rasterization Kernel Fusion").
//
// A thread takes four consecutive Gaussians, so the planes of Gaussians
// whose nine accumulators are all zero (not rendered, or hidden behind
// terminated pixels; the large majority) are streamed with 16-byte accesses.
// A lane then loops over its own Gaussians that did receive a gradient, so the
// lanes of a wave evaluate the chain rule together.  The forward quantities it
// needs are recomputed from the parameters; the conic, opacity and the
// colour-clip flags are read from the forward record.
//
// The fused variant (Sec. 3.3 "Fusing Backward and Optimizer") evaluates the
// chain rule only for the Gaussians that received a gradient, keeps their
// gradients in slots of a compact buffer, and leaves every parameter update
// to one streaming Adam pass (see k_touched_list below).
//
// Chain (per Gaussian, K = conic = H^-1 with H the dilated Sigma2D):
//   dL/dH = -K dL/dK K                         (b counted on both off-diagonals)
//   dL/dSigma = T^T dL/dSigma2D T,  dL/dT = 2 dL/dSigma2D T Sigma,  T = J W3
//   J(x, y, z) of Eq. (2) and Eq. (1) give dL/d(camera position); dL/dmu = W3^T (.)
//   Sigma = M M^T, M = R diag(s): dL/dM = 2 dL/dSigma M
//   R(q/|q|) and the normalisation; s = exp(log s); o = sigmoid(logit)
//   colour: SH coefficients and the view direction (through mu).
#include <algorithm>

#include "fgs_internal.h"

namespace fgs {

__device__ __forceinline__ void sh_basis_and_grad(float x, float y, float z, float* Y, float* dYx, float* dYy,
                                                  float* dYz) {
  const float xx = x * x, yy = y * y, zz = z * z;
  const float C1 = 0.4886025119029199f;
  const float C20 = 1.0925484305920792f, C21 = -1.0925484305920792f, C22 = 0.31539156525252005f,
              C23 = -1.0925484305920792f, C24 = 0.5462742152960396f;
  const float C30 = -0.5900435899266435f, C31 = 2.890611442640554f, C32 = -0.4570457994644658f,
              C33 = 0.3731763325901154f, C34 = -0.4570457994644658f, C35 = 1.445305721320277f,
              C36 = -0.5900435899266435f;
  Y[0] = 0.28209479177387814f; dYx[0] = 0.f; dYy[0] = 0.f; dYz[0] = 0.f;
  Y[1] = -C1 * y; dYx[1] = 0.f; dYy[1] = -C1; dYz[1] = 0.f;
  Y[2] = C1 * z; dYx[2] = 0.f; dYy[2] = 0.f; dYz[2] = C1;
  Y[3] = -C1 * x; dYx[3] = -C1; dYy[3] = 0.f; dYz[3] = 0.f;
  Y[4] = C20 * x * y; dYx[4] = C20 * y; dYy[4] = C20 * x; dYz[4] = 0.f;
  Y[5] = C21 * y * z; dYx[5] = 0.f; dYy[5] = C21 * z; dYz[5] = C21 * y;
  Y[6] = C22 * (2.f * zz - xx - yy); dYx[6] = -2.f * C22 * x; dYy[6] = -2.f * C22 * y; dYz[6] = 4.f * C22 * z;
  Y[7] = C23 * x * z; dYx[7] = C23 * z; dYy[7] = 0.f; dYz[7] = C23 * x;
  Y[8] = C24 * (xx - yy); dYx[8] = 2.f * C24 * x; dYy[8] = -2.f * C24 * y; dYz[8] = 0.f;
  Y[9] = C30 * y * (3.f * xx - yy); dYx[9] = C30 * 6.f * x * y; dYy[9] = C30 * 3.f * (xx - yy); dYz[9] = 0.f;
  Y[10] = C31 * x * y * z; dYx[10] = C31 * y * z; dYy[10] = C31 * x * z; dYz[10] = C31 * x * y;
  Y[11] = C32 * y * (4.f * zz - xx - yy); dYx[11] = C32 * (-2.f * x * y);
  dYy[11] = C32 * (4.f * zz - xx - 3.f * yy); dYz[11] = C32 * 8.f * y * z;
  Y[12] = C33 * z * (2.f * zz - 3.f * xx - 3.f * yy); dYx[12] = C33 * (-6.f * x * z);
  dYy[12] = C33 * (-6.f * y * z); dYz[12] = C33 * (6.f * zz - 3.f * xx - 3.f * yy);
  Y[13] = C34 * x * (4.f * zz - xx - yy); dYx[13] = C34 * (4.f * zz - 3.f * xx - yy);
  dYy[13] = C34 * (-2.f * x * y); dYz[13] = C34 * 8.f * x * z;
  Y[14] = C35 * z * (xx - yy); dYx[14] = C35 * 2.f * x * z; dYy[14] = C35 * (-2.f * y * z); dYz[14] = C35 * (xx - yy);
  Y[15] = C36 * x * (xx - 3.f * yy); dYx[15] = C36 * 3.f * (xx - yy); dYy[15] = C36 * (-6.f * x * y); dYz[15] = 0.f;
}

// The 59 raw parameters of a Gaussian, as planes of six groups: means (3),
// log_scales (3), quats (4), opacity logit (1), sh_dc (3), sh_rest (45).
constexpr int kParams = 59;
__host__ __device__ constexpr int group_of(int p) {
  return p < 3 ? 0 : p < 6 ? 1 : p < 10 ? 2 : p < 11 ? 3 : p < 14 ? 4 : 5;
}
__host__ __device__ constexpr int first_plane(int grp) {
  return grp == 0 ? 0 : grp == 1 ? 3 : grp == 2 ? 6 : grp == 3 ? 10 : grp == 4 ? 11 : 14;
}

// Plane p of a group set (groups 4 and 5 hold the SH element type).
template <bool SHB>
__device__ __forceinline__ float plane_load(const void* const* base, int p, size_t n, size_t i) {
  const int gi = group_of(p);
  const size_t off = (size_t)(p - first_plane(gi)) * n + i;
  if (gi >= 4) return sh_load<SHB>(base[gi], off);
  return static_cast<const float*>(base[gi])[off];
}
template <bool SHB>
__device__ __forceinline__ void plane_store(void* const* base, int p, size_t n, size_t i, float v) {
  const int gi = group_of(p);
  const size_t off = (size_t)(p - first_plane(gi)) * n + i;
  if (gi >= 4) sh_store<SHB>(base[gi], off, v);
  else static_cast<float*>(base[gi])[off] = v;
}
// Four consecutive elements (i0 % 4 == 0, planes aligned).
template <bool SHB>
__device__ __forceinline__ float4 plane_load4(const void* const* base, int p, size_t n, size_t i0) {
  const int gi = group_of(p);
  const size_t off = (size_t)(p - first_plane(gi)) * n + i0;
  if (SHB && gi >= 4) {
    const uint2 v = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(base[gi]) + off);
    return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                       __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
  }
  return *reinterpret_cast<const float4*>(static_cast<const float*>(base[gi]) + off);
}
template <bool SHB>
__device__ __forceinline__ void plane_store4(void* const* base, int p, size_t n, size_t i0, float4 v) {
  const int gi = group_of(p);
  const size_t off = (size_t)(p - first_plane(gi)) * n + i0;
  if (SHB && gi >= 4) {
    *reinterpret_cast<uint2*>(static_cast<uint16_t*>(base[gi]) + off) =
        make_uint2((uint32_t)f32_to_bf16(v.x) | ((uint32_t)f32_to_bf16(v.y) << 16),
                   (uint32_t)f32_to_bf16(v.z) | ((uint32_t)f32_to_bf16(v.w) << 16));
  } else {
    *reinterpret_cast<float4*>(static_cast<float*>(base[gi]) + off) = v;
  }
}

// The part of the chain rule every covariance model shares: from the nine
// accumulated 2D gradients acc = dL/d(mu2D.x, mu2D.y, a, b, c, o, r, g, b)
// of Gaussian i (record rec[rj], mean mu, 3D covariance S) to dL/dmu (with
// the colour's view-direction term), the symmetric matrix gradient dL/dS, and
// the SH coefficients, handed to emit(11..58, value).  go = dL/d(opacity of
// the record).
struct SplatGrads {
  float dmu[3];
  float dS[3][3];
  float go, o;
};

template <bool SHB, typename Emit>
__device__ __forceinline__ SplatGrads splat_grads(const GaussDev& g, const CamDev& cam, const float4* __restrict__ rec,
                                                  const float* acc, uint32_t i, size_t rj, const float* mu,
                                                  const float (&S)[3][3], Emit&& emit) {
#pragma clang fp contract(on)
  const size_t n = g.n;
  const float gmx = acc[0], gmy = acc[1], ga = acc[2], gb = acc[3], gc = acc[4], go = acc[5];
  const float4 r0 = rec[kRecWords * rj + 0];
  const float4 r1 = rec[kRecWords * rj + 1];
  const float4 r2 = rec[kRecWords * rj + 2];
  const float o = r0.z, ka = r1.x, kb = r1.y, kc = r1.z;
  const uint32_t clip = __float_as_uint(r2.w);
  const float* W = cam.w;

  // ---- recompute the forward quantities
  const float mu0 = mu[0], mu1 = mu[1], mu2 = mu[2];
  const float X = W[0] * mu0 + W[1] * mu1 + W[2] * mu2 + W[3];
  const float Yc = W[4] * mu0 + W[5] * mu1 + W[6] * mu2 + W[7];
  const float Z = W[8] * mu0 + W[9] * mu1 + W[10] * mu2 + W[11];
  const float iz = 1.0f / Z;
  const float u = X * iz, v = Yc * iz;
  const float j00 = cam.fx * iz, j11 = cam.fy * iz, j02 = -j00 * u, j12 = -j11 * v;
  float Tm[2][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Tm[0][k] = j00 * W[k] + j02 * W[8 + k];
    Tm[1][k] = j11 * W[4 + k] + j12 * W[8 + k];
  }
  float U[2][3];  // T Sigma
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) U[a][k] = Tm[a][0] * S[0][k] + Tm[a][1] * S[1][k] + Tm[a][2] * S[2][k];

  // ---- conic -> dilated covariance -> Sigma2D (dilation is additive)
  const float hb = 0.5f * gb;  // b appears on both off-diagonals of K
  const float P00 = ga * ka + hb * kb, P01 = ga * kb + hb * kc;
  const float P10 = hb * ka + gc * kb, P11 = hb * kb + gc * kc;
  const float Q00 = ka * P00 + kb * P10, Q01 = ka * P01 + kb * P11, Q11 = kb * P01 + kc * P11;
  const float G00 = -Q00, G11 = -Q11, G01 = -Q01;  // matrix-form dL/dSigma2D (symmetric)

  // ---- Sigma2D = T Sigma T^T
  float A[2][3];  // G2 T
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A[0][k] = G00 * Tm[0][k] + G01 * Tm[1][k];
    A[1][k] = G01 * Tm[0][k] + G11 * Tm[1][k];
  }
  float dS[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dS[a][b] = Tm[0][a] * A[0][b] + Tm[1][a] * A[1][b];
  float dT[2][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dT[0][k] = 2.f * (G00 * U[0][k] + G01 * U[1][k]);
    dT[1][k] = 2.f * (G01 * U[0][k] + G11 * U[1][k]);
  }
  // ---- T = J W3
  const float dj00 = dT[0][0] * W[0] + dT[0][1] * W[1] + dT[0][2] * W[2];
  const float dj02 = dT[0][0] * W[8] + dT[0][1] * W[9] + dT[0][2] * W[10];
  const float dj11 = dT[1][0] * W[4] + dT[1][1] * W[5] + dT[1][2] * W[6];
  const float dj12 = dT[1][0] * W[8] + dT[1][1] * W[9] + dT[1][2] * W[10];
  const float iz2 = iz * iz, iz3 = iz2 * iz;
  const float dX = -cam.fx * iz2 * dj02 + gmx * cam.fx * iz;
  const float dY = -cam.fy * iz2 * dj12 + gmy * cam.fy * iz;
  const float dZ = -cam.fx * iz2 * dj00 - cam.fy * iz2 * dj11 + 2.f * cam.fx * X * iz3 * dj02 +
                   2.f * cam.fy * Yc * iz3 * dj12 - gmx * cam.fx * X * iz2 - gmy * cam.fy * Yc * iz2;
  float dmu[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) dmu[k] = W[k] * dX + W[4 + k] * dY + W[8 + k] * dZ;

  // ---- colour: SH coefficients and the view direction
  const float dc0 = (clip & 1u) ? 0.f : acc[6];
  const float dc1 = (clip & 2u) ? 0.f : acc[7];
  const float dc2 = (clip & 4u) ? 0.f : acc[8];
  float ddx = mu0 - cam.campos[0], ddy = mu1 - cam.campos[1], ddz = mu2 - cam.campos[2];
  const float len = sqrtf(ddx * ddx + ddy * ddy + ddz * ddz);
  const float il = 1.0f / len;
  ddx *= il; ddy *= il; ddz *= il;
  float Y[16], dYx[16], dYy[16], dYz[16];
  sh_basis_and_grad(ddx, ddy, ddz, Y, dYx, dYy, dYz);
  float gdx = 0.f, gdy = 0.f, gdz = 0.f;
  // the DC band: Y[0] is constant, so it adds no view-direction term
  emit(11, dc0 * Y[0]);
  emit(12, dc1 * Y[0]);
  emit(13, dc2 * Y[0]);
  // every coefficient is loaded before the first is used (loads guarded by the
  // run-time band count would each be waited for in turn)
  const int K = g.sh_coeffs;  // 1, 4, 9 or 16
  float rest[45];
  if (K == 16) {  // uniform
#pragma unroll
    for (int q = 0; q < 45; ++q) rest[q] = sh_load<SHB>(g.sh_rest, (size_t)q * n + i);
  } else {
#pragma unroll
    for (int q = 0; q < 45; ++q) rest[q] = (q < 3 * (K - 1)) ? sh_load<SHB>(g.sh_rest, (size_t)q * n + i) : 0.0f;
  }
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    const int q = 14 + 3 * (k - 1);
    if (k < K) {
      const int q3 = 3 * (k - 1);
      const float e = dc0 * rest[q3] + dc1 * rest[q3 + 1] + dc2 * rest[q3 + 2];
      gdx = fmaf(e, dYx[k], gdx);
      gdy = fmaf(e, dYy[k], gdy);
      gdz = fmaf(e, dYz[k], gdz);
      emit(q, dc0 * Y[k]);
      emit(q + 1, dc1 * Y[k]);
      emit(q + 2, dc2 * Y[k]);
    } else {
      emit(q, 0.f);
      emit(q + 1, 0.f);
      emit(q + 2, 0.f);
    }
  }
  const float dot = ddx * gdx + ddy * gdy + ddz * gdz;
  SplatGrads out;
  out.dmu[0] = dmu[0] + (gdx - ddx * dot) * il;
  out.dmu[1] = dmu[1] + (gdy - ddy * dot) * il;
  out.dmu[2] = dmu[2] + (gdz - ddz * dot) * il;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) out.dS[a][b] = dS[a][b];
  out.go = go;
  out.o = o;
  return out;

}

// Gradient of the loss w.r.t. the 59 raw parameters of a 3D Gaussian i:
// Sigma = M M^T, M = R(q / |q|) diag(exp(log s)), opacity = sigmoid(logit).
// Each gradient is handed to emit(p, value) as soon as it is known, with the
// parameter index p a compile-time constant after unrolling.  mu is the mean
// the view saw (the means themselves, or mean(t) of a dynamic scene), and
// emit(0..2, .) receives dL/dmu.
template <bool SHB, typename Emit>
__device__ __forceinline__ void gaussian_grads(const GaussDev& g, const CamDev& cam, const float4* __restrict__ rec,
                                               const float* acc, uint32_t i, size_t rj, const float* mu,
                                               Emit&& emit) {
#pragma clang fp contract(on)
  const size_t n = g.n;
  const float qw0 = g.quats[i], qx0 = g.quats[n + i], qy0 = g.quats[2 * n + i], qz0 = g.quats[3 * n + i];
  const float qn = sqrtf(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
  const float iqn = 1.0f / qn;
  const float w = qw0 * iqn, x = qx0 * iqn, y = qy0 * iqn, z = qz0 * iqn;
  float R[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                   {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                   {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
  const float s[3] = {expf(g.log_scales[i]), expf(g.log_scales[n + i]), expf(g.log_scales[2 * n + i])};
  float M[3][3], S[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[a][b] = R[a][b] * s[b];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) S[a][b] = M[a][0] * M[b][0] + M[a][1] * M[b][1] + M[a][2] * M[b][2];
  const SplatGrads sg = splat_grads<SHB>(g, cam, rec, acc, i, rj, mu, S, emit);
  emit(0, sg.dmu[0]);
  emit(1, sg.dmu[1]);
  emit(2, sg.dmu[2]);
  const float(&dS)[3][3] = sg.dS;

  // ---- Sigma = M M^T, M = R diag(s)
  float dM[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dM[a][b] = 2.f * (dS[a][0] * M[0][b] + dS[a][1] * M[1][b] + dS[a][2] * M[2][b]);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const float ds = dM[0][b] * R[0][b] + dM[1][b] * R[1][b] + dM[2][b] * R[2][b];
    emit(3 + b, ds * s[b]);
  }
  float dR[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dR[a][b] = dM[a][b] * s[b];
  const float dw = 2.f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
  const float dx = 2.f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.f * x * dR[1][1] - w * dR[1][2] +
                          z * dR[2][0] + w * dR[2][1] - 2.f * x * dR[2][2]);
  const float dy = 2.f * (-2.f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] -
                          w * dR[2][0] + z * dR[2][1] - 2.f * y * dR[2][2]);
  const float dz = 2.f * (-2.f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.f * z * dR[1][1] +
                          y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
  const float qdot = w * dw + x * dx + y * dy + z * dz;
  emit(6, (dw - w * qdot) * iqn);
  emit(7, (dx - x * qdot) * iqn);
  emit(8, (dy - y * qdot) * iqn);
  emit(9, (dz - z * qdot) * iqn);

  // ---- opacity = sigmoid(logit)
  emit(10, sg.go * sg.o * (1.f - sg.o));
}

// Gradient of the loss w.r.t. the raw parameters of a conditional 4D
// Gaussian i seen at time t (Sec. 3.4): planes 0..58 as for a 3D Gaussian
// (means = the spatial mean, log_scales = the spatial log-scales, quats =
// the left quaternion) and 59 = mean_t, 60 = log_scale_t, 61..64 = quats_r.
// Forward: Sigma4 = M M^T, M = R4 diag(s), R4 from the two unit quaternions;
// b = Sigma_xyz,t, c = Sigma_tt, dt = t - mean_t;
// mean = mu + b dt / c, S = Sigma_xyz,xyz - b b^T / c, p = exp(-dt^2 / (2c)),
// opacity = sigmoid(logit) p.  Chain (G = dL/dS, gm = dL/dmean, gp = dL/dp):
//   dL/db = -2 G b / c + gm dt / c
//   dL/dc = b^T G b / c^2 - (gm . b) dt / c^2 + gp p dt^2 / (2 c^2)
//   dL/dmean_t = -(gm . b) / c + gp p dt / c
//   dL/dSigma4: G on the spatial block, dL/db / 2 on each off-diagonal
//   border, dL/dc in the corner; dL/dM = 2 dL/dSigma4 M
//   R4 = L(a) R(b) (reordered): dL/dL = dP R^T, dL/dR = L^T dP.
constexpr int kCond4Params = kParams + 6;

template <bool SHB, typename Emit>
__device__ __forceinline__ void gaussian_grads_cond4(const GaussDev& g, const CamDev& cam,
                                                     const float4* __restrict__ rec, const float* acc, uint32_t i,
                                                     size_t rj, float t, Emit&& emit) {
#pragma clang fp contract(on)
  const size_t n = g.n;
  const float ql[4] = {g.quats[i], g.quats[n + i], g.quats[2 * n + i], g.quats[3 * n + i]};
  const float qr[4] = {g.quats_r[i], g.quats_r[n + i], g.quats_r[2 * n + i], g.quats_r[3 * n + i]};
  const float s[4] = {expf(g.log_scales[i]), expf(g.log_scales[n + i]), expf(g.log_scales[2 * n + i]),
                      expf(g.log_scale_t[i])};
  const float dt = t - g.mean_t[i];
  const float logit = g.logits[i];
  float a[4], b[4], qna, qnb;
  unit_quat(ql, a, qna);
  unit_quat(qr, b, qnb);
  float L[4][4], Rq[4][4];
  quat_lr(a, b, L, Rq);
  float R4[4][4];
  rotation4(a, b, R4);
  float M[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) M[r][k] = R4[r][k] * s[k];
  // the conditional Gaussian as the forward pass evaluates it
  float h[3], e, S6[6];
  condition_m(M, dt, h, e, S6);
  const float mu[3] = {g.means[i] + h[0] * e, g.means[n + i] + h[1] * e, g.means[2 * n + i] + h[2] * e};
  const float S[3][3] = {{S6[0], S6[1], S6[2]}, {S6[1], S6[3], S6[4]}, {S6[2], S6[4], S6[5]}};
  const float p = expf(-0.5f * e * e);
  // Sigma_xyz,t and Sigma_tt for the chain
  auto sig = [&](int r) { return M[r][0] * M[3][0] + M[r][1] * M[3][1] + M[r][2] * M[3][2] + M[r][3] * M[3][3]; };
  const float bv[3] = {sig(0), sig(1), sig(2)};
  const float ic = 1.0f / sig(3);
  const SplatGrads sg = splat_grads<SHB>(g, cam, rec, acc, i, rj, mu, S, emit);
  const float os = 1.0f / (1.0f + expf(-logit));
  const float gp = sg.go * os;
  emit(10, sg.go * p * os * (1.f - os));
  emit(0, sg.dmu[0]);
  emit(1, sg.dmu[1]);
  emit(2, sg.dmu[2]);
  // ---- conditioning
  float Gb[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) Gb[r] = sg.dS[r][0] * bv[0] + sg.dS[r][1] * bv[1] + sg.dS[r][2] * bv[2];
  const float bGb = bv[0] * Gb[0] + bv[1] * Gb[1] + bv[2] * Gb[2];
  const float gmb = sg.dmu[0] * bv[0] + sg.dmu[1] * bv[1] + sg.dmu[2] * bv[2];
  const float gpp = gp * p;
  float G4[4][4];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float db = (-2.f * Gb[r] + sg.dmu[r] * dt) * ic;
#pragma unroll
    for (int q = 0; q < 3; ++q) G4[r][q] = sg.dS[r][q];
    G4[r][3] = 0.5f * db;
    G4[3][r] = 0.5f * db;
  }
  G4[3][3] = (bGb - gmb * dt + 0.5f * gpp * dt * dt) * ic * ic;
  emit(kParams, (-gmb + gpp * dt) * ic);  // mean_t
  // ---- Sigma4 = M M^T, M = R4 diag(s)
  float dM[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k)
      dM[r][k] = 2.f * (G4[r][0] * M[0][k] + G4[r][1] * M[1][k] + G4[r][2] * M[2][k] + G4[r][3] * M[3][k]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float ds = dM[0][k] * R4[0][k] + dM[1][k] * R4[1][k] + dM[2][k] * R4[2][k] + dM[3][k] * R4[3][k];
    emit(k < 3 ? 3 + k : kParams + 1, ds * s[k]);
  }
  // ---- R4 = L(a) R(b), reordered from (w, x, y, z) to (x, y, z, t)
  constexpr int pm[4] = {1, 2, 3, 0};
  float dP[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) dP[pm[r]][pm[q]] = dM[r][q] * s[q];
  float dL[4][4], dR[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dL[r][q] = dP[r][0] * Rq[q][0] + dP[r][1] * Rq[q][1] + dP[r][2] * Rq[q][2] + dP[r][3] * Rq[q][3];
      dR[r][q] = L[0][r] * dP[0][q] + L[1][r] * dP[1][q] + L[2][r] * dP[2][q] + L[3][r] * dP[3][q];
    }
  const float da[4] = {dL[0][0] + dL[1][1] + dL[2][2] + dL[3][3], -dL[0][1] + dL[1][0] - dL[2][3] + dL[3][2],
                       -dL[0][2] + dL[1][3] + dL[2][0] - dL[3][1], -dL[0][3] - dL[1][2] + dL[2][1] + dL[3][0]};
  const float db4[4] = {dR[0][0] + dR[1][1] + dR[2][2] + dR[3][3], -dR[0][1] + dR[1][0] + dR[2][3] - dR[3][2],
                        -dR[0][2] - dR[1][3] + dR[2][0] + dR[3][1], -dR[0][3] + dR[1][2] - dR[2][1] + dR[3][0]};
  // ---- normalisation of both quaternions
  const float adot = a[0] * da[0] + a[1] * da[1] + a[2] * da[2] + a[3] * da[3];
  const float bdot = b[0] * db4[0] + b[1] * db4[1] + b[2] * db4[2] + b[3] * db4[3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    emit(6 + k, (da[k] - a[k] * adot) / qna);
    emit(kParams + 2 + k, (db4[k] - b[k] * bdot) / qnb);
  }
}

// The nine accumulators of Gaussians i0..i0+3 (zero past n; accum is
// [n][9], so the four are 36 consecutive floats: nine 16-byte loads when
// `full`) and the mask of those with any nonzero one.
__device__ __forceinline__ uint32_t load_accum4(const float* __restrict__ accum, size_t n, uint32_t i0, bool full,
                                                float (&acc)[4][9]) {
  const float* src = accum + (size_t)i0 * 9;
  if (full) {
    float f[36];
#pragma unroll
    for (int w = 0; w < 9; ++w) {
      const float4 a = reinterpret_cast<const float4*>(src)[w];
      f[4 * w] = a.x; f[4 * w + 1] = a.y; f[4 * w + 2] = a.z; f[4 * w + 3] = a.w;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 9; ++q) acc[j][q] = f[9 * j + q];
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 9; ++q) acc[j][q] = (i0 + j < n) ? src[9 * j + q] : 0.0f;
  }
  uint32_t mask = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < 9; ++q) any |= acc[j][q] != 0.0f;
    mask |= any ? (1u << j) : 0u;
  }
  return mask;
}

// acc[j] for a lane-varying j, by selects (no indexed register arrays).
__device__ __forceinline__ void pick_accum(const float (&acc)[4][9], int j, float* a) {
#pragma unroll
  for (int q = 0; q < 9; ++q)
    a[q] = j == 0 ? acc[0][q] : j == 1 ? acc[1][q] : j == 2 ? acc[2][q] : acc[3][q];
}

// vec: n % 4 == 0 and every plane base aligned for 4-element accesses.
template <bool SHB>
__global__ __launch_bounds__(kBlock) void k_preprocess_bwd(GaussDev g, CamDev cam, const float4* __restrict__ rec,
                                                           const float* __restrict__ accum, GradDev gr, int vec) {
  const uint32_t i0 = (blockIdx.x * kBlock + threadIdx.x) * 4u;
  const size_t n = g.n;
  if (i0 >= n) return;
  void* const out[6] = {gr.means, gr.log_scales, gr.quats, gr.logits, gr.sh_dc, gr.sh_rest};
  const bool full = vec && i0 + 4 <= n;
  float acc[4][9];
  const uint32_t mask = load_accum4(accum, n, i0, full, acc);
  // zeros first (16-byte stores when the four are complete); the Gaussians
  // with a gradient overwrite theirs below
  if (full) {
    if (mask != 0xfu) {
#pragma unroll
      for (int p = 0; p < kParams; ++p) plane_store4<SHB>(out, p, n, i0, make_float4(0.f, 0.f, 0.f, 0.f));
    }
  } else {
    for (int j = 0; j < 4; ++j) {
      if (i0 + j >= n || (mask >> j & 1u)) continue;
#pragma unroll
      for (int p = 0; p < kParams; ++p) plane_store<SHB>(out, p, n, i0 + j, 0.0f);
    }
  }
  uint32_t todo = mask;
  while (todo) {
    const int j = __builtin_ctz(todo);
    todo &= todo - 1u;
    float a[9];
    pick_accum(acc, j, a);
    const uint32_t i = i0 + j;
    const float mu[3] = {g.means[i], g.means[n + i], g.means[2 * n + i]};
    gaussian_grads<SHB>(g, cam, rec, a, i, i, mu, [&](int p, float v) { plane_store<SHB>(out, p, n, i, v); });
  }
}

// ---------------------------------------------------------------------------
// Fused backward + Adam (Sec. 3.3 "Fusing Backward and Optimizer").  In a
// step only a small share of the Gaussians receives a gradient, scattered
// over the index range; updating their parameters where they lie costs a
// memory sector per 4-byte access, and the streaming step then reads the same
// lines again.  So no full gradient buffer and no separate update:
//   k_touched_list   one pass over the blend backward's byte marks (1 byte
//                    per Gaussian instead of its 36-byte accumulator row):
//                    the 4-bit mark of each group of four Gaussians, and for
//                    the marked ones a compact list and each one's slot in it
//                    (one atomic per wave on a counter)
//   k_touched_grads  the chain rule for the listed Gaussians only; their 59
//                    gradients go to slot s of plane-major [59][n] storage,
//                    so a plane's gradients of neighbouring Gaussians are
//                    adjacent
//   k_adam_sparse    one streaming Adam pass over every parameter, which
//                    takes a marked Gaussian's gradient from its slot and
//                    zero for all others (adam_loss.hip).
__global__ __launch_bounds__(kBlock) void k_touched_list(uint8_t* __restrict__ marks, uint32_t n,
                                                         uint8_t* __restrict__ touched,
                                                         uint32_t* __restrict__ counter,
                                                         uint32_t* __restrict__ list,
                                                         uint32_t* __restrict__ slot_of, bool rezero) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t i0 = (blockIdx.x * kBlock + threadIdx.x) * 4u;
  if ((blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1u))) * 4u >= n) return;  // whole wave past the end
  uint32_t mask = 0;
  if (i0 < n) {
    uint32_t m4 = 0;  // the four mark bytes (the region is 256-byte aligned, i0 a multiple of 4)
    if (i0 + 4 <= n) {
      m4 = *reinterpret_cast<const uint32_t*>(marks + i0);
      if (rezero && m4) *reinterpret_cast<uint32_t*>(marks + i0) = 0u;  // read: cleared for the next backward
    } else {
      for (uint32_t j = 0; i0 + j < n; ++j) m4 |= (uint32_t)marks[i0 + j] << (8 * j);
      if (rezero)
        for (uint32_t j = 0; i0 + j < n; ++j) marks[i0 + j] = 0u;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) mask |= ((m4 >> (8 * j)) & 0xffu) ? (1u << j) : 0u;
    touched[i0 / 4] = (uint8_t)mask;
  }
  // exclusive prefix of the lanes' counts (0..4, three bit planes) and the wave total
  const uint32_t cnt = (uint32_t)__popc(mask);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const uint64_t m = __ballot((cnt >> b) & 1u);
    pre += (uint32_t)__popcll(m & below) << b;
    tot += (uint32_t)__popcll(m) << b;
  }
  if (tot == 0) return;  // wave-uniform
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(counter, tot);
  base = (uint32_t)__shfl((int)base, 0, kWave);
  uint32_t slot = base + pre;
  for (int j = 0; j < 4; ++j) {
    if (!(mask >> j & 1u)) continue;
    list[slot] = i0 + j;
    slot_of[i0 + j] = slot;
    ++slot;
  }
}

// One thread per listed Gaussian (grid-stride; every thread exits once the
// list is done).  A bfloat16 SH gradient is rounded as a stored one would be.
template <bool SHB>
__global__ __launch_bounds__(kBlock) void k_touched_grads(GaussDev g, CamDev cam, const float4* __restrict__ rec,
                                                          float* __restrict__ accum,
                                                          const uint32_t* __restrict__ counter,
                                                          const uint32_t* __restrict__ list,
                                                          float* __restrict__ grads, bool rezero) {
  const size_t n = g.n;
  const uint32_t count = min(*counter, (uint32_t)n);
  for (uint32_t slot = blockIdx.x * kBlock + threadIdx.x; slot < count; slot += gridDim.x * kBlock) {
    const uint32_t i = list[slot];
    float a[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) a[q] = accum[(size_t)i * 9 + q];
    const float mu[3] = {g.means[i], g.means[n + i], g.means[2 * n + i]};
    // the 59 gradients are kept in registers and stored after the chain rule,
    // so that none of its loads has to wait behind a store (the kernel runs
    // few waves and is bound by this thread's chain of memory round trips)
    float out[kParams];
#pragma unroll
    for (int p = 0; p < kParams; ++p) out[p] = 0.0f;
    gaussian_grads<SHB>(g, cam, rec, a, i, i, mu, [&](int p, float v) {
      out[p] = group_of(p) >= 4 ? sh_round<SHB>(v) : v;
    });
#pragma unroll
    for (int p = 0; p < kParams; ++p) grads[(size_t)p * n + slot] = out[p];
    if (rezero) {  // read: cleared for the next backward
#pragma unroll
      for (int q = 0; q < 9; ++q) accum[(size_t)i * 9 + q] = 0.0f;
    }
  }
}

// Several views (or timesteps): Gaussian i sums, over the views that gave it
// a gradient, the chain rule through view v's camera and record j = v n + i.
// Dynamic scenes (mean(t) = mu + v t + a t^2) also get dL/dvelocity =
// sum_t t dL/dmean(t) and dL/daccel = sum_t t^2 dL/dmean(t).  Every gradient
// plane is written in full.
//
// One wave per 64 Gaussians.  The entries with a nonzero accumulator row are
// the ones the blend backward marked; the wave walks its Gaussians' marked
// entries 64 at a time (load-balanced, each Gaussian's in view order), so
// every lane evaluates the chain rule of a real entry, where a lane per
// Gaussian would leave most lanes idle whenever a view is needed by only a
// few Gaussians of the wave.  A step's gradients pass through LDS, one row
// per lane; the lane of each Gaussian then adds the rows of its entries in
// view order (the same additions, in the same order, as a loop over its
// views) and writes the sums once at the end.
template <bool SHB, bool C4>
__global__ __launch_bounds__(kWave) void k_preprocess_bwd_views(GaussDev g, ViewSet vs,
                                                                const float4* __restrict__ rec,
                                                                float* __restrict__ accum,
                                                                uint8_t* __restrict__ marks, GradDev gr,
                                                                bool rezero) {
  constexpr int kSum = C4 ? kCond4Params : kParams;
  constexpr int kRow = C4 ? kSum : kSum + 6;  // + t dL/dmean(t) and t^2 dL/dmean(t) of a dynamic scene
  __shared__ float s_row[kWave][kRow + 1];
  __shared__ uint32_t s_owner_at[kWave];
  const int lane = threadIdx.x;
  const size_t n = g.n;
  const uint32_t i = blockIdx.x * kWave + (uint32_t)lane;
  const bool dyn = g.velocity != nullptr;
  // this lane's Gaussian's marked views and its run in the wave's list
  uint32_t vmask = 0;
  if (i < n)
    for (uint32_t v = 0; v < vs.n_views; ++v) vmask |= marks[(size_t)v * n + i] ? (1u << v) : 0u;
  // rezero: the marks and rows read here are cleared for the next backward
  if (rezero)
    for (uint32_t m = vmask; m != 0u; m &= m - 1u) marks[(size_t)__builtin_ctz(m) * n + i] = 0u;
  const uint32_t cnt = (uint32_t)__popc(vmask);
  const uint32_t incl = wave_inclusive_scan(cnt, lane);
  const uint32_t start = incl - cnt;
  const uint32_t total = __shfl(incl, kWave - 1, kWave);
  const uint64_t upto = ((lane == 0) ? 0ull : (~0ull >> (64 - lane))) | (1ull << lane);
  float sum[kRow];
#pragma unroll
  for (int p = 0; p < kRow; ++p) sum[p] = 0.0f;
  lds_volatile_u32* owner_at = lds_volatile(s_owner_at);
  owner_at[lane] = 0xffffffffu;  // no step tag matches
  wave_lds_sync();
  float* row = s_row[lane];
  uint32_t tag = 0;
  for (uint32_t c0 = 0; c0 < total; c0 += kWave, tag += 0x100u) {
    bool claims;
    uint32_t first;
    const int owner = wave_run_owner(start, cnt, c0, tag, owner_at, upto, claims, first);
    const uint32_t pos = c0 + (uint32_t)lane;
    const uint32_t o_start = (uint32_t)__shfl((int)start, owner, kWave);
    const uint32_t o_mask = (uint32_t)__shfl((int)vmask, owner, kWave);
    if (pos < total) {
      // the owner's (pos - o_start)-th marked view
      uint32_t m = o_mask;
      for (uint32_t k = pos - o_start; k > 0; --k) m &= m - 1u;
      const uint32_t v = (uint32_t)__builtin_ctz(m);
      const uint32_t gi = blockIdx.x * kWave + (uint32_t)owner;
      const size_t rj = (size_t)v * n + gi;
      float a[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) a[q] = accum[rj * 9 + q];
      if (rezero) {
#pragma unroll
        for (int q = 0; q < 9; ++q) accum[rj * 9 + q] = 0.0f;
      }
      const float t = vs.time[v], tt = t * t;
      if (C4) {
        gaussian_grads_cond4<SHB>(g, vs.cam[v], rec, a, gi, rj, t, [&](int p, float val) { row[p] = val; });
      } else {
        float mu[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          mu[k] = g.means[k * n + gi];
          if (dyn) mu[k] = (mu[k] + g.velocity[k * n + gi] * t) + g.accel[k * n + gi] * tt;
        }
        gaussian_grads<SHB>(g, vs.cam[v], rec, a, gi, rj, mu, [&](int p, float val) {
          row[p] = val;
          if (p < 3) {
            row[kSum + p] = t * val;
            row[kSum + 3 + p] = tt * val;
          }
        });
      }
    }
    wave_lds_sync();
    // the lane of each Gaussian with entries in this step adds their rows
    if (claims) {
      const uint32_t hi = min(start + cnt - c0, (uint32_t)kWave);  // exclusive
      for (uint32_t q = first; q < hi; ++q) {
#pragma unroll
        for (int p = 0; p < kRow; ++p) sum[p] += s_row[q][p];
      }
    }
    wave_lds_sync();  // the rows are read before the next step writes them
  }
  if (i >= n) return;
  void* const out[6] = {gr.means, gr.log_scales, gr.quats, gr.logits, gr.sh_dc, gr.sh_rest};
#pragma unroll
  for (int p = 0; p < kParams; ++p) plane_store<SHB>(out, p, n, i, sum[p]);
  if (C4) {
    gr.mean_t[i] = sum[kParams];
    gr.log_scale_t[i] = sum[kParams + 1];
#pragma unroll
    for (int k = 0; k < 4; ++k) gr.quats_r[k * n + i] = sum[kParams + 2 + k];
  }
  if (dyn) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gr.velocity[k * n + i] = sum[kSum + k];
      gr.accel[k * n + i] = sum[kSum + 3 + k];
    }
  }
}

hipError_t launch_preprocess_backward_views(const GaussDev& g, const ViewSet& vs, const float4* rec, float* accum,
                                            uint8_t* marks, const GradDev& gr, bool rezero, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const uint32_t grid = ceil_div(g.n, kWave);
  const bool c4 = g.quats_r != nullptr;
  if (g.sh_bf16 && c4)
    k_preprocess_bwd_views<true, true><<<grid, kWave, 0, s>>>(g, vs, rec, accum, marks, gr, rezero);
  else if (g.sh_bf16)
    k_preprocess_bwd_views<true, false><<<grid, kWave, 0, s>>>(g, vs, rec, accum, marks, gr, rezero);
  else if (c4)
    k_preprocess_bwd_views<false, true><<<grid, kWave, 0, s>>>(g, vs, rec, accum, marks, gr, rezero);
  else
    k_preprocess_bwd_views<false, false><<<grid, kWave, 0, s>>>(g, vs, rec, accum, marks, gr, rezero);
  return hipGetLastError();
}

static bool planes_vec(const void* const* base, int count, bool sh_bf16, size_t n) {
  if (n % 4 != 0) return false;
  for (int k = 0; k < count; ++k) {
    const uintptr_t a = (uintptr_t)base[k];
    const uintptr_t need = (sh_bf16 && (k % 6) >= 4) ? 8u : 16u;
    if (a % need) return false;
  }
  return true;
}

hipError_t launch_preprocess_backward(const GaussDev& g, const CamDev& cam, const float4* rec, const float* accum,
                                      const GradDev& gr, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const void* const planes[6] = {gr.means, gr.log_scales, gr.quats, gr.logits, gr.sh_dc, gr.sh_rest};
  const int vec = planes_vec(planes, 6, g.sh_bf16, g.n) ? 1 : 0;
  const uint32_t grid = ceil_div(ceil_div(g.n, 4), kBlock);
  if (g.sh_bf16)
    k_preprocess_bwd<true><<<grid, kBlock, 0, s>>>(g, cam, rec, accum, gr, vec);
  else
    k_preprocess_bwd<false><<<grid, kBlock, 0, s>>>(g, cam, rec, accum, gr, vec);
  return hipGetLastError();
}

hipError_t launch_touched_gradients(const GaussDev& g, const CamDev& cam, const float4* rec, float* accum,
                                    uint8_t* marks, uint8_t* touched, uint32_t* counter, uint32_t* list,
                                    uint32_t* slot_of, float* grads, bool rezero, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  if ((uintptr_t)marks % 4) return hipErrorInvalidValue;
  k_touched_list<<<ceil_div(ceil_div(g.n, 4), kBlock), kBlock, 0, s>>>(marks, g.n, touched, counter, list, slot_of,
                                                                        rezero);
  const uint32_t grid = std::min<uint32_t>(ceil_div(g.n, kBlock), 2048u);
  if (g.sh_bf16)
    k_touched_grads<true><<<grid, kBlock, 0, s>>>(g, cam, rec, accum, counter, list, grads, rezero);
  else
    k_touched_grads<false><<<grid, kBlock, 0, s>>>(g, cam, rec, accum, counter, list, grads, rezero);
  return hipGetLastError();
}

}  // namespace fgs
