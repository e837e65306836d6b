// Backward of the per-Gaussian preprocess: from the accumulated gradients of
// the 2D splat (mu2D, conic, opacity, colour) to the raw parameters, with the
// activation gradients fused in (Sec. 3.2 "Rasterization Kernel Fusion").
//
// One thread per Gaussian.  Gaussians whose nine accumulators are all zero
// (not rendered, or hidden behind terminated pixels) get zero gradients
// without touching their parameters.  The forward quantities needed by the
// chain rule are recomputed from the parameters; the conic, opacity and the
// colour-clip flags are read from the forward record.
//
// Chain (per Gaussian, K = conic = H^-1 with H the dilated Sigma2D):
//   dL/dH = -K dL/dK K                         (b counted on both off-diagonals)
//   dL/dSigma = T^T dL/dSigma2D T,  dL/dT = 2 dL/dSigma2D T Sigma,  T = J W3
//   J(x, y, z) of Eq. (2) and Eq. (1) give dL/d(camera position); dL/dmu = W3^T (.)
//   Sigma = M M^T, M = R diag(s): dL/dM = 2 dL/dSigma M
//   R(q/|q|) and the normalisation; s = exp(log s); o = sigmoid(logit)
//   colour: SH coefficients and the view direction (through mu).
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

__global__ __launch_bounds__(kBlock) void k_preprocess_bwd(GaussDev g, CamDev cam, SetDev st,
                                                           const float4* __restrict__ rec,
                                                           const float* __restrict__ accum, GradDev gr) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= g.n) return;
  const size_t n = g.n;
  float acc[9];
  bool any = false;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    acc[q] = accum[q * n + i];
    any |= acc[q] != 0.0f;
  }
  if (!any) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gr.means[k * n + i] = 0.f;
      gr.log_scales[k * n + i] = 0.f;
      gr.sh_dc[k * n + i] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) gr.quats[k * n + i] = 0.f;
    gr.logits[i] = 0.f;
    for (int k = 0; k < 45; ++k) gr.sh_rest[k * n + i] = 0.f;
    return;
  }
  const float gmx = acc[0], gmy = acc[1], ga = acc[2], gb = acc[3], gc = acc[4], go = acc[5];
  const float4 r0 = rec[3 * (size_t)i + 0];
  const float4 r1 = rec[3 * (size_t)i + 1];
  const float4 r2 = rec[3 * (size_t)i + 2];
  const float o = r0.z, ka = r1.x, kb = r1.y, kc = r1.z;
  const uint32_t clip = __float_as_uint(r2.w);
  const float* W = cam.w;

  // ---- recompute the forward quantities
  const float mu0 = g.means[i], mu1 = g.means[n + i], mu2 = g.means[2 * n + i];
  const float X = W[0] * mu0 + W[1] * mu1 + W[2] * mu2 + W[3];
  const float Yc = W[4] * mu0 + W[5] * mu1 + W[6] * mu2 + W[7];
  const float Z = W[8] * mu0 + W[9] * mu1 + W[10] * mu2 + W[11];
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
  float dX = -cam.fx * iz2 * dj02 + gmx * cam.fx * iz;
  float dY = -cam.fy * iz2 * dj12 + gmy * cam.fy * iz;
  float dZ = -cam.fx * iz2 * dj00 - cam.fy * iz2 * dj11 + 2.f * cam.fx * X * iz3 * dj02 +
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
  gr.sh_dc[i] = dc0 * Y[0];
  gr.sh_dc[n + i] = dc1 * Y[0];
  gr.sh_dc[2 * n + i] = dc2 * Y[0];
  for (int k = 1; k < 16; ++k) {
    float* gp = gr.sh_rest + (size_t)(3 * (k - 1)) * n + i;
    if (k < g.sh_coeffs) {
      const float* p = g.sh_rest + (size_t)(3 * (k - 1)) * n + i;
      const float e = dc0 * p[0] + dc1 * p[n] + dc2 * p[2 * n];
      gdx = fmaf(e, dYx[k], gdx);
      gdy = fmaf(e, dYy[k], gdy);
      gdz = fmaf(e, dYz[k], gdz);
      gp[0] = dc0 * Y[k];
      gp[n] = dc1 * Y[k];
      gp[2 * n] = dc2 * Y[k];
    } else {
      gp[0] = 0.f;
      gp[n] = 0.f;
      gp[2 * n] = 0.f;
    }
  }
  const float dot = ddx * gdx + ddy * gdy + ddz * gdz;
  dmu[0] += (gdx - ddx * dot) * il;
  dmu[1] += (gdy - ddy * dot) * il;
  dmu[2] += (gdz - ddz * dot) * il;
  gr.means[i] = dmu[0];
  gr.means[n + i] = dmu[1];
  gr.means[2 * n + i] = dmu[2];

  // ---- Sigma = M M^T, M = R diag(s)
  float dM[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dM[a][b] = 2.f * (dS[a][0] * M[0][b] + dS[a][1] * M[1][b] + dS[a][2] * M[2][b]);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const float ds = dM[0][b] * R[0][b] + dM[1][b] * R[1][b] + dM[2][b] * R[2][b];
    gr.log_scales[b * n + i] = ds * s[b];
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
  gr.quats[i] = (dw - w * qdot) * iqn;
  gr.quats[n + i] = (dx - x * qdot) * iqn;
  gr.quats[2 * n + i] = (dy - y * qdot) * iqn;
  gr.quats[3 * n + i] = (dz - z * qdot) * iqn;

  // ---- opacity = sigmoid(logit)
  gr.logits[i] = go * o * (1.f - o);
  (void)st;
}

hipError_t launch_preprocess_backward(const GaussDev& g, const CamDev& cam, const SetDev& st, const float4* rec,
                                      const float* accum, const GradDev& gr, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  k_preprocess_bwd<<<ceil_div(g.n, kBlock), kBlock, 0, s>>>(g, cam, st, rec, accum, gr);
  return hipGetLastError();
}

}  // namespace fgs
