// Per-Gaussian projection math, evaluated by the preprocess kernel and
// re-evaluated (instead of stored) by the backward kernel.
//
// Formulation notes (same function as the definition in gs.h, arranged for
// float32 accuracy):
//  * Sigma2 = J W Sigma W^T J^T is formed as A A^T with A = J (W R(q) S),
//    a 2x3 matrix, so Sigma2 = [[|A0|^2, A0.A1], [A0.A1, |A1|^2]].
//  * det(Sigma2 + 0.3 I) = |A0 x A1|^2 + 0.3 tr(Sigma2) + 0.09 (Lagrange's
//    identity): a sum of non-negative terms, free of the cancellation that
//    ac - b^2 suffers for elongated splats.
//  * lambda_max = (a + c)/2 + sqrt(((a - c)/2)^2 + b^2), again without
//    cancellation.
#pragma once

#include "gs_internal.h"

namespace gsmi {

// Real spherical-harmonic basis constants (orthonormal real SH with the
// Condon-Shortley phase, index l^2 + l + m), written as Cartesian polynomials
// of the unit direction.
constexpr float kSH0 = 0.28209479177387814f;
constexpr float kSH1 = 0.4886025119029199f;
constexpr float kSH2_0 = 1.0925484305920792f;
constexpr float kSH2_1 = -1.0925484305920792f;
constexpr float kSH2_2 = 0.31539156525252005f;
constexpr float kSH2_3 = -1.0925484305920792f;
constexpr float kSH2_4 = 0.5462742152960396f;
constexpr float kSH3_0 = -0.5900435899266435f;
constexpr float kSH3_1 = 2.890611442640554f;
constexpr float kSH3_2 = -0.4570457994644658f;
constexpr float kSH3_3 = 0.3731763325901154f;
constexpr float kSH3_4 = -0.4570457994644658f;
constexpr float kSH3_5 = 1.445305721320277f;
constexpr float kSH3_6 = -0.5900435899266435f;

template <int DEG>
struct SHDim {
  static constexpr int K = (DEG + 1) * (DEG + 1);
};

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kSH0;
  if (DEG >= 1) {
    Y[1] = -kSH1 * y;
    Y[2] = kSH1 * z;
    Y[3] = -kSH1 * x;
  }
  if (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kSH2_0 * x * y;
    Y[5] = kSH2_1 * y * z;
    Y[6] = kSH2_2 * (2.0f * zz - xx - yy);
    Y[7] = kSH2_3 * x * z;
    Y[8] = kSH2_4 * (xx - yy);
    if (DEG >= 3) {
      Y[9] = kSH3_0 * y * (3.0f * xx - yy);
      Y[10] = kSH3_1 * x * y * z;
      Y[11] = kSH3_2 * y * (4.0f * zz - xx - yy);
      Y[12] = kSH3_3 * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
      Y[13] = kSH3_4 * x * (4.0f * zz - xx - yy);
      Y[14] = kSH3_5 * z * (xx - yy);
      Y[15] = kSH3_6 * x * (xx - 3.0f * yy);
    }
  }
}

// sum_k w[k] grad Y_k(x, y, z) (gradient of the Cartesian polynomials).
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float* w,
                                              float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if (DEG >= 1) {
    gy += -kSH1 * w[1];
    gz += kSH1 * w[2];
    gx += -kSH1 * w[3];
  }
  if (DEG >= 2) {
    gx += kSH2_0 * y * w[4];
    gy += kSH2_0 * x * w[4];
    gy += kSH2_1 * z * w[5];
    gz += kSH2_1 * y * w[5];
    gx += -2.0f * kSH2_2 * x * w[6];
    gy += -2.0f * kSH2_2 * y * w[6];
    gz += 4.0f * kSH2_2 * z * w[6];
    gx += kSH2_3 * z * w[7];
    gz += kSH2_3 * x * w[7];
    gx += 2.0f * kSH2_4 * x * w[8];
    gy += -2.0f * kSH2_4 * y * w[8];
    if (DEG >= 3) {
      const float xx = x * x, yy = y * y, zz = z * z;
      gx += 6.0f * kSH3_0 * x * y * w[9];
      gy += 3.0f * kSH3_0 * (xx - yy) * w[9];
      gx += kSH3_1 * y * z * w[10];
      gy += kSH3_1 * x * z * w[10];
      gz += kSH3_1 * x * y * w[10];
      gx += -2.0f * kSH3_2 * x * y * w[11];
      gy += kSH3_2 * (4.0f * zz - xx - 3.0f * yy) * w[11];
      gz += 8.0f * kSH3_2 * y * z * w[11];
      gx += -6.0f * kSH3_3 * x * z * w[12];
      gy += -6.0f * kSH3_3 * y * z * w[12];
      gz += kSH3_3 * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
      gx += kSH3_4 * (4.0f * zz - 3.0f * xx - yy) * w[13];
      gy += -2.0f * kSH3_4 * x * y * w[13];
      gz += 8.0f * kSH3_4 * x * z * w[13];
      gx += 2.0f * kSH3_5 * x * z * w[14];
      gy += -2.0f * kSH3_5 * y * z * w[14];
      gz += kSH3_5 * (xx - yy) * w[14];
      gx += 3.0f * kSH3_6 * (xx - yy) * w[15];
      gy += -6.0f * kSH3_6 * x * y * w[15];
    }
  }
}

// View-independent state of one Gaussian.
struct GaussState {
  float mu[3];
  float s[3];       // exp(log_scale)
  float q[4];       // normalised (w, x, y, z)
  float qnorm;
  float Rq[9];      // R(q), row-major
  float M[9];       // R(q) diag(s), row-major
  float o;          // sigmoid(logit)
  bool ok;          // finite and |q| > 0
};

__device__ __forceinline__ void load_gauss(const float* __restrict__ means,
                                           const float* __restrict__ log_scales,
                                           const float* __restrict__ quats,
                                           const float* __restrict__ ologit, int64_t n, int64_t i,
                                           GaussState& G) {
  float ls[3], q[4];
  for (int k = 0; k < 3; ++k) {
    G.mu[k] = means[k * n + i];
    ls[k] = log_scales[k * n + i];
  }
  for (int k = 0; k < 4; ++k) q[k] = quats[k * n + i];
  const float ol = ologit[i];
  bool ok = isfinite(ol);
  for (int k = 0; k < 3; ++k) ok = ok && isfinite(G.mu[k]) && isfinite(ls[k]);
  for (int k = 0; k < 4; ++k) ok = ok && isfinite(q[k]);
  const float qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  ok = ok && qn2 > 0.0f;
  G.ok = ok;
  const float qn = ok ? sqrtf(qn2) : 1.0f;
  G.qnorm = qn;
  const float inv = 1.0f / qn;
  const float w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
  G.q[0] = w; G.q[1] = x; G.q[2] = y; G.q[3] = z;
  for (int k = 0; k < 3; ++k) G.s[k] = ok ? expf(ls[k]) : 0.0f;
  G.o = ok ? 1.0f / (1.0f + expf(-ol)) : 0.0f;
  float* R = G.Rq;
  R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
  R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
  R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) G.M[r * 3 + c] = R[r * 3 + c] * G.s[c];
}

// Per-view state of one Gaussian.
struct ViewState {
  float p[3];           // camera-frame position
  float inv_z;
  float tx, ty;         // clamped x/z, y/z
  bool clx, cly;        // clamp active
  float J00, J02, J11, J12;
  float B[9];           // W R(q) diag(s), row-major
  float A0[3], A1[3];   // rows of J B
  float a, b, c;        // Sigma2 entries (before dilation)
  float det;            // det(Sigma')
  float q0, q1, q2;     // conic
  float u, v;
  int32_t radius;
  float dir[3];         // unit direction camera centre -> mean
  float dnorm;
  float rgb[3];
  bool rgb_pos[3];      // unclamped colour >= 0
  bool visible;
};

// SH coefficients of one Gaussian, [3][K] in registers.
template <int DEG>
struct SHCoef {
  float f[3 * SHDim<DEG>::K];
};

template <int DEG>
__device__ __forceinline__ void load_sh(const float* __restrict__ sh, int64_t n, int64_t i,
                                        SHCoef<DEG>& C) {
  constexpr int K = SHDim<DEG>::K;
#pragma unroll
  for (int k = 0; k < 3 * K; ++k) C.f[k] = sh[k * n + i];
}

template <int DEG>
__device__ __forceinline__ void project_view(const GaussState& G, const gs_camera& cam,
                                             const SHCoef<DEG>& C, ViewState& S) {
  const float* W = cam.R;
  S.visible = false;
  S.radius = 0;
  // Camera-frame point in float64 from the float32 inputs (the products are
  // exact), rounded once: the float32 depth that orders splats is then the
  // correctly rounded depth, independent of summation order.
  for (int r = 0; r < 3; ++r) {
    const double pr = fma((double)W[r * 3 + 0], (double)G.mu[0],
                          fma((double)W[r * 3 + 1], (double)G.mu[1],
                              fma((double)W[r * 3 + 2], (double)G.mu[2], (double)cam.t[r])));
    S.p[r] = (float)pr;
  }
  const float z = S.p[2];
  if (!G.ok || !(z > kZNear)) return;
  S.inv_z = __builtin_amdgcn_rcpf(z);
  const float fx = cam.fx, fy = cam.fy;
  const float rx = S.p[0] * S.inv_z, ry = S.p[1] * S.inv_z;
  S.u = fx * rx + cam.cx;
  S.v = fy * ry + cam.cy;
  const float limx = kGuard * (0.5f * (float)cam.width / fx);
  const float limy = kGuard * (0.5f * (float)cam.height / fy);
  S.clx = !(rx >= -limx && rx <= limx);
  S.cly = !(ry >= -limy && ry <= limy);
  S.tx = fminf(fmaxf(rx, -limx), limx);
  S.ty = fminf(fmaxf(ry, -limy), limy);
  S.J00 = fx * S.inv_z;
  S.J02 = -fx * S.tx * S.inv_z;
  S.J11 = fy * S.inv_z;
  S.J12 = -fy * S.ty * S.inv_z;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      S.B[r * 3 + c] = W[r * 3 + 0] * G.M[0 * 3 + c] + W[r * 3 + 1] * G.M[1 * 3 + c] +
                       W[r * 3 + 2] * G.M[2 * 3 + c];
  for (int c = 0; c < 3; ++c) {
    S.A0[c] = S.J00 * S.B[0 * 3 + c] + S.J02 * S.B[2 * 3 + c];
    S.A1[c] = S.J11 * S.B[1 * 3 + c] + S.J12 * S.B[2 * 3 + c];
  }
  S.a = S.A0[0] * S.A0[0] + S.A0[1] * S.A0[1] + S.A0[2] * S.A0[2];
  S.b = S.A0[0] * S.A1[0] + S.A0[1] * S.A1[1] + S.A0[2] * S.A1[2];
  S.c = S.A1[0] * S.A1[0] + S.A1[1] * S.A1[1] + S.A1[2] * S.A1[2];
  const float m01 = S.A0[0] * S.A1[1] - S.A0[1] * S.A1[0];
  const float m02 = S.A0[0] * S.A1[2] - S.A0[2] * S.A1[0];
  const float m12 = S.A0[1] * S.A1[2] - S.A0[2] * S.A1[1];
  S.det = (m01 * m01 + m02 * m02 + m12 * m12) + kDilation * (S.a + S.c) + kDilation * kDilation;
  if (!(S.det > 0.0f)) return;
  const float inv_det = __builtin_amdgcn_rcpf(S.det);
  const float s0 = S.a + kDilation, s2 = S.c + kDilation;
  S.q0 = s2 * inv_det;
  S.q1 = -S.b * inv_det;
  S.q2 = s0 * inv_det;
  const float mid = 0.5f * (s0 + s2);
  const float hd = 0.5f * (S.a - S.c);
  const float lam = mid + sqrtf(hd * hd + S.b * S.b);
  S.radius = (int32_t)ceilf(3.0f * sqrtf(lam));
  // colour
  float cc[3];
  for (int k = 0; k < 3; ++k)
    cc[k] = -(W[0 * 3 + k] * cam.t[0] + W[1 * 3 + k] * cam.t[1] + W[2 * 3 + k] * cam.t[2]);
  float d[3] = {G.mu[0] - cc[0], G.mu[1] - cc[1], G.mu[2] - cc[2]};
  S.dnorm = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const float invd = __builtin_amdgcn_rsqf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int k = 0; k < 3; ++k) S.dir[k] = d[k] * invd;
  constexpr int K = SHDim<DEG>::K;
  float Y[K];
  sh_basis<DEG>(S.dir[0], S.dir[1], S.dir[2], Y);
  for (int ch = 0; ch < 3; ++ch) {
    float acc = 0.5f;
    for (int k = 0; k < K; ++k) acc += C.f[ch * K + k] * Y[k];
    S.rgb_pos[ch] = acc >= 0.0f;
    S.rgb[ch] = fmaxf(acc, 0.0f);
  }
  S.visible = S.radius > 0;
}

}  // namespace gsmi
