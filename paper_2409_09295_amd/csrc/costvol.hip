// Plain Gaussian initialiser: the photometric cost volume of Eq. 1 over a
// window of keyframes at 1/4 resolution with 64 depth hypotheses evenly
// spaced over 0.25-25 m (Sec. III-A1), reduced per pixel by winner-take-all.
//
//   luma_down4   intensity 0.299 R + 0.587 G + 0.114 B averaged over 4x4
//                blocks, every keyframe
//   cost_wta     one lane per low-resolution pixel of the reference (last)
//                keyframe: for each hypothesis d the pixel's block centre is
//                back-projected at depth d, moved into every other keyframe,
//                projected and sampled bilinearly on that keyframe's
//                low-resolution grid; the cost is the mean absolute intensity
//                difference over the views where the sample is valid, and the
//                depth is the first hypothesis of minimum cost
#include "gs_internal.h"
#include "gs_nn.h"

namespace gsmi {

namespace {

constexpr int kHyp = 64;
constexpr float kDMin = 0.25f, kDMax = 25.0f;

__global__ void luma_down4_kernel(const float* __restrict__ rgb, int K, int H, int W,
                                  float* __restrict__ low) {
  const int Hl = H / 4, Wl = W / 4;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)K * Hl * Wl) return;
  const int k = (int)(i / ((int64_t)Hl * Wl));
  const int r = (int)(i - (int64_t)k * Hl * Wl);
  const int y = r / Wl, x = r % Wl;
  const int64_t plane = (int64_t)H * W;
  const float* img = rgb + (int64_t)k * 3 * plane;
  float s = 0.f;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const int64_t o = (int64_t)(4 * y + a) * W + 4 * x + b;
      s += 0.299f * img[o] + 0.587f * img[plane + o] + 0.114f * img[2 * plane + o];
    }
  low[i] = s * (1.0f / 16.0f);
}

__device__ __forceinline__ bool bilinear(const float* __restrict__ img, int Hl, int Wl, float x,
                                         float y, float& out) {
  if (!(x >= 0.f && y >= 0.f && x <= (float)(Wl - 1) && y <= (float)(Hl - 1))) return false;
  const int x0 = (int)floorf(x), y0 = (int)floorf(y);
  const int x1 = min(x0 + 1, Wl - 1), y1 = min(y0 + 1, Hl - 1);
  const float fx = x - (float)x0, fy = y - (float)y0;
  const float a = img[y0 * Wl + x0], b = img[y0 * Wl + x1];
  const float c = img[y1 * Wl + x0], d = img[y1 * Wl + x1];
  out = (1.f - fy) * ((1.f - fx) * a + fx * b) + fy * ((1.f - fx) * c + fx * d);
  return true;
}

__global__ __launch_bounds__(256) void cost_wta_kernel(const float* __restrict__ low, int K,
                                                       int Hl, int Wl,
                                                       const gs_camera* __restrict__ cams,
                                                       float* __restrict__ cost,
                                                       float* __restrict__ depth) {
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= (int64_t)Hl * Wl) return;
  const int y = (int)(pix / Wl), x = (int)(pix % Wl);
  const gs_camera ref = cams[K - 1];
  const float* Iref = low + (int64_t)(K - 1) * Hl * Wl;
  const float iref = Iref[pix];
  const float u = 4.0f * x + 2.0f, v = 4.0f * y + 2.0f;
  const float rx = (u - ref.cx) / ref.fx, ry = (v - ref.cy) / ref.fy;
  float best = INFINITY, best_d = 0.0f;
  for (int h = 0; h < kHyp; ++h) {
    const float d = kDMin + (kDMax - kDMin) * (float)h / (float)(kHyp - 1);
    // camera -> world: X_w = R^T (X_c - t)
    const float cx = rx * d - ref.t[0], cy = ry * d - ref.t[1], cz = d - ref.t[2];
    const float wx = ref.R[0] * cx + ref.R[3] * cy + ref.R[6] * cz;
    const float wy = ref.R[1] * cx + ref.R[4] * cy + ref.R[7] * cz;
    const float wz = ref.R[2] * cx + ref.R[5] * cy + ref.R[8] * cz;
    float sum = 0.f;
    int valid = 0;
    for (int k = 0; k < K - 1; ++k) {
      const gs_camera c = cams[k];
      const float px = c.R[0] * wx + c.R[1] * wy + c.R[2] * wz + c.t[0];
      const float py = c.R[3] * wx + c.R[4] * wy + c.R[5] * wz + c.t[1];
      const float pz = c.R[6] * wx + c.R[7] * wy + c.R[8] * wz + c.t[2];
      if (!(pz > 1e-6f)) continue;
      const float us = c.fx * px / pz + c.cx, vs = c.fy * py / pz + c.cy;
      float sample;
      if (!bilinear(low + (int64_t)k * Hl * Wl, Hl, Wl, (us - 2.0f) * 0.25f, (vs - 2.0f) * 0.25f,
                    sample))
        continue;
      sum += fabsf(iref - sample);
      ++valid;
    }
    const float cv = valid ? sum / (float)valid : INFINITY;
    if (cost) cost[(int64_t)h * Hl * Wl + pix] = cv;
    if (cv < best) {
      best = cv;
      best_d = d;
    }
  }
  depth[pix] = best_d;
}

}  // namespace

size_t cost_volume_ws_bytes(int K, int H, int W) {
  return (size_t)K * (H / 4) * (W / 4) * sizeof(float);
}

hipError_t launch_cost_volume(const float* keyframes, int K, int H, int W,
                              const gs_camera* cams_dev, float* cost, float* depth, void* ws,
                              hipStream_t s) {
  float* low = static_cast<float*>(ws);
  const int Hl = H / 4, Wl = W / 4;
  const int64_t nl = (int64_t)K * Hl * Wl;
  hipLaunchKernelGGL(luma_down4_kernel, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s,
                     keyframes, K, H, W, low);
  const int64_t np = (int64_t)Hl * Wl;
  hipLaunchKernelGGL(cost_wta_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, low, K,
                     Hl, Wl, cams_dev, cost, depth);
  return hipGetLastError();
}

}  // namespace gsmi
