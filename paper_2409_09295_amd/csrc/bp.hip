// gs_bp_labels: loopy min-sum belief propagation over the photometric cost
// volume (Sec. III-A2; Felzenszwalb and Huttenlocher's formulation) on the
// 4-connected grid with the truncated linear smoothness min(lam |l - l'|, trunc).
//
// The 64 depth hypotheses map onto the 64 lanes of a wavefront: one wavefront
// per pixel, one label per lane, so a pixel's data costs and messages are one
// 256-byte coalesced row each.  A message is the lower envelope of the
// sender's costs under the cone lam |l - l'|, computed as a prefix minimum of
// h(l) - lam l and a suffix minimum of h(l) + lam l across the lanes (six
// shuffle steps each) instead of the 64 x 64 minimum, then cut at
// min h + trunc and shifted to a zero minimum.  Iterations are synchronous
// (every message of an iteration from the previous iteration's), with two
// message buffers in turn.
#include "gs_internal.h"
#include "gs_nn.h"

namespace gsmi {

namespace {

constexpr int kL = 64;   // labels = hypotheses = lanes

__device__ __forceinline__ float wave_min(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = fminf(x, __shfl_xor(x, d, 64));
  return x;
}

// min over l of h(l) + min(lam |l - l'|, trunc) for l' = this lane, shifted
// so that its minimum over l' is 0.
__device__ __forceinline__ float send(float h, int lane, float lam, float trunc) {
  const float fl = (float)lane * lam;
  float a = h - fl, b = h + fl;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float up = __shfl_up(a, d, 64);
    const float dn = __shfl_down(b, d, 64);
    if (lane >= d) a = fminf(a, up);
    if (lane + d < 64) b = fminf(b, dn);
  }
  float r = fminf(a + fl, b - fl);
  r = fminf(r, wave_min(h) + trunc);
  return r - wave_min(r);
}

// D[p][l] from cost[l][p]; +inf (no valid view) becomes `invalid`.
__global__ __launch_bounds__(256) void bp_init_kernel(const float* __restrict__ cost, int64_t np,
                                                      float invalid, float* __restrict__ D) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np * kL) return;
  const int64_t p = i >> 6;
  const int l = (int)(i & 63);
  const float c = cost[(int64_t)l * np + p];
  D[i] = isfinite(c) ? c : invalid;
}

__global__ void zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// One synchronous iteration: min[k] are the messages each pixel received from
// its left (0), right (1), upper (2) and lower (3) neighbour; mout the next.
__global__ __launch_bounds__(256) void bp_iter_kernel(const float* __restrict__ D,
                                                      const float* __restrict__ min_,
                                                      float* __restrict__ mout, int H, int W,
                                                      float lam, float trunc) {
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t np = (int64_t)H * W;
  if (p >= np) return;
  const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
  const int64_t o = p * kL + lane;
  const int64_t plane = np * kL;
  const float a0 = min_[o], a1 = min_[plane + o], a2 = min_[2 * plane + o],
              a3 = min_[3 * plane + o];
  const float tot = D[o] + a0 + a1 + a2 + a3;
  if (x + 1 < W) mout[0 * plane + o + kL] = send(tot - a1, lane, lam, trunc);
  if (x > 0) mout[1 * plane + o - kL] = send(tot - a0, lane, lam, trunc);
  if (y + 1 < H) mout[2 * plane + o + (int64_t)W * kL] = send(tot - a3, lane, lam, trunc);
  if (y > 0) mout[3 * plane + o - (int64_t)W * kL] = send(tot - a2, lane, lam, trunc);
}

// Belief = data + the four incoming messages; label = its first minimum.
__global__ __launch_bounds__(256) void bp_label_kernel(const float* __restrict__ D,
                                                       const float* __restrict__ m, int64_t np,
                                                       int32_t* __restrict__ labels,
                                                       float* __restrict__ depth) {
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= np) return;
  const int64_t o = p * kL + lane;
  const int64_t plane = np * kL;
  const float b = D[o] + m[o] + m[plane + o] + m[2 * plane + o] + m[3 * plane + o];
  const float mn = wave_min(b);
  const uint64_t at = __ballot(b == mn);
  const int l = __builtin_ctzll(at);
  if (lane == 0) {
    if (labels) labels[p] = l;
    // the hypothesis depth exactly as the cost volume evaluates it
    if (depth) depth[p] = 0.25f + (25.0f - 0.25f) * (float)l / (float)(kL - 1);
  }
}

}  // namespace

size_t bp_ws_bytes(int h, int w) {
  const size_t np = (size_t)h * w;
  return (np * kL + 2 * 4 * np * kL) * sizeof(float);   // data costs + two message sets
}

hipError_t launch_bp(const float* cost, int h, int w, float lam, float trunc, int iters,
                     float invalid, int32_t* labels, float* depth, void* ws, hipStream_t s) {
  const int64_t np = (int64_t)h * w;
  float* D = static_cast<float*>(ws);
  float* mA = D + np * kL;
  float* mB = mA + 4 * np * kL;
  hipLaunchKernelGGL(bp_init_kernel, dim3((unsigned)((np * kL + 255) / 256)), dim3(256), 0, s,
                     cost, np, invalid, D);
  const int64_t nm = 2 * 4 * np * kL;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, mA, nm);
  const dim3 grid((unsigned)((np + 3) / 4));
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(bp_iter_kernel, grid, dim3(256), 0, s, D, mA, mB, h, w, lam, trunc);
    std::swap(mA, mB);
  }
  hipLaunchKernelGGL(bp_label_kernel, grid, dim3(256), 0, s, D, mA, np, labels, depth);
  return hipGetLastError();
}

}  // namespace gsmi
