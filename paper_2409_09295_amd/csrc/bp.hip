// gs_bp_labels: loopy min-sum belief propagation over the photometric cost
// volume (Sec. III-A2; Felzenszwalb and Huttenlocher's formulation) on the
// 4-connected grid with the truncated linear smoothness min(lam |l - l'|, trunc).
//
// The 64 depth hypotheses map onto the 64 lanes of a wavefront: one wavefront
// per pixel, one label per lane, so a pixel's data costs and messages are one
// 256-byte coalesced row each.  A message is the lower envelope of the
// sender's costs under the cone lam |l - l'|, computed as a prefix minimum of
// h(l) - lam l and a suffix minimum of h(l) + lam l across the lanes (DPP row
// shifts and broadcasts, no LDS round trips) instead of the 64 x 64 minimum,
// then cut at min h + trunc and shifted to a zero minimum.  Iterations are synchronous
// (every message of an iteration from the previous iteration's), with two
// message buffers in turn.
#include "gs_internal.h"
#include "gs_nn.h"

namespace gsmi {

namespace {

constexpr int kL = 64;   // labels = hypotheses = lanes

// x of another lane by DPP; lanes whose source lies outside the pattern
// keep +inf (the identity of min)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_or_inf(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(INFINITY), __float_as_int(x), CTRL,
                                                    ROW_MASK, 0xf, false));
}

// Minimum over the 64 lanes, in every lane: DPP within the 16-lane rows,
// then the four row minima.
__device__ __forceinline__ float wave_min(float x) {
  x = fminf(x, dpp_or_inf<0xb1, 0xf>(x));    // quad_perm [1,0,3,2]
  x = fminf(x, dpp_or_inf<0x4e, 0xf>(x));    // quad_perm [2,3,0,1]
  x = fminf(x, dpp_or_inf<0x124, 0xf>(x));   // row_ror:4
  x = fminf(x, dpp_or_inf<0x128, 0xf>(x));   // row_ror:8: every lane holds its row minimum
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
  return fminf(fminf(r0, r1), fminf(r2, r3));
}

// Inclusive minimum over lanes 0 .. lane (Hillis-Steele within the rows by
// row shifts, then the previous rows' minima by row broadcasts).
__device__ __forceinline__ float prefix_min(float x) {
  x = fminf(x, dpp_or_inf<0x111, 0xf>(x));   // row_shr:1
  x = fminf(x, dpp_or_inf<0x112, 0xf>(x));   // row_shr:2
  x = fminf(x, dpp_or_inf<0x114, 0xf>(x));   // row_shr:4
  x = fminf(x, dpp_or_inf<0x118, 0xf>(x));   // row_shr:8
  x = fminf(x, dpp_or_inf<0x142, 0xa>(x));   // row_bcast:15 into rows 1 and 3
  x = fminf(x, dpp_or_inf<0x143, 0xc>(x));   // row_bcast:31 into rows 2 and 3
  return x;
}

// Inclusive minimum over lanes lane .. 63: row shifts the other way, then
// the later rows' minima (each row's first lane holds its row minimum).
__device__ __forceinline__ float suffix_min(float x, int lane) {
  x = fminf(x, dpp_or_inf<0x101, 0xf>(x));   // row_shl:1
  x = fminf(x, dpp_or_inf<0x102, 0xf>(x));   // row_shl:2
  x = fminf(x, dpp_or_inf<0x104, 0xf>(x));   // row_shl:4
  x = fminf(x, dpp_or_inf<0x108, 0xf>(x));   // row_shl:8
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
  const float s2 = r3, s1 = fminf(r2, r3), s0 = fminf(r1, s1);
  const int row = lane >> 4;
  const float later = row == 0 ? s0 : row == 1 ? s1 : row == 2 ? s2 : INFINITY;
  return fminf(x, later);
}

// min over l of h(l) + min(lam |l - l'|, trunc) for l' = this lane, shifted
// so that its minimum over l' is 0.
__device__ __forceinline__ float send(float h, int lane, float lam, float trunc) {
  const float fl = (float)lane * lam;
  const float a = prefix_min(h - fl);
  const float b = suffix_min(h + fl, lane);
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
