// Map maintenance and the regulariser of the global mapping stage (Sec. III-B2):
//   gs_concat        insertion of the local map into the global map (the
//                    local part of any array may be replaced by a constant,
//                    e.g. the lowered insertion opacity or zero moments)
//   gs_prune_mask    the opacity rule of the pruning step
//   gs_compact       stable stream compaction of structure-of-arrays data
//   gs_iso_loss_grad the isotropic regulariser E_iso and its gradient
// All of them are elementwise or scan-shaped and bound by HBM bandwidth.
#include "gs_internal.h"

namespace gsmi {

namespace {

// ---------------------------------------------------------------------------
// concatenation: dst[k] = [a[k] | b[k]] per component, [C][n_a + n_b]
// ---------------------------------------------------------------------------

struct ConcatTable {
  const float* a[GS_SOA_MAX_ARRAYS];
  const float* b[GS_SOA_MAX_ARRAYS];
  float* dst[GS_SOA_MAX_ARRAYS];
  float fill[GS_SOA_MAX_ARRAYS];
  int64_t first[GS_SOA_MAX_ARRAYS + 1];   // first block of each array
  int32_t comps[GS_SOA_MAX_ARRAYS];
  int32_t count;
};

constexpr int kPerThread = 4;
constexpr int kBlockElems = 256 * kPerThread;

__global__ __launch_bounds__(256) void concat_kernel(ConcatTable T, int64_t na, int64_t nb) {
  const int64_t blk = blockIdx.x;
  int k = 0;
  for (int q = 1; q < T.count; ++q) k = (blk >= T.first[q]) ? q : k;
  const int64_t nd = na + nb;
  const int64_t total = (int64_t)T.comps[k] * nd;
  const int64_t e0 = (blk - T.first[k]) * kBlockElems + threadIdx.x;
  const float* __restrict__ a = T.a[k];
  const float* __restrict__ b = T.b[k];
  float* __restrict__ dst = T.dst[k];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t e = e0 + (int64_t)r * 256;
    if (e >= total) return;
    const int64_t c = e / nd, i = e - c * nd;
    dst[e] = i < na ? a[c * na + i] : (b ? b[c * nb + (i - na)] : T.fill[k]);
  }
}

// ---------------------------------------------------------------------------
// pruning mask and stable compaction
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void prune_mask_kernel(const float* __restrict__ ologit,
                                                         int64_t n, float min_logit,
                                                         uint8_t* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keep[i] = ologit[i] >= min_logit ? 1 : 0;
}

constexpr int kScanBlock = 1024;   // elements per scan block (256 threads x 4)

// Per-block count of kept elements.
__global__ __launch_bounds__(256) void keep_count_kernel(const uint8_t* __restrict__ keep,
                                                         int64_t n, uint32_t* __restrict__ part) {
  __shared__ uint32_t s_w[4];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    c += (i < n && keep[i]) ? 1u : 0u;
  }
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Exclusive scan of the per-block counts in one workgroup (sequential chunks
// per thread, then a scan of the chunk totals); the total goes to *n_kept.
__global__ __launch_bounds__(1024) void keep_scan_kernel(uint32_t* __restrict__ part,
                                                         int64_t nblocks,
                                                         uint32_t* __restrict__ n_kept) {
  __shared__ uint32_t s[1024];
  const int64_t per = (nblocks + 1023) / 1024;
  const int64_t lo = (int64_t)threadIdx.x * per, hi = min(nblocks, lo + per);
  uint32_t t = 0;
  for (int64_t i = lo; i < hi; ++i) t += part[i];
  s[threadIdx.x] = t;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {   // inclusive Hillis-Steele scan of the chunk totals
    const uint32_t x = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0u;
    __syncthreads();
    s[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - t;
  for (int64_t i = lo; i < hi; ++i) {
    const uint32_t c = part[i];
    part[i] = run;
    run += c;
  }
  if (threadIdx.x == 1023) *n_kept = s[1023];
}

// Destination position of every kept element (stable: ascending index).
__global__ __launch_bounds__(256) void keep_pos_kernel(const uint8_t* __restrict__ keep, int64_t n,
                                                       const uint32_t* __restrict__ part,
                                                       uint32_t* __restrict__ pos) {
  __shared__ uint32_t s_w[16];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  bool k[4];
  uint32_t mine = 0;
  // thread t owns elements base + 4 t .. base + 4 t + 3 (ascending with t)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = base + 4 * (int64_t)threadIdx.x + r;
    k[r] = i < n && keep[i];
    mine += k[r] ? 1u : 0u;
  }
  uint32_t incl = mine;   // inclusive scan over the wavefront
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t x = __shfl_up(incl, d, 64);
    if (lane >= d) incl += x;
  }
  if (lane == 63) s_w[w] = incl;
  __syncthreads();
  uint32_t off = part[blockIdx.x];
  for (int q = 0; q < w; ++q) off += s_w[q];
  uint32_t p = off + incl - mine;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = base + 4 * (int64_t)threadIdx.x + r;
    if (i < n) pos[i] = k[r] ? p : 0xFFFFFFFFu;
    p += k[r] ? 1u : 0u;
  }
}

struct CompactTable {
  const float* src[GS_SOA_MAX_ARRAYS];
  float* dst[GS_SOA_MAX_ARRAYS];
  int64_t first[GS_SOA_MAX_ARRAYS + 1];
  int32_t comps[GS_SOA_MAX_ARRAYS];
  int32_t count;
};

// dst[c][pos[i]] = src[c][i] for kept i; dst's component stride is the
// device count of kept elements.
__global__ __launch_bounds__(256) void compact_scatter_kernel(CompactTable T, int64_t n,
                                                              const uint32_t* __restrict__ pos,
                                                              const uint32_t* __restrict__ n_kept) {
  const int64_t blk = blockIdx.x;
  int k = 0;
  for (int q = 1; q < T.count; ++q) k = (blk >= T.first[q]) ? q : k;
  const int64_t total = (int64_t)T.comps[k] * n;
  const int64_t stride = (int64_t)*n_kept;
  const int64_t e0 = (blk - T.first[k]) * kBlockElems + threadIdx.x;
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t e = e0 + (int64_t)r * 256;
    if (e >= total) return;
    const int64_t c = e / n, i = e - c * n;
    const uint32_t p = pos[i];
    if (p != 0xFFFFFFFFu) T.dst[k][c * stride + p] = T.src[k][e];
  }
}

// ---------------------------------------------------------------------------
// isotropic regulariser
// ---------------------------------------------------------------------------

__device__ __forceinline__ float sgnf(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// E = coef * sum_i sum_j |s_ij - mean_k s_ik| with coef = weight / (3 n);
// dE/dlog s_ij = s_ij coef (sgn d_ij - mean_k sgn d_ik), accumulated into grad.
__global__ __launch_bounds__(256) void iso_kernel(const float* __restrict__ ls, int64_t n,
                                                  float coef, float* __restrict__ grad,
                                                  double* __restrict__ loss) {
  __shared__ float s_w[4];
  float acc = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float s0 = __expf(ls[i]), s1 = __expf(ls[n + i]), s2 = __expf(ls[2 * n + i]);
    // s_j - mean as a third of two differences: exactly 0 for equal scales
    // (an isotropic Gaussian gets no gradient), and no rounded mean to cancel
    const float d0 = ((s0 - s1) + (s0 - s2)) * (1.0f / 3.0f);
    const float d1 = ((s1 - s0) + (s1 - s2)) * (1.0f / 3.0f);
    const float d2 = ((s2 - s0) + (s2 - s1)) * (1.0f / 3.0f);
    acc += fabsf(d0) + fabsf(d1) + fabsf(d2);
    const float g0 = sgnf(d0), g1 = sgnf(d1), g2 = sgnf(d2);
    const float gm = (g0 + g1 + g2) * (1.0f / 3.0f);
    grad[i] += s0 * coef * (g0 - gm);
    grad[n + i] += s1 * coef * (g1 - gm);
    grad[2 * n + i] += s2 * coef * (g2 - gm);
  }
  if (!loss) return;
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicAdd(loss, (double)coef * ((double)s_w[0] + s_w[1] + s_w[2] + s_w[3]));
}

__global__ void zero_f64_kernel(double* p) { *p = 0.0; }

// ---------------------------------------------------------------------------
// pose update: Adam on the tangent, then T <- Exp(delta) T
// ---------------------------------------------------------------------------

// 4x4 exponential of the twist (rho, phi) in closed form (Rodrigues for the
// rotation, the left Jacobian for the translation), float64.
__device__ void se3_exp_d(const double xi[6], double R[9], double t[3]) {
  const double px = xi[3], py = xi[4], pz = xi[5];
  const double th2 = px * px + py * py + pz * pz, th = sqrt(th2);
  double A, B, C;   // R = I + A K + B K^2, V = I + B K + C K^2
  if (th < 1e-5) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  const double K[9] = {0.0, -pz, py, pz, 0.0, -px, -py, px, 0.0};
  double K2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
  double Vm[9];
  for (int i = 0; i < 9; ++i) {
    const double I = (i % 4 == 0) ? 1.0 : 0.0;
    R[i] = I + A * K[i] + B * K2[i];
    Vm[i] = I + B * K[i] + C * K2[i];
  }
  for (int r = 0; r < 3; ++r) t[r] = Vm[3 * r] * xi[0] + Vm[3 * r + 1] * xi[1] + Vm[3 * r + 2] * xi[2];
}

__global__ void pose_adam_kernel(gs_camera* __restrict__ cams, const float* __restrict__ g,
                                 float* __restrict__ m, float* __restrict__ v, int n_views,
                                 const uint8_t* __restrict__ view_mask, float lr_trans,
                                 float lr_rot, float b1, float b2, float eps,
                                 const int32_t* __restrict__ step_dev) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_views || (view_mask && view_mask[k] == 0)) return;
  const double t = (double)(*step_dev + 1);
  const double bc1 = 1.0 - pow((double)b1, t), bc2 = 1.0 - pow((double)b2, t);
  double d[6];
  for (int j = 0; j < 6; ++j) {
    const double gj = (double)g[6 * k + j];
    const double mj = (double)b1 * m[6 * k + j] + (1.0 - (double)b1) * gj;
    const double vj = (double)b2 * v[6 * k + j] + (1.0 - (double)b2) * gj * gj;
    m[6 * k + j] = (float)mj;
    v[6 * k + j] = (float)vj;
    const double lr = j < 3 ? (double)lr_trans : (double)lr_rot;
    d[j] = -lr * (mj / bc1) / (sqrt(vj / bc2) + (double)eps);
  }
  double E[9], e[3];
  se3_exp_d(d, E, e);
  gs_camera& c = cams[k];
  double R0[9], t0[3];
  for (int i = 0; i < 9; ++i) R0[i] = c.R[i];
  for (int i = 0; i < 3; ++i) t0[i] = c.t[i];
  for (int r = 0; r < 3; ++r) {
    for (int q = 0; q < 3; ++q)
      c.R[3 * r + q] = (float)(E[3 * r] * R0[q] + E[3 * r + 1] * R0[3 + q] + E[3 * r + 2] * R0[6 + q]);
    c.t[r] = (float)(E[3 * r] * t0[0] + E[3 * r + 1] * t0[1] + E[3 * r + 2] * t0[2] + e[r]);
  }
}

__global__ void step_commit_kernel(int32_t* step_dev) { *step_dev = *step_dev + 1; }

constexpr int64_t kIsoMaxBlocks = 1024;

}  // namespace

hipError_t launch_concat(const gs_concat_array* arrays, int n_arrays, int64_t na, int64_t nb,
                         hipStream_t s) {
  ConcatTable T{};
  T.count = n_arrays;
  int64_t blocks = 0;
  for (int k = 0; k < n_arrays; ++k) {
    T.a[k] = arrays[k].a;
    T.b[k] = arrays[k].b;
    T.dst[k] = arrays[k].dst;
    T.fill[k] = arrays[k].fill;
    T.comps[k] = arrays[k].components;
    T.first[k] = blocks;
    blocks += ((int64_t)arrays[k].components * (na + nb) + kBlockElems - 1) / kBlockElems;
  }
  T.first[n_arrays] = blocks;
  if (blocks > 0)
    hipLaunchKernelGGL(concat_kernel, dim3((unsigned)blocks), dim3(256), 0, s, T, na, nb);
  return hipGetLastError();
}

hipError_t launch_prune_mask(const float* ologit, int64_t n, float min_logit, uint8_t* keep,
                             hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(prune_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       ologit, n, min_logit, keep);
  return hipGetLastError();
}

size_t compact_ws_bytes(int64_t n) {
  const int64_t nblocks = std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
  const size_t a = ((size_t)nblocks * 4 + 255) & ~(size_t)255;
  const size_t b = ((size_t)std::max<int64_t>(n, 1) * 4 + 255) & ~(size_t)255;
  return a + b;
}

hipError_t launch_compact(const gs_compact_array* arrays, int n_arrays, int64_t n,
                          const uint8_t* keep, uint32_t* n_kept, void* ws, hipStream_t s) {
  const int64_t nblocks = std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
  uint32_t* part = static_cast<uint32_t*>(ws);
  uint32_t* pos = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) +
                                              (((size_t)nblocks * 4 + 255) & ~(size_t)255));
  hipLaunchKernelGGL(keep_count_kernel, dim3((unsigned)nblocks), dim3(256), 0, s, keep, n, part);
  hipLaunchKernelGGL(keep_scan_kernel, dim3(1), dim3(1024), 0, s, part, nblocks, n_kept);
  if (n == 0) return hipGetLastError();
  hipLaunchKernelGGL(keep_pos_kernel, dim3((unsigned)nblocks), dim3(256), 0, s, keep, n, part, pos);
  CompactTable T{};
  T.count = n_arrays;
  int64_t blocks = 0;
  for (int k = 0; k < n_arrays; ++k) {
    T.src[k] = arrays[k].src;
    T.dst[k] = arrays[k].dst;
    T.comps[k] = arrays[k].components;
    T.first[k] = blocks;
    blocks += ((int64_t)arrays[k].components * n + kBlockElems - 1) / kBlockElems;
  }
  T.first[n_arrays] = blocks;
  if (blocks > 0)
    hipLaunchKernelGGL(compact_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, s, T, n, pos,
                       n_kept);
  return hipGetLastError();
}

hipError_t launch_pose_adam(gs_camera* cams_dev, const float* grad_xi, float* m, float* v,
                            int n_views, const uint8_t* view_mask, float lr_trans, float lr_rot,
                            float beta1, float beta2, float eps, int32_t* step_dev,
                            hipStream_t s) {
  hipLaunchKernelGGL(pose_adam_kernel, dim3(1), dim3(64), 0, s, cams_dev, grad_xi, m, v, n_views,
                     view_mask, lr_trans, lr_rot, beta1, beta2, eps, step_dev);
  hipLaunchKernelGGL(step_commit_kernel, dim3(1), dim3(1), 0, s, step_dev);
  return hipGetLastError();
}

hipError_t launch_iso_loss_grad(const float* log_scales, int64_t n, float weight,
                                float* grad_log_scales, double* loss, hipStream_t s) {
  if (loss) hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(1), 0, s, loss);
  if (n > 0) {
    const float coef = (float)((double)weight / (3.0 * (double)n));
    const int64_t blocks = std::min<int64_t>(kIsoMaxBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(iso_kernel, dim3((unsigned)blocks), dim3(256), 0, s, log_scales, n, coef,
                       grad_log_scales, loss);
  }
  return hipGetLastError();
}

}  // namespace gsmi
