// gs_adam_step and gs_l1_loss_grad: elementwise, HBM-bound kernels.
//
// Adam streams p, g, m, v once (16 B read, 12 B written per parameter) with
// 16-byte vector accesses when the four arrays are 16-byte aligned.
#include "gs_internal.h"

namespace gsmi {

namespace {

struct AdamCoef {
  float lr, b1, b2, eps, inv_bc1, inv_bc2;
};

// Written with explicit fused multiply-adds so that every kernel that uses
// it rounds identically, whatever contraction the compiler would choose.
__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, const AdamCoef& c) {
  m = __builtin_fmaf(c.b1, m, (1.0f - c.b1) * g);
  v = __builtin_fmaf(c.b2, v, ((1.0f - c.b2) * g) * g);
  const float mhat = m * c.inv_bc1;
  const float vhat = v * c.inv_bc2;
  const float step = mhat / (__builtin_sqrtf(vhat) + c.eps);
  p = __builtin_fmaf(-c.lr, step, p);
}

__global__ __launch_bounds__(256) void adam_vec4_kernel(float4* __restrict__ p,
                                                        const float4* __restrict__ g,
                                                        float4* __restrict__ m,
                                                        float4* __restrict__ v, int64_t n4,
                                                        AdamCoef c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  float4 pp = p[i], gg = g[i], mm = m[i], vv = v[i];
  adam_one(pp.x, gg.x, mm.x, vv.x, c);
  adam_one(pp.y, gg.y, mm.y, vv.y, c);
  adam_one(pp.z, gg.z, mm.z, vv.z, c);
  adam_one(pp.w, gg.w, mm.w, vv.w, c);
  p[i] = pp;
  m[i] = mm;
  v[i] = vv;
}

__global__ __launch_bounds__(256) void adam_scalar_kernel(float* __restrict__ p,
                                                          const float* __restrict__ g,
                                                          float* __restrict__ m,
                                                          float* __restrict__ v, int64_t begin,
                                                          int64_t n, const uint8_t* __restrict__ mask,
                                                          AdamCoef c) {
  const int64_t i = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (mask && mask[i] == 0) return;
  float pp = p[i], mm = m[i], vv = v[i];
  adam_one(pp, g[i], mm, vv, c);
  p[i] = pp;
  m[i] = mm;
  v[i] = vv;
}

// Device-step variant: coefficients derived in-kernel from *step_dev.
__device__ __forceinline__ bool dev_coef(const int32_t* step_dev, const uint32_t* guard,
                                         int64_t guard_cap, float lr, float b1, float b2,
                                         float eps, AdamCoef& c) {
  if (guard && (int64_t)(*guard) > guard_cap) return false;
  const float t = (float)(*step_dev + 1);
  c.lr = lr;
  c.b1 = b1;
  c.b2 = b2;
  c.eps = eps;
  // 1 - b^t = -expm1(t log1p(b - 1)): b - 1 is exact in float32, and this form
  // avoids the cancellation of 1 - powf(b, t), which for b2 = 0.999 and small
  // t loses about five of float32's digits
  c.inv_bc1 = -1.0f / expm1f(t * log1pf(b1 - 1.0f));
  c.inv_bc2 = -1.0f / expm1f(t * log1pf(b2 - 1.0f));
  return true;
}

__global__ __launch_bounds__(256) void adam_dev_kernel(float* __restrict__ p,
                                                       const float* __restrict__ g,
                                                       float* __restrict__ m,
                                                       float* __restrict__ v, int64_t n,
                                                       const uint8_t* __restrict__ mask, float lr,
                                                       float b1, float b2, float eps,
                                                       const int32_t* __restrict__ step_dev,
                                                       const uint32_t* __restrict__ guard,
                                                       int64_t guard_cap) {
  AdamCoef c;
  if (!dev_coef(step_dev, guard, guard_cap, lr, b1, b2, eps, c)) return;
  const int64_t i4 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = i4 + k;
    if (i >= n) return;
    if (mask && mask[i] == 0) continue;
    float pp = p[i], mm = m[i], vv = v[i];
    adam_one(pp, g[i], mm, vv, c);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

// All groups in one grid: group k owns blocks [first[k], first[k + 1]), each
// thread updates four consecutive parameters (one 16-byte access per array
// when the group's arrays are 16-byte aligned).
struct AdamGroups {
  float* p[GS_ADAM_MAX_GROUPS];
  const float* g[GS_ADAM_MAX_GROUPS];
  float* m[GS_ADAM_MAX_GROUPS];
  float* v[GS_ADAM_MAX_GROUPS];
  int64_t n[GS_ADAM_MAX_GROUPS];
  float lr[GS_ADAM_MAX_GROUPS];
  int32_t vec[GS_ADAM_MAX_GROUPS];
  int64_t first[GS_ADAM_MAX_GROUPS + 1];
  int32_t count;
  // optional per-Gaussian mask: element e of a group ([C][n_gauss] layout)
  // belongs to Gaussian e % n_gauss and is updated only if its byte is nonzero
  const uint8_t* gmask;
  int64_t n_gauss;
};

__global__ __launch_bounds__(256) void adam_groups_kernel(AdamGroups G, float b1, float b2,
                                                          float eps,
                                                          const int32_t* __restrict__ step_dev,
                                                          const uint32_t* __restrict__ guard,
                                                          int64_t guard_cap) {
  const int64_t b = blockIdx.x;
  int k = 0;
  for (int q = 1; q < G.count; ++q) k = (b >= G.first[q]) ? q : k;
  AdamCoef c;
  if (!dev_coef(step_dev, guard, guard_cap, G.lr[k], b1, b2, eps, c)) return;
  const int64_t i4 = ((b - G.first[k]) * blockDim.x + threadIdx.x) * 4;
  const int64_t n = G.n[k];
  if (i4 >= n) return;
  float* __restrict__ p = G.p[k];
  const float* __restrict__ g = G.g[k];
  float* __restrict__ m = G.m[k];
  float* __restrict__ v = G.v[k];
  const uint8_t* __restrict__ gm = G.gmask;
  uint32_t on = 0xFu;   // bit j: element i4 + j is updated
  if (gm) {
    int64_t r = i4 % G.n_gauss;
    on = 0u;
    for (int j = 0; j < 4; ++j) {
      on |= (uint32_t)(gm[r] != 0) << j;
      if (++r == G.n_gauss) r = 0;
    }
    if (on == 0u) return;
  }
  if (G.vec[k] && i4 + 4 <= n && on == 0xFu) {
    float4 pp = *reinterpret_cast<float4*>(p + i4);
    const float4 gg = *reinterpret_cast<const float4*>(g + i4);
    float4 mm = *reinterpret_cast<float4*>(m + i4);
    float4 vv = *reinterpret_cast<float4*>(v + i4);
    adam_one(pp.x, gg.x, mm.x, vv.x, c);
    adam_one(pp.y, gg.y, mm.y, vv.y, c);
    adam_one(pp.z, gg.z, mm.z, vv.z, c);
    adam_one(pp.w, gg.w, mm.w, vv.w, c);
    *reinterpret_cast<float4*>(p + i4) = pp;
    *reinterpret_cast<float4*>(m + i4) = mm;
    *reinterpret_cast<float4*>(v + i4) = vv;
    return;
  }
  for (int64_t i = i4; i < min(n, i4 + 4); ++i) {
    if (!((on >> (i - i4)) & 1u)) continue;
    float pp = p[i], mm = m[i], vv = v[i];
    adam_one(pp, g[i], mm, vv, c);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
  }
}

__global__ void adam_commit_kernel(int32_t* __restrict__ step_dev,
                                   const uint32_t* __restrict__ guard, int64_t guard_cap) {
  if (guard && (int64_t)(*guard) > guard_cap) return;
  *step_dev = *step_dev + 1;
}

// Grid-stride over one view per blockIdx.y with a bounded number of blocks,
// so the loss needs at most kL1Blocks float64 atomics per view.
constexpr int kL1Blocks = 128;

__global__ __launch_bounds__(256) void l1_grad_kernel(const float* __restrict__ image,
                                                      const float* __restrict__ target,
                                                      ViewTable vt, float* __restrict__ grad,
                                                      double* __restrict__ loss) {
  __shared__ float s_wave[4];
  const int v = blockIdx.y;
  const ViewInfo& vi = vt.v[v];
  const int64_t count = 3 * (int64_t)vi.width * vi.height;
  const float inv = 1.0f / (float)count;
  const int64_t base = 3 * vi.pix_base;
  float a = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = image[base + i] - target[base + i];
    grad[base + i] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
    a += fabsf(d);
  }
  if (loss == nullptr) return;
  for (int d = 32; d > 0; d >>= 1) a += __shfl_xor(a, d, 64);
  if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double sum = (double)s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    atomicAdd(loss, sum / (double)count);
  }
}

__global__ void zero_f64_kernel(double* p) { *p = 0.0; }

}  // namespace

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int32_t step, const uint8_t* mask,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  AdamCoef c;
  c.lr = lr;
  c.b1 = beta1;
  c.b2 = beta2;
  c.eps = eps;
  c.inv_bc1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
  c.inv_bc2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
  const bool aligned = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(g) |
                         reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15) == 0;
  int64_t begin = 0;
  if (aligned && mask == nullptr) {
    const int64_t n4 = n / 4;
    if (n4 > 0)
      hipLaunchKernelGGL(adam_vec4_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                         reinterpret_cast<float4*>(p), reinterpret_cast<const float4*>(g),
                         reinterpret_cast<float4*>(m), reinterpret_cast<float4*>(v), n4, c);
    begin = n4 * 4;
  }
  if (begin < n)
    hipLaunchKernelGGL(adam_scalar_kernel, dim3((unsigned)((n - begin + 255) / 256)), dim3(256), 0,
                       s, p, g, m, v, begin, n, mask, c);
  return hipGetLastError();
}

hipError_t launch_adam_dev(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float beta1, float beta2, float eps, int32_t* step_dev, int32_t commit,
                           const uint8_t* mask, const uint32_t* guard_n_keys,
                           int64_t guard_capacity, hipStream_t s) {
  if (n > 0) {
    const int64_t threads = (n + 3) / 4;
    hipLaunchKernelGGL(adam_dev_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       p, g, m, v, n, mask, lr, beta1, beta2, eps, step_dev, guard_n_keys,
                       guard_capacity);
  }
  if (commit)
    hipLaunchKernelGGL(adam_commit_kernel, dim3(1), dim3(1), 0, s, step_dev, guard_n_keys,
                       guard_capacity);
  return hipGetLastError();
}

hipError_t launch_adam_groups(const gs_adam_group* groups, int n_groups, float beta1,
                              float beta2, float eps, int32_t* step_dev,
                              const uint32_t* guard_n_keys, int64_t guard_capacity,
                              hipStream_t s, const uint8_t* gauss_mask, int64_t n_gauss) {
  AdamGroups G{};
  G.count = n_groups;
  G.gmask = gauss_mask;
  G.n_gauss = gauss_mask ? n_gauss : 1;
  int64_t blocks = 0;
  for (int k = 0; k < n_groups; ++k) {
    const gs_adam_group& q = groups[k];
    G.p[k] = q.p;
    G.g[k] = q.g;
    G.m[k] = q.m;
    G.v[k] = q.v;
    G.n[k] = q.n;
    G.lr[k] = q.lr;
    G.vec[k] = ((reinterpret_cast<uintptr_t>(q.p) | reinterpret_cast<uintptr_t>(q.g) |
                 reinterpret_cast<uintptr_t>(q.m) | reinterpret_cast<uintptr_t>(q.v)) & 15) == 0;
    G.first[k] = blocks;
    blocks += (q.n + 1023) / 1024;
  }
  G.first[n_groups] = blocks;
  if (blocks > 0)
    hipLaunchKernelGGL(adam_groups_kernel, dim3((unsigned)blocks), dim3(256), 0, s, G, beta1,
                       beta2, eps, step_dev, guard_n_keys, guard_capacity);
  hipLaunchKernelGGL(adam_commit_kernel, dim3(1), dim3(1), 0, s, step_dev, guard_n_keys,
                     guard_capacity);
  return hipGetLastError();
}

hipError_t launch_l1_loss_grad(const float* image, const float* target, const ViewTable& vt,
                               float* dL_dimage, double* loss, hipStream_t s) {
  int64_t max_count = 0;
  for (int v = 0; v < vt.n_views; ++v)
    max_count = std::max<int64_t>(max_count, 3 * (int64_t)vt.v[v].width * vt.v[v].height);
  if (loss) hipLaunchKernelGGL(zero_f64_kernel, dim3(1), dim3(1), 0, s, loss);
  const int64_t blocks = std::min<int64_t>(kL1Blocks, (max_count + 255) / 256);
  hipLaunchKernelGGL(l1_grad_kernel, dim3((unsigned)blocks, vt.n_views), dim3(256), 0, s, image,
                     target, vt, dL_dimage, loss);
  return hipGetLastError();
}

}  // namespace gsmi
