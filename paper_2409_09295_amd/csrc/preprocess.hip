// gs_preprocess: project every Gaussian into every view of a batch.
//
// One lane per (Gaussian, group of kViewsPerLane views).  The Gaussian's
// parameters are read with coalesced component-major loads (lane i reads
// element i of each component array) and reused for every view of the group,
// so a batch of V views costs ceil(V / kViewsPerLane) reads of the map
// plus, per view, 48 bytes written for a visible splat
// (44 without tile counts) and 8 for a culled one (4); splitting
// the views over grid.y keeps enough wavefronts in flight to hide the long
// per-view dependency chain.  Camera records are wave-uniform.
#include "project.h"

namespace gsmi {

// 16 rather than 32: the grid then holds twice as many, half as long
// wavefronts, so the last ones do not run alone in a second round
// (3,125 wavefronts of 32 views against 3,072 resident at 200k Gaussians).
constexpr int kViewsPerLane = 16;

template <int DEG>
__global__ __launch_bounds__(256) void preprocess_kernel(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ ologit,
    const float* __restrict__ sh, int64_t n, const gs_camera* __restrict__ cams, int n_views,
    float2* __restrict__ xy, float4* __restrict__ co, float4* __restrict__ rd,
    int32_t* __restrict__ radius, uint32_t* __restrict__ tiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  GaussState G;
  load_gauss(means, log_scales, quats, ologit, n, i, G);
  SHCoef<DEG> C;
  load_sh<DEG>(sh, n, i, C);
  const int v0 = blockIdx.y * kViewsPerLane;
  const int v1 = min(n_views, v0 + kViewsPerLane);
  for (int v = v0; v < v1; ++v) {
    const gs_camera cam = cams[v];
    ViewState S;
    project_view<DEG>(G, cam, C, S);
    const int64_t o = (int64_t)v * n + i;
    if (S.visible) {
      xy[o] = make_float2(S.u, S.v);
      co[o] = make_float4(S.q0, S.q1, S.q2, G.o);
      rd[o] = make_float4(S.rgb[0], S.rgb[1], S.rgb[2], S.p[2]);
      radius[o] = S.radius;
      if (tiles) {   // tiles of the rectangle, as the binning counts them
        Rect rc;
        const bool ok = tile_rect(S.u, S.v, S.radius, cam.width, cam.height, rc);
        tiles[o] = ok ? (uint32_t)((rc.x1 - rc.x0) * (rc.y1 - rc.y0)) : 0u;
      }
    } else {
      radius[o] = 0;   // the other fields of a culled entry are never read
      if (tiles) tiles[o] = 0u;
    }
  }
}

hipError_t launch_preprocess(const gs_gaussians& g, const gs_camera* cams_dev, int n_views,
                             const gs_projected& out, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const dim3 block(256);
  const dim3 grid((unsigned)((g.n + 255) / 256), (unsigned)((n_views + kViewsPerLane - 1) / kViewsPerLane));
  auto* xy = reinterpret_cast<float2*>(out.xy);
  auto* co = reinterpret_cast<float4*>(out.conic_opacity);
  auto* rd = reinterpret_cast<float4*>(out.rgb_depth);
  kernel_event_start(GS_KERNEL_PREPROCESS, s);
  switch (g.sh_degree) {
    case 0:
      hipLaunchKernelGGL(preprocess_kernel<0>, grid, block, 0, s, g.means, g.log_scales, g.quats,
                         g.opacity_logits, g.sh, g.n, cams_dev, n_views, xy, co, rd, out.radius,
                         out.tiles);
      break;
    case 1:
      hipLaunchKernelGGL(preprocess_kernel<1>, grid, block, 0, s, g.means, g.log_scales, g.quats,
                         g.opacity_logits, g.sh, g.n, cams_dev, n_views, xy, co, rd, out.radius,
                         out.tiles);
      break;
    case 2:
      hipLaunchKernelGGL(preprocess_kernel<2>, grid, block, 0, s, g.means, g.log_scales, g.quats,
                         g.opacity_logits, g.sh, g.n, cams_dev, n_views, xy, co, rd, out.radius,
                         out.tiles);
      break;
    default:
      hipLaunchKernelGGL(preprocess_kernel<3>, grid, block, 0, s, g.means, g.log_scales, g.quats,
                         g.opacity_logits, g.sh, g.n, cams_dev, n_views, xy, co, rd, out.radius,
                         out.tiles);
      break;
  }
  kernel_event_stop(GS_KERNEL_PREPROCESS, s);
  return hipGetLastError();
}

}  // namespace gsmi
