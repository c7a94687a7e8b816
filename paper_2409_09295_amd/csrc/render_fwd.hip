// gs_render_fwd: front-to-back compositing, one workgroup per 16x16 tile of
// any view in the batch (a single grid spans all views).
//
// A workgroup of 256 / PPL threads covers the tile, each lane owning PPL
// pixels (PPL = 1, 2 or 4, chosen by the tuner): tile-local pixel
// i = k * (256 / PPL) + thread maps to quadrant i / 64 and position i % 64
// inside it, so with PPL = 1 each wavefront owns one 8x8 quadrant and with
// PPL = 4 one wavefront owns the tile, every lane holding the same position
// in the four quadrants.  The tile's sorted splats are staged in LDS 256 at
// a time (128 with PPL = 4; gathered once per workgroup) and read back as
// wave-uniform broadcasts, so a staged record serves 64 * PPL pixels per LDS
// read.  A workgroup stops once every pixel has terminated.
#include <mutex>

#include "gs_internal.h"

namespace gsmi {

// Per-tile loss shares of gs_render_fwd_l1_noalloc: a library-owned device
// array instead of a caller workspace.  Every GPU holds its own copy until
// the process ends; host code reaches it only through the per-device address
// taken by noalloc_scratch().
static __device__ __align__(256) float scratch[GS_NOALLOC_MAX_TILES];

namespace {

// L1: also the photometric L1 gradient against `target` and the tile's
// share of the loss (written to tile_loss[tile]).  The fused pass at one
// wavefront per tile is held to 72 VGPRs, seven wavefronts per SIMD (from
// 74 and six; measured 3.5% faster, no spills; the other instances spill at
// that bound and keep the compiler's choice).  SPL: splats each thread
// stages per LDS batch (1 or 2).
template <int PPL, int SPL, bool L1, bool Q>
__global__ __launch_bounds__(kBlock / PPL, PPL == 4 && SPL == 1 && L1 && !Q ? 7 : 1) void render_fwd_kernel(
    ViewTable vt, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ values,
    const uint32_t* __restrict__ order,
    const float2* __restrict__ xy, const float4* __restrict__ co, const float4* __restrict__ rd,
    float3 bg, float* __restrict__ image, float* __restrict__ final_T,
    uint32_t* __restrict__ n_contrib, float* __restrict__ depth_out,
    const float* __restrict__ target, float* __restrict__ dL, float* __restrict__ tile_loss,
    uint32_t* __restrict__ counter) {
  constexpr int NT = kBlock / PPL;
  // splats staged per batch (a smaller batch takes less LDS per workgroup,
  // and a tile whose pixels all terminate early stages fewer splats it
  // never walks)
  constexpr int kStage = SPL * NT;
  constexpr int kPerThread = kStage / NT;
  constexpr int kWords = kStage / 64;
  __shared__ StagedSplat s_splat[kStage];
  // s_reach[q][w] bit b: staged splat 64 w + b can reach quadrant q
  __shared__ uint64_t s_reach[4][kWords];
  __shared__ uint32_t s_slot;
  // slot i: tile order[i] (longest lists first) when the binning produced
  // an order; one slot per workgroup, or (Q) slots drawn from `counter`
  for (uint32_t slot = blockIdx.x;;) {
    if constexpr (Q) slot = next_slot(counter, (uint32_t)vt.n_tiles, &s_slot);
    if (slot >= (uint32_t)vt.n_tiles) break;
    const int tile = order ? (int)order[slot] : (int)slot;
    const int v = find_view(vt, tile);
    const ViewInfo& vi = vt.v[v];
    const int lt = tile - vi.tile_base;
    const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
    const int lane = threadIdx.x & 63;

    // pixel k of a lane lies in column k % NC: with 2 pixels per lane both
    // share their x, with 4 the even and the odd ones do
    constexpr int NC = PPL == 4 ? 2 : 1;
    int px[PPL], py[PPL];
    uint32_t qbit[PPL];   // quadrant bit of each of the lane's pixels (wave-uniform)
    // T > 0: transmittance of a live pixel; T < 0: the pixel has terminated
    // (or lies outside the image) and -T is its final transmittance
    float fpx[PPL], fpy[PPL], T[PPL], C0[PPL], C1[PPL], C2[PPL], D[PPL];
    uint32_t last[PPL];
    bool inside[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int i = k * NT + (int)threadIdx.x;
      const int q = i >> 6, l = i & 63;
      px[k] = tx * kTile + (q & 1) * 8 + (l & 7);
      py[k] = ty * kTile + (q >> 1) * 8 + (l >> 3);
      qbit[k] = __builtin_amdgcn_readfirstlane(1u << q);
      inside[k] = px[k] < vi.width && py[k] < vi.height;
      fpx[k] = (float)px[k] + 0.5f;
      fpy[k] = (float)py[k] + 0.5f;
      T[k] = inside[k] ? 1.0f : -1.0f;
      C0[k] = C1[k] = C2[k] = D[k] = 0.0f;
      last[k] = 0;
    }

    const uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
    for (int64_t b = s; b < (int64_t)e; b += kStage) {
      bool all_done = true;
#pragma unroll
      for (int k = 0; k < PPL; ++k) all_done = all_done && !(T[k] > 0.0f);
      if (__syncthreads_count(all_done ? 0 : 1) == 0) break;
#pragma unroll
      for (int r = 0; r < kPerThread; ++r) {
        const int slot = r * NT + (int)threadIdx.x;
        const int64_t idx = b + slot;
        uint32_t reach = 0;
        if (idx < (int64_t)e)
          reach = stage_splat(values[idx], xy, co, rd, tx * kTile, ty * kTile, vi.width,
                              vi.height, s_splat[slot]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint64_t bq = __ballot((reach >> q) & 1u);
          if (lane == 0) s_reach[q][slot >> 6] = bq;
        }
      }
      __syncthreads();
      // Walk, in list order, only the staged splats that reach one of this
      // wave's quadrants; stop once every pixel of the wave has terminated.
      if (__all(all_done)) continue;
      for (int w = 0; w < kWords; ++w) {
        uint64_t m = 0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) m |= s_reach[__builtin_ctz(qbit[k])][w];
        m = uniform_u64(m);
        while (m) {
          const int j = 64 * w + __builtin_ctzll(m);
          m &= m - 1;
          const float4 geo = s_splat[j].geo;
          const float4 app = s_splat[j].app;
          const float4 ext = s_splat[j].ext;
          const uint32_t reach = PPL > 1 ? __builtin_amdgcn_readfirstlane(__float_as_uint(ext.y)) : ~0u;
          ColumnTerms ct[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) ct[c] = column_terms(geo, fpx[c]);
#pragma unroll
          for (int k = 0; k < PPL; ++k) {
            if (!(reach & qbit[k])) continue;   // slot-uniform
            float alpha, raw, G, dy;
            const bool ok = eval_alpha_at<false>(ct[k % NC], geo, app, fpy[k], alpha, raw, G, dy);
            // a terminated pixel (T < 0) gets Tn <= 0 < kTMin: it never blends again
            const float Tn = __builtin_fmaf(-T[k], alpha, T[k]);   // T (1 - alpha), one rounding
            const bool term = ok && Tn < kTMin;   // stops before this splat
            if (term) T[k] = -fabsf(T[k]);
            if (!ok || term) continue;
            const float wgt = alpha * T[k];
            C0[k] += app.z * wgt;
            C1[k] += app.w * wgt;
            C2[k] += ext.x * wgt;
            D[k] += ext.z * wgt;
            T[k] = Tn;
            last[k] = (uint32_t)(b - (int64_t)s) + (uint32_t)j + 1;
          }
          // every pixel of the wave has terminated: stop.  Tested after every
          // fourth splat only (a terminated pixel never blends again, so a
          // late test changes nothing; measured 2.4% faster than every splat)
          if ((__popcll(m) & 3) == 0) {
            bool live = false;
#pragma unroll
            for (int k = 0; k < PPL; ++k) live = live || __float_as_int(T[k]) > 0;
            if (!__any(live)) m = 0;
          }
        }
      }
    }
    const int64_t plane = (int64_t)vi.width * vi.height;
    float* img = image + 3 * vi.pix_base;
    // L1 against the target, as gs_l1_loss_grad computes it from the image
    const float inv = 1.0f / (float)(3 * plane);
    float lsum = 0.0f;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      if (!inside[k]) continue;
      const int64_t off = (int64_t)py[k] * vi.width + px[k];
      const float Tf = fabsf(T[k]);
      const float c[3] = {C0[k] + Tf * bg.x, C1[k] + Tf * bg.y, C2[k] + Tf * bg.z};
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) img[ch * plane + off] = c[ch];
      final_T[vi.pix_base + off] = Tf;
      n_contrib[vi.pix_base + off] = last[k];
      if (!L1 && depth_out) depth_out[vi.pix_base + off] = D[k];
      if (L1) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          const int64_t o = 3 * vi.pix_base + ch * plane + off;
          const float d = c[ch] - target[o];
          dL[o] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
          lsum += fabsf(d);
        }
      }
    }
    if (L1) {
      __shared__ float s_l[kBlock / 64];
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) lsum += __shfl_xor(lsum, d, 64);
      if ((threadIdx.x & 63) == 0) s_l[threadIdx.x >> 6] = lsum;
      __syncthreads();
      if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < NT / 64; ++w) t += s_l[w];
        tile_loss[tile] = t * inv;
      }
    }
    if constexpr (!Q) break;
  }
}

// Loss = sum of the per-tile shares, in float64 and a fixed order.
__global__ __launch_bounds__(1024) void tile_loss_sum_kernel(const float* __restrict__ tile_loss,
                                                             int n_tiles,
                                                             double* __restrict__ loss) {
  __shared__ double s_acc[1024];
  double a = 0.0;
  // lane t sums tiles t, t + 1024, t + 2048, ... in that order; eight loads
  // in flight per round trip
  for (int t0 = threadIdx.x; t0 < n_tiles; t0 += 8 * 1024) {
    float x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {   // in-bounds loads without a branch, masked after
      const int t = t0 + u * 1024;
      x[u] = tile_loss[min(t, n_tiles - 1)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = t0 + u * 1024 < n_tiles ? x[u] : 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) a += (double)x[u];
  }
  s_acc[threadIdx.x] = a;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_acc[threadIdx.x] += s_acc[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = s_acc[0];
}

}  // namespace

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {   // once per device, with that device current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

namespace {
template <int P, int S, bool L>
void launch_fwd(int schedule, const gs_bins& bins, const ViewTable& vt, const float2* xy,
                const float4* co, const float4* rd, float3 bg, float* image, float* final_T,
                uint32_t* n_contrib, float* depth, const float* target, float* dL,
                float* tile_loss, hipStream_t s) {
  const int resident = schedule >= GS_SCHEDULE_PERSISTENT
                           ? resident_workgroups((const void*)render_fwd_kernel<P, S, L, true>,
                                                 kBlock / P)
                           : 0;
  const TileSchedule sc = tile_schedule(schedule, bins, GS_QUEUE_FWD, vt.n_tiles, resident);
  if (sc.counter)
    hipLaunchKernelGGL((render_fwd_kernel<P, S, L, true>), dim3(sc.grid), dim3(kBlock / P), 0, s, vt,
                       bins.ranges, bins.values, sc.order, xy, co, rd, bg, image, final_T,
                       n_contrib, depth, target, dL, tile_loss, sc.counter);
  else
    hipLaunchKernelGGL((render_fwd_kernel<P, S, L, false>), dim3(sc.grid), dim3(kBlock / P), 0, s,
                       vt, bins.ranges, bins.values, sc.order, xy, co, rd, bg, image, final_T,
                       n_contrib, depth, target, dL, tile_loss, nullptr);
}
}  // namespace

hipError_t launch_render_fwd(const gs_projected& p, const gs_bins& bins, const ViewTable& vt,
                             float3 bg, float* image, float* final_T, uint32_t* n_contrib,
                             float* depth, const float* target, float* dL, double* loss,
                             float* tile_loss, hipStream_t s) {
  if (vt.n_tiles == 0) return hipSuccess;
  const auto* xy = reinterpret_cast<const float2*>(p.xy);
  const auto* co = reinterpret_cast<const float4*>(p.conic_opacity);
  const auto* rd = reinterpret_cast<const float4*>(p.rgb_depth);
  const int ppl = tuning(GS_TUNE_FWD_PIXELS_PER_LANE);
  const int sched = tuning(GS_TUNE_FWD_SCHEDULE);
  // splats per thread and batch: 64 per batch at one wavefront per tile was
  // measured 4.5% faster than 128; 256 at two and four wavefronts
  const int spl = stage_per_thread(tuning(GS_TUNE_FWD_STAGE), ppl == 2 ? 2 : 1);
  const bool l1 = target != nullptr;
#define GS_FWD(P, S, L)                                                                          \
  launch_fwd<P, S, L>(sched, bins, vt, xy, co, rd, bg, image, final_T, n_contrib, depth, target, \
                      dL, tile_loss, s)
#define GS_FWD_PPL(P)                                     \
  if (spl == 2) {                                         \
    if (l1) GS_FWD(P, 2, true); else GS_FWD(P, 2, false); \
  } else {                                                \
    if (l1) GS_FWD(P, 1, true); else GS_FWD(P, 1, false); \
  }
  kernel_event_start(GS_KERNEL_RENDER_FWD, s);
  if (ppl == 4) {
    GS_FWD_PPL(4)
  } else if (ppl == 2) {
    GS_FWD_PPL(2)
  } else {
    GS_FWD_PPL(1)
  }
#undef GS_FWD_PPL
#undef GS_FWD
  kernel_event_stop(GS_KERNEL_RENDER_FWD, s);
  if (l1 && loss)
    hipLaunchKernelGGL(tile_loss_sum_kernel, dim3(1), dim3(1024), 0, s, tile_loss, vt.n_tiles,
                       loss);
  return hipGetLastError();
}

}  // namespace gsmi
