// gs_render_bwd: backward of compositing and projection.
//
// Pass 1 (per tile, 256 threads, same pixel mapping as the forward): each
// pixel starts at its last blended splat (n_contrib) with T = final_T and the
// normalised colour behind it S = bg, and walks the tile list in reverse,
// recovering the transmittance before splat i as T_i = T_{i+1} / (1 - a_i).
// Only the projection of S on the pixel's dL/dC is needed (dL/dalpha_i =
// T_i (c_i - S_i) . dL/dC), so that scalar is what the walk carries.
// For each splat the 9 screen-space partials (u, v, Q00, Q01, Q11, o, r, g, b)
// are summed over the wavefront with DPP row operations and added to a
// per-(view, splat) accumulator with one 9-lane atomic.
//
// The screen-space partials live in a view-major [V][n][9] buffer (the
// layout of the projected splats), so both passes touch it coalesced.
//
// Pass 2 (one lane per Gaussian, looping over the views): for every view
// where some lane of the wavefront has a visible splat with nonzero partials,
// re-evaluates the projection and chains the partials to the map parameters
// (accumulated in the lane) and to the view's pose tangent (summed over the
// wavefront, then per workgroup in float64, then over workgroups by a final
// small kernel in a fixed order: deterministic).
#include "project.h"

namespace gsmi {

namespace {

__device__ __forceinline__ float lane63(float x) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Transposed wavefront reduction of nine values with the gfx950 cross-half
// swaps.  v_permlane32_swap(a, b) exchanges a's lanes 32-63 with b's lanes
// 0-31, so adding its two results leaves a's 32-lane partial sums in lanes
// 0-31 and b's in lanes 32-63: one swap and one add halve two values.
// v_permlane16_swap does the same on 16-lane rows.  After both levels each
// 16-lane row of two registers holds a distinct value, and four row-local
// DPP adds finish the sums:
//   q0 rows = {v0, v2, v1, v3}, q1 rows = {v4, v6, v5, v7};
// the ninth value takes the plain DPP reduction to lane 63.
__device__ __forceinline__ float swap32_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap16_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// x + x of another lane of the same 16-lane row (every lane is a valid source)
template <int CTRL>
__device__ __forceinline__ float dpp_add(float x) {
  return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf,
                                                        true));
}

__device__ __forceinline__ float row16_sum(float x) {
  x = dpp_add<0x128>(x);   // row_ror:8
  x = dpp_add<0x124>(x);   // row_ror:4
  x = dpp_add<0x4e>(x);    // quad_perm [2,3,0,1]
  x = dpp_add<0xb1>(x);    // quad_perm [1,0,3,2]
  return x;                // every lane of the row holds the row total
}

struct Reduced9 {
  float q0, q1, q2;
};

// q0 and q1 as described above; the ninth value's total lands in lane 63 of q2.
__device__ __forceinline__ Reduced9 wave_reduce9(float v0, float v1, float v2, float v3, float v4,
                                                 float v5, float v6, float v7, float v8) {
  const float h0 = swap32_add(v0, v1), h1 = swap32_add(v2, v3);
  const float h2 = swap32_add(v4, v5), h3 = swap32_add(v6, v7);
  Reduced9 r;
  r.q0 = row16_sum(swap16_add(h0, h1));
  r.q1 = row16_sum(swap16_add(h2, h3));
  r.q2 = wave_sum_to_lane63(v8);
  return r;
}

// SPL: splats each thread stages per LDS batch (1 or 2).
template <int PPL, int SPL, bool Q>
__global__ __launch_bounds__(kBlock / PPL) void render_bwd_kernel(
    ViewTable vt, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ values,
    const uint32_t* __restrict__ order,
    const float2* __restrict__ xy, const float4* __restrict__ co, const float4* __restrict__ rd,
    float3 bg, const float* __restrict__ dL_dimage, const float* __restrict__ final_T,
    const uint32_t* __restrict__ n_contrib, float* __restrict__ grad2d,
    uint32_t* __restrict__ counter) {
  constexpr int NT = kBlock / PPL;
  constexpr int kStage = SPL * NT;   // splats staged per batch
  constexpr int kPerThread = kStage / NT;
  constexpr int kWords = kStage / 64;
  __shared__ StagedSplat s_splat[kStage];
  // s_reach[q][w] bit b: staged splat 64 w + b can reach quadrant q
  __shared__ uint64_t s_reach[4][kWords];
  __shared__ uint32_t s_maxlast;
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
    // where wave_reduce9 leaves each value: row r = lane / 16 of q0 holds value
    // {0, 2, 1, 3}[r] and of q1 value 4 + {0, 2, 1, 3}[r]; lane 63 of q2 holds
    // value 8
    // One atomic instruction adds all nine: lane 16 r takes q0's row total,
    // lane 16 r + 1 q1's, lane 63 the ninth value.
    const int row = lane >> 4, col16 = lane & 15;
    const int red_off0 = (row == 0) ? 0 : (row == 1) ? 2 : (row == 2) ? 1 : 3;
    const bool red_q0 = col16 == 0, red_q1 = col16 == 1, red_q2 = lane == 63;
    const int red_off = red_q0 ? red_off0 : red_q1 ? red_off0 + 4 : 8;

    // pixel k of a lane lies in column k % NC (see the forward kernel)
    constexpr int NC = PPL == 4 ? 2 : 1;
    // sdc: (colour behind the current splat) . dL/dC of the pixel
    float fpx[PPL], fpy[PPL], T[PPL], dC0[PPL], dC1[PPL], dC2[PPL], sdc[PPL];
    uint32_t last[PPL], qbit[PPL];
    uint32_t mylast = 0;
    const int64_t plane = (int64_t)vi.width * vi.height;
    const float* gimg = dL_dimage + 3 * vi.pix_base;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int i = k * NT + (int)threadIdx.x;
      const int q = i >> 6, l = i & 63;
      const int px = tx * kTile + (q & 1) * 8 + (l & 7);
      const int py = ty * kTile + (q >> 1) * 8 + (l >> 3);
      qbit[k] = __builtin_amdgcn_readfirstlane(1u << q);   // uniform over the wave
      fpx[k] = (float)px + 0.5f;
      fpy[k] = (float)py + 0.5f;
      T[k] = 1.0f;
      dC0[k] = dC1[k] = dC2[k] = sdc[k] = 0.f;
      last[k] = 0;
      if (px < vi.width && py < vi.height) {
        const int64_t off = (int64_t)py * vi.width + px;
        dC0[k] = gimg[off];
        dC1[k] = gimg[plane + off];
        dC2[k] = gimg[2 * plane + off];
        T[k] = final_T[vi.pix_base + off];
        sdc[k] = bg.x * dC0[k] + bg.y * dC1[k] + bg.z * dC2[k];
        last[k] = n_contrib[vi.pix_base + off];
        mylast = max(mylast, last[k]);
      }
    }
    // list positions this wave has to walk: below the largest n_contrib of its pixels
    uint32_t slot_last[PPL];   // per pixel slot: largest n_contrib over the wave
    uint32_t wave_last = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      uint32_t x = last[k];
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, d, 64));
      slot_last[k] = __builtin_amdgcn_readfirstlane(x);
      wave_last = max(wave_last, slot_last[k]);
    }
    if (threadIdx.x == 0) s_maxlast = 0;
    __syncthreads();
    if (lane == 0 && wave_last) atomicMax(&s_maxlast, wave_last);
    __syncthreads();
    const uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
    // n_contrib never exceeds the tile's list length for a matching forward;
    // the clamp keeps every list read inside [s, e) regardless.
    const int64_t list_len = (int64_t)e - (int64_t)s;
    const int64_t maxlast = min((int64_t)s_maxlast, max(list_len, (int64_t)0));

    for (int64_t bend = maxlast; bend > 0; bend -= kStage) {
      const int64_t bstart = max((int64_t)0, bend - kStage);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kPerThread; ++r) {
        const int slot = r * NT + (int)threadIdx.x;
        const int64_t k = bstart + slot;
        uint32_t reach = 0;
        if (k < bend)
          reach = stage_splat(values[s + (uint32_t)k], xy, co, rd,
                              tx * kTile, ty * kTile, vi.width, vi.height, s_splat[slot]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint64_t bq = __ballot((reach >> q) & 1u);
          if (lane == 0) s_reach[q][slot >> 6] = bq;
        }
      }
      __syncthreads();
      // Walk, in reverse list order, only the staged splats below this wave's
      // last blended position that reach one of its quadrants.
      for (int w = kWords - 1; w >= 0; --w) {
        const int64_t lim = (int64_t)wave_last - bstart - 64 * w;   // allowed bits: b < lim
        if (lim <= 0) continue;
        uint64_t m = 0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) m |= s_reach[__builtin_ctz(qbit[k])][w];
        m = uniform_u64(m);
        if (lim < 64) m &= (uint64_t(1) << lim) - 1;
        while (m) {
          const int bit = 63 - __builtin_clzll(m);
          m &= ~(uint64_t(1) << bit);
          const int j = 64 * w + bit;
          const uint32_t pos = (uint32_t)(bstart + j);
          const float4 geo = s_splat[j].geo;
          const float4 app = s_splat[j].app;
          const float4 ext = s_splat[j].ext;
          const uint32_t reach = PPL > 1 ? __builtin_amdgcn_readfirstlane(__float_as_uint(ext.y)) : ~0u;
          // Per pixel slot, branch-free over the wave: a lane whose pixel does
          // not blend this splat takes alpha = 0, which leaves T and S exactly
          // as they were and contributes exact zeros.
          float g0 = -0.0f, g1 = -0.0f, g2 = -0.0f, g3 = -0.0f, g4 = -0.0f, g5 = -0.0f,
                g6 = -0.0f, g7 = -0.0f, g8 = -0.0f;   // -0 + x == x exactly
          bool started = false;
          ColumnTerms ct[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) ct[c] = column_terms(geo, fpx[c]);
#pragma unroll
          for (int k = 0; k < PPL; ++k) {
            // slot-uniform skips: quadrant not reached, or every pixel of the
            // slot in this wave already past its last blended splat
            if (!(reach & qbit[k]) || pos >= slot_last[k]) continue;
            float alpha, raw, G, dy;
            const float dx = ct[k % NC].dx;
            const bool ok =
                eval_alpha_at<true>(ct[k % NC], geo, app, fpy[k], alpha, raw, G, dy) &&
                pos < last[k];
            if (!__ballot(ok)) continue;
            const float a = ok ? alpha : 0.0f;
            const float Tk = T[k] * __builtin_amdgcn_rcpf(1.0f - a);
            const float wgt = a * Tk;
            const float dot = __builtin_fmaf(
                ext.x, dC2[k], __builtin_fmaf(app.w, dC1[k], __builtin_fmaf(app.z, dC0[k], -sdc[k])));
            const float dalpha = Tk * dot;   // (c - S) . dL/dC
            // colour behind the next splat in front: S + alpha (c - S)
            sdc[k] = __builtin_fmaf(a, dot, sdc[k]);
            T[k] = Tk;
            // below the 0.99 clamp alpha = o G: d alpha/do = G, d alpha/dpower = alpha
            const float live = (ok && raw <= kAlphaMax) ? dalpha : 0.0f;
            const float gP = a * live;   // dL/dpower
            const float gdx = gP * dx, gdy = gP * dy;
            // d power/du = Q00 dx + Q01 dy (and likewise v): the conic factor is
            // the same for every pixel, so only sum(gP d) is accumulated here
            const float v2 = gdx * dx, v3 = gdx * dy, v4 = gdy * dy, v5 = G * live;
            const float v6 = wgt * dC0[k], v7 = wgt * dC1[k], v8 = wgt * dC2[k];
            g0 += gdx; g1 += gdy; g2 += v2; g3 += v3; g4 += v4; g5 += v5; g6 += v6; g7 += v7;
            g8 += v8;
            started = true;
          }
          if (started) {
            const Reduced9 r = wave_reduce9(g0, g1, g2, g3, g4, g5, g6, g7, g8);
            const uint32_t acc = __builtin_amdgcn_readfirstlane(__float_as_uint(ext.w));
            float* dst = grad2d + (int64_t)acc * 9;   // wave-uniform
            const float val = red_q0 ? r.q0 : red_q1 ? r.q1 : r.q2;
            if (red_q0 || red_q1 || red_q2) unsafeAtomicAdd(dst + red_off, val);
          }
        }
      }
    }
    if constexpr (!Q) break;
  }
}

// ---------------------------------------------------------------------------
// per-Gaussian backward through the projection
// ---------------------------------------------------------------------------

// Slots of the per-(Gaussian, view) contribution vector.
constexpr int kCMu = 0, kCRq = 3, kCSc = 12, kCOl = 15, kCSh = 16;

// Chain the nine screen-space partials of one (Gaussian, view) to the map
// parameters (accumulated into c) and to the view's pose tangent.
template <int DEG>
__device__ __forceinline__ void chain_one(const GaussState& G, const gs_camera& cam,
                                          const SHCoef<DEG>& C, const float* g2, float* c,
                                          float* pose) {
  constexpr int K = SHDim<DEG>::K;
  ViewState S;
  project_view<DEG>(G, cam, C, S);
  const float* W = cam.R;
  const float* t = cam.t;
  float GW[9] = {0.f}, gt[3] = {0.f, 0.f, 0.f}, gp[3];
  // opacity
  c[kCOl] += G.o * (1.0f - G.o) * g2[5];
  // colour -> SH coefficients and view direction
  float Y[K];
  sh_basis<DEG>(S.dir[0], S.dir[1], S.dir[2], Y);
  const float grgb[3] = {S.rgb_pos[0] ? g2[6] : 0.f, S.rgb_pos[1] ? g2[7] : 0.f,
                         S.rgb_pos[2] ? g2[8] : 0.f};
  float wk[K];
  for (int k = 0; k < K; ++k) wk[k] = 0.f;
  for (int ch = 0; ch < 3; ++ch)
    for (int k = 0; k < K; ++k) {
      c[kCSh + ch * K + k] += grgb[ch] * Y[k];
      wk[k] += grgb[ch] * C.f[ch * K + k];
    }
  float gdir[3];
  sh_basis_grad<DEG>(S.dir[0], S.dir[1], S.dir[2], wk, gdir[0], gdir[1], gdir[2]);
  const float dd = S.dir[0] * gdir[0] + S.dir[1] * gdir[1] + S.dir[2] * gdir[2];
  const float invn = 1.0f / S.dnorm;
  float gcc[3];
  for (int k = 0; k < 3; ++k) {
    const float gv = (gdir[k] - S.dir[k] * dd) * invn;
    c[kCMu + k] += gv;
    gcc[k] = -gv;
  }
  // camera centre c = -W^T t
  for (int jj = 0; jj < 3; ++jj)
    for (int ii = 0; ii < 3; ++ii) {
      GW[jj * 3 + ii] -= t[jj] * gcc[ii];
      gt[jj] -= W[jj * 3 + ii] * gcc[ii];
    }
  // conic -> Sigma2 entries: dL/dSigma' = -Q Gq Q
  const float h = 0.5f * g2[3];
  const float X00 = S.q0 * (S.q0 * g2[2] + S.q1 * h) + S.q1 * (S.q0 * h + S.q1 * g2[4]);
  const float X01 = S.q0 * (S.q1 * g2[2] + S.q2 * h) + S.q1 * (S.q1 * h + S.q2 * g2[4]);
  const float X11 = S.q1 * (S.q1 * g2[2] + S.q2 * h) + S.q2 * (S.q1 * h + S.q2 * g2[4]);
  const float ga = -X00, gb = -2.0f * X01, gc = -X11;
  float gA0[3], gA1[3];
  for (int k = 0; k < 3; ++k) {
    gA0[k] = 2.0f * ga * S.A0[k] + gb * S.A1[k];
    gA1[k] = gb * S.A0[k] + 2.0f * gc * S.A1[k];
  }
  float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f, gB[9];
  for (int k = 0; k < 3; ++k) {
    gJ00 += gA0[k] * S.B[0 * 3 + k];
    gJ02 += gA0[k] * S.B[2 * 3 + k];
    gJ11 += gA1[k] * S.B[1 * 3 + k];
    gJ12 += gA1[k] * S.B[2 * 3 + k];
    gB[0 * 3 + k] = S.J00 * gA0[k];
    gB[1 * 3 + k] = S.J11 * gA1[k];
    gB[2 * 3 + k] = S.J02 * gA0[k] + S.J12 * gA1[k];
  }
  // camera-frame position (projection and Jacobian)
  const float iz = S.inv_z, iz2 = iz * iz;
  const float fx = cam.fx, fy = cam.fy;
  // screen-space centre: slots 0, 1 hold sum(dL/dpower * (dx, dy)) over the
  // pixels; dL/du = Q00 s0 + Q01 s1, dL/dv = Q01 s0 + Q11 s1
  const float gu = S.q0 * g2[0] + S.q1 * g2[1];
  const float gv = S.q1 * g2[0] + S.q2 * g2[1];
  gp[0] = gu * fx * iz;
  gp[1] = gv * fy * iz;
  gp[2] = -(gu * fx * S.p[0] + gv * fy * S.p[1]) * iz2;
  gp[2] += -gJ00 * fx * iz2 - gJ11 * fy * iz2;
  if (!S.clx) {
    gp[0] += -gJ02 * fx * iz2;
    gp[2] += gJ02 * 2.0f * fx * S.p[0] * iz2 * iz;
  } else {
    gp[2] += gJ02 * fx * S.tx * iz2;
  }
  if (!S.cly) {
    gp[1] += -gJ12 * fy * iz2;
    gp[2] += gJ12 * 2.0f * fy * S.p[1] * iz2 * iz;
  } else {
    gp[2] += gJ12 * fy * S.ty * iz2;
  }
  // p = W mu + t
  for (int r = 0; r < 3; ++r) {
    gt[r] += gp[r];
    for (int k = 0; k < 3; ++k) {
      c[kCMu + k] += W[r * 3 + k] * gp[r];
      GW[r * 3 + k] += gp[r] * G.mu[k];
    }
  }
  // B = W M with M = R(q) diag(s)
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      float gm = 0.f, gw = 0.f;
      for (int q = 0; q < 3; ++q) {
        gm += W[q * 3 + r] * gB[q * 3 + k];
        gw += gB[r * 3 + q] * G.M[k * 3 + q];
      }
      c[kCRq + r * 3 + k] += gm * G.s[k];
      c[kCSc + k] += gm * G.Rq[r * 3 + k];
      GW[r * 3 + k] += gw;
    }
  // dL/dphi = <dL/dW, [e]x W> + <dL/dt, [e]x t>, dL/drho = dL/dt
  float Mm[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      Mm[r * 3 + k] = GW[r * 3 + 0] * W[k * 3 + 0] + GW[r * 3 + 1] * W[k * 3 + 1] +
                      GW[r * 3 + 2] * W[k * 3 + 2];
  pose[0] += gt[0];
  pose[1] += gt[1];
  pose[2] += gt[2];
  pose[3] += Mm[7] - Mm[5] + (t[1] * gt[2] - t[2] * gt[1]);
  pose[4] += Mm[2] - Mm[6] + (t[2] * gt[0] - t[0] * gt[2]);
  pose[5] += Mm[3] - Mm[1] + (t[0] * gt[1] - t[1] * gt[0]);
}

constexpr int kProjBwdMaxBlocks = 2048;

// One lane per Gaussian (grid-stride), views in turn.  Map gradients
// accumulate in the lane; each view's pose partials are summed over the
// wavefront and added, in float64, to the wave's row of s_pose.
template <int DEG>
__global__ __launch_bounds__(256) void project_bwd_kernel(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ ologit,
    const float* __restrict__ sh, int64_t n, const gs_camera* __restrict__ cams, int n_views,
    const int32_t* __restrict__ radius, float* __restrict__ grad2d,
    float* __restrict__ g_means, float* __restrict__ g_log_scales, float* __restrict__ g_quats,
    float* __restrict__ g_ologit, float* __restrict__ g_sh, double* __restrict__ pose_part,
    uint32_t flags) {
  constexpr int K = SHDim<DEG>::K;
  constexpr int NC = kCSh + 3 * K;
  __shared__ double s_pose[4][GS_MAX_VIEWS][6];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool want_pose = !(flags & GS_BWD_NO_POSE);
  const bool want_map = !(flags & GS_BWD_POSE_ONLY);
  const bool overwrite = (flags & GS_BWD_OVERWRITE) != 0;
  const bool keep_clear = (flags & GS_BWD_KEEP_CLEAR) != 0;
  for (int t = threadIdx.x; t < 4 * GS_MAX_VIEWS * 6; t += 256) (&s_pose[0][0][0])[t] = 0.0;
  __syncthreads();
  for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < n;
    GaussState G;
    if (valid) load_gauss(means, log_scales, quats, ologit, n, i, G);
    else G.ok = false;
    // views where this Gaussian is visible, loaded up front (the loads are in
    // flight together), so a view that no lane of the wave sees costs no
    // memory round trip (measured 0.150 -> 0.130 ms on the 32-view room)
    uint64_t vis = 0;
    if (G.ok) {
#pragma unroll 8
      for (int v = 0; v < n_views; ++v)
        vis |= (uint64_t)(radius[(int64_t)v * n + i] > 0) << v;
    }
    SHCoef<DEG> C;
    if (G.ok) load_sh<DEG>(sh, n, i, C);
    float c[NC];
    for (int k = 0; k < NC; ++k) c[k] = 0.f;
    // the views any lane of the wave sees, walked in order; each view's
    // screen-space records are loaded one view ahead, so the load latency
    // overlaps the previous view's chain
    uint64_t wvis = vis;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)wvis, d, 64);
      const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(wvis >> 32), d, 64);
      wvis |= ((uint64_t)hi << 32) | lo;
    }
    wvis = uniform_u64(wvis);
    float g2n[9];
    auto load_rec = [&](int v) {
      const bool act = (vis >> v) & 1u;
      const float* src = grad2d + ((int64_t)v * n + i) * 9;
#pragma unroll
      for (int k = 0; k < 9; ++k) g2n[k] = act ? src[k] : 0.0f;
    };
    int vnext = wvis ? __builtin_ctzll(wvis) : -1;
    if (vnext >= 0) {
      wvis &= wvis - 1;
      load_rec(vnext);
    }
    while (vnext >= 0) {
      const int v = vnext;
      float g2[9];
      bool nz = false;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        g2[k] = g2n[k];
        nz = nz || g2[k] != 0.0f;
      }
      vnext = wvis ? __builtin_ctzll(wvis) : -1;
      if (vnext >= 0) {
        wvis &= wvis - 1;
        load_rec(vnext);
      }
      const bool active = ((vis >> v) & 1u) && nz;
      if (!__any(active)) continue;
      if (keep_clear && active) {   // leave the record clear for the next call
        float* src = grad2d + ((int64_t)v * n + i) * 9;
        for (int k = 0; k < 9; ++k) src[k] = 0.0f;
      }
      // slots 2-4 hold sum(dL/dpower * (dx^2, dx dy, dy^2)); dL/dQ00,
      // dL/dQ01, dL/dQ11 are those times -1/2, -1, -1/2 (exact scalings)
      g2[2] *= -0.5f;
      g2[3] = -g2[3];
      g2[4] *= -0.5f;
      float pose[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (active) chain_one<DEG>(G, cams[v], C, g2, c, pose);
      if (want_pose) {
        for (int k = 0; k < 6; ++k) {
          const float tot = lane63(wave_sum_to_lane63(pose[k]));
          if (lane == 0) s_pose[w][v][k] += (double)tot;
        }
      }
    }
    if (!want_map || !valid) continue;
    if (!G.ok) {
      if (overwrite) {
        for (int k = 0; k < 3; ++k) g_means[k * n + i] = g_log_scales[k * n + i] = 0.f;
        for (int k = 0; k < 4; ++k) g_quats[k * n + i] = 0.f;
        g_ologit[i] = 0.f;
        for (int k = 0; k < 3 * K; ++k) g_sh[k * n + i] = 0.f;
      }
      continue;
    }
    auto put = [&](float* ptr, float val) { *ptr = overwrite ? val : *ptr + val; };
    for (int k = 0; k < 3; ++k) {
      put(&g_means[k * n + i], c[kCMu + k]);
      put(&g_log_scales[k * n + i], G.s[k] * c[kCSc + k]);
    }
    put(&g_ologit[i], c[kCOl]);
    for (int k = 0; k < 3 * K; ++k) put(&g_sh[k * n + i], c[kCSh + k]);
    // R(q) -> normalised quaternion -> raw quaternion
    const float qw = G.q[0], qx = G.q[1], qy = G.q[2], qz = G.q[3];
    const float* g = c + kCRq;
    float dq[4];
    dq[0] = 2.f * (-qz * g[1] + qy * g[2] + qz * g[3] - qx * g[5] - qy * g[6] + qx * g[7]);
    dq[1] = 2.f * (qy * g[1] + qz * g[2] + qy * g[3] - 2.f * qx * g[4] - qw * g[5] + qz * g[6] +
                   qw * g[7] - 2.f * qx * g[8]);
    dq[2] = 2.f * (-2.f * qy * g[0] + qx * g[1] + qw * g[2] + qx * g[3] + qz * g[5] - qw * g[6] +
                   qz * g[7] - 2.f * qy * g[8]);
    dq[3] = 2.f * (-2.f * qz * g[0] - qw * g[1] + qx * g[2] + qw * g[3] - 2.f * qz * g[4] +
                   qy * g[5] + qx * g[6] + qy * g[7]);
    const float dot = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
    const float inv = 1.0f / G.qnorm;
    for (int k = 0; k < 4; ++k) put(&g_quats[k * n + i], (dq[k] - G.q[k] * dot) * inv);
  }
  if (!want_pose) return;
  __syncthreads();
  for (int t = threadIdx.x; t < n_views * 6; t += 256) {
    const int vv = t / 6, k = t % 6;
    pose_part[(int64_t)blockIdx.x * n_views * 6 + t] =
        s_pose[0][vv][k] + s_pose[1][vv][k] + s_pose[2][vv][k] + s_pose[3][vv][k];
  }
}

// Clears the partials of visible splats (radius > 0): the only records the
// reverse walk adds to and the projection backward reads.
__global__ __launch_bounds__(256) void zero_visible_kernel(const int32_t* __restrict__ radius,
                                                           int64_t n_entries,
                                                           float* __restrict__ grad2d) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_entries || radius[e] <= 0) return;
  float* d = grad2d + e * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) d[k] = 0.0f;
}

// An empty map under GS_BWD_OVERWRITE: the pose gradient is zero.
__global__ __launch_bounds__(256) void zero_f32_kernel(float* __restrict__ p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0f;
}

// One workgroup per (view, component): strided float64 sum over the
// per-workgroup partials, then a tree reduction in LDS (fixed order).
__global__ __launch_bounds__(256) void pose_reduce_kernel(const double* __restrict__ pose_part,
                                                          int64_t nblocks, int n_views,
                                                          float* __restrict__ xi, int overwrite) {
  __shared__ double s_acc[256];
  const int t = blockIdx.x;   // view * 6 + component
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += 256) acc += pose_part[b * n_views * 6 + t];
  s_acc[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_acc[threadIdx.x] += s_acc[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) xi[t] = overwrite ? (float)s_acc[0] : xi[t] + (float)s_acc[0];
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t proj_bwd_blocks(int64_t n, int /*n_views*/) {
  return std::max<int64_t>(1, std::min<int64_t>(kProjBwdMaxBlocks, (n + 255) / 256));
}

}  // namespace

BwdPlan make_bwd_plan(int64_t n, const ViewTable& vt) {
  BwdPlan P{};
  const int64_t nblocks = proj_bwd_blocks(n, vt.n_views);
  size_t off = 0;
  P.off_grad2d = off;
  off += align_up(sizeof(float) * 9 * (size_t)n * vt.n_views);
  P.off_pose = off;
  off += align_up(sizeof(double) * 6 * (size_t)std::max<int64_t>(nblocks, 1) * vt.n_views);
  P.total = off;
  return P;
}

namespace {

template <int DEG>
void launch_project_bwd_deg(const gs_gaussians& g, const gs_camera* cams, int V,
                            const int32_t* radius, float* grad2d, const gs_grads& gr,
                            double* pose_part, uint32_t flags, dim3 grid, dim3 block,
                            hipStream_t s) {
  hipLaunchKernelGGL((project_bwd_kernel<DEG>), grid, block, 0, s, g.means, g.log_scales, g.quats,
                     g.opacity_logits, g.sh, g.n, cams, V, radius, grad2d, gr.means,
                     gr.log_scales, gr.quats, gr.opacity_logits, gr.sh, pose_part, flags);
}

void launch_project_bwd(const gs_gaussians& g, const gs_camera* cams, int V, const int32_t* radius,
                        float* grad2d, const gs_grads& gr, double* pose_part, uint32_t flags,
                        dim3 grid, dim3 block, hipStream_t s) {
  switch (g.sh_degree) {
    case 0: launch_project_bwd_deg<0>(g, cams, V, radius, grad2d, gr, pose_part, flags, grid, block, s); break;
    case 1: launch_project_bwd_deg<1>(g, cams, V, radius, grad2d, gr, pose_part, flags, grid, block, s); break;
    case 2: launch_project_bwd_deg<2>(g, cams, V, radius, grad2d, gr, pose_part, flags, grid, block, s); break;
    default: launch_project_bwd_deg<3>(g, cams, V, radius, grad2d, gr, pose_part, flags, grid, block, s); break;
  }
}

template <int P, int S>
void launch_bwd(int schedule, const gs_bins& bins, const ViewTable& vt, const float2* xy,
                const float4* co, const float4* rd, float3 bg, const float* dL_dimage,
                const float* final_T, const uint32_t* n_contrib,
                float* grad2d, hipStream_t s) {
  const int resident = schedule >= GS_SCHEDULE_PERSISTENT
                           ? resident_workgroups((const void*)render_bwd_kernel<P, S, true>,
                                                 kBlock / P)
                           : 0;
  const TileSchedule sc = tile_schedule(schedule, bins, GS_QUEUE_BWD, vt.n_tiles, resident);
  if (sc.counter)
    hipLaunchKernelGGL((render_bwd_kernel<P, S, true>), dim3(sc.grid), dim3(kBlock / P), 0, s, vt,
                       bins.ranges, bins.values, sc.order, xy, co, rd, bg, dL_dimage, final_T,
                       n_contrib, grad2d, sc.counter);
  else
    hipLaunchKernelGGL((render_bwd_kernel<P, S, false>), dim3(sc.grid), dim3(kBlock / P), 0, s, vt,
                       bins.ranges, bins.values, sc.order, xy, co, rd, bg, dL_dimage, final_T,
                       n_contrib, grad2d, nullptr);
}

}  // namespace

hipError_t launch_render_bwd(const gs_gaussians& g, const gs_projected& p, const gs_bins& bins,
                             const gs_camera* cams_dev, const ViewTable& vt, float3 bg,
                             const float* dL_dimage, const float* final_T,
                             const uint32_t* n_contrib, const gs_grads& grads, uint32_t flags,
                             char* ws, const BwdPlan& plan, hipStream_t s) {
  float* grad2d = reinterpret_cast<float*>(ws + plan.off_grad2d);
  double* pose_part = reinterpret_cast<double*>(ws + plan.off_pose);
  const int64_t n_entries = g.n * (int64_t)vt.n_views;
  if (n_entries > 0 && !(flags & GS_BWD_KEEP_CLEAR))
    hipLaunchKernelGGL(zero_visible_kernel, dim3((unsigned)((n_entries + 255) / 256)), dim3(256), 0,
                       s, p.radius, n_entries, grad2d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (vt.n_tiles > 0) {
    const auto* xy = reinterpret_cast<const float2*>(p.xy);
    const auto* co = reinterpret_cast<const float4*>(p.conic_opacity);
    const auto* rd = reinterpret_cast<const float4*>(p.rgb_depth);
    const int ppl = tuning(GS_TUNE_BWD_PIXELS_PER_LANE);
    const int sched = tuning(GS_TUNE_BWD_SCHEDULE);
    // splats per thread and batch: 128 per batch at one and two wavefronts
    // per tile, 256 at four
    const int spl = stage_per_thread(tuning(GS_TUNE_BWD_STAGE), ppl == 1 ? 1 : 2);
#define GS_BWD(P, S) \
  launch_bwd<P, S>(sched, bins, vt, xy, co, rd, bg, dL_dimage, final_T, n_contrib, grad2d, s)
    kernel_event_start(GS_KERNEL_RENDER_BWD, s);
    if (ppl == 4) {
      if (spl == 2) GS_BWD(4, 2); else GS_BWD(4, 1);
    } else if (ppl == 2) {
      if (spl == 2) GS_BWD(2, 2); else GS_BWD(2, 1);
    } else {
      if (spl == 2) GS_BWD(1, 2); else GS_BWD(1, 1);
    }
#undef GS_BWD
    kernel_event_stop(GS_KERNEL_RENDER_BWD, s);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (g.n == 0) {   // nothing to chain; an overwritten pose gradient is zero
    if (!(flags & GS_BWD_NO_POSE) && (flags & GS_BWD_OVERWRITE) && vt.n_views > 0)
      hipLaunchKernelGGL(zero_f32_kernel, dim3(1), dim3(256), 0, s, grads.xi, vt.n_views * 6);
    return hipGetLastError();
  }
  const int64_t nblocks = proj_bwd_blocks(g.n, vt.n_views);
  const dim3 grid((unsigned)nblocks), block(256);
  kernel_event_start(GS_KERNEL_PROJECT_BWD, s);
  launch_project_bwd(g, cams_dev, vt.n_views, p.radius, grad2d, grads, pose_part, flags, grid,
                     block, s);
  kernel_event_stop(GS_KERNEL_PROJECT_BWD, s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!(flags & GS_BWD_NO_POSE)) {
    const int nt = vt.n_views * 6;
    hipLaunchKernelGGL(pose_reduce_kernel, dim3(nt), dim3(256), 0, s, pose_part,
                       nblocks, vt.n_views, grads.xi, (flags & GS_BWD_OVERWRITE) ? 1 : 0);
  }
  return hipGetLastError();
}

}  // namespace gsmi
