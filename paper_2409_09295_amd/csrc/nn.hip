// Kernels of the learned Gaussian initialiser: a small U-Net over BF16 NHWC
// activations with FP32 accumulation on MFMA (v_mfma_f32_16x16x32_bf16).
//
// conv3x3 (forward and, with flipped/transposed weights, backward-data) is an
// implicit GEMM: M = pixels, N = output channels, K = 9 taps x input
// channels.  A 256-thread workgroup owns a 64-pixel x 64-channel tile; each
// wavefront computes a 32 x 32 quarter as 2 x 2 MFMA tiles.  Per K step
// (one tap, 32 input channels) the workgroup stages the 64 x 32 activation
// slice (zero outside the image; channels may come from two tensors, which
// is how the decoder's skip concatenation is read without materialising it)
// and the 64 x 32 weight slice in LDS, both K-contiguous so that every MFMA
// operand fragment is one 16-byte LDS read.  An optional mask tensor zeroes
// input entries whose mask value is <= 0 (the ReLU backward fused into the
// backward-data pass).
//
// conv3x3_wgrad: dW[tap][co][ci] = sum_p dz[p][co] x[p + tap][ci] as a GEMM
// with M = Cout, N = Cin, K = pixels, split over pixel chunks with float32
// atomics; tiles are transposed through LDS so fragments stay contiguous.
//
// MFMA 16x16x32 operand layout (lane l, 8 values each): A row l % 16, B
// column l % 16, both covering k = 8 (l / 16) .. 8 (l / 16) + 7; result D row
// 4 (l / 16) + j, column l % 16, j = 0..3.
#include "gs_internal.h"
#include "gs_nn.h"

namespace gsmi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round-to-nearest-even float -> bf16 (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LDK = BK + 8;   // LDS row pitch in bf16 (16-byte aligned, skews banks)

struct ActView {
  const uint16_t* p;
  int32_t c, stride, offset;
};

// Zeroes the bf16 elements of v whose mask element is <= 0.
__device__ __forceinline__ uint4 apply_mask8(uint4 v, uint4 mk) {
  const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
  uint32_t vw[4] = {v.x, v.y, v.z, v.w};
  for (int q = 0; q < 4; ++q) {
    const uint32_t lo = (int16_t)(mw[q] & 0xFFFF) > 0 ? 0xFFFFu : 0u;   // bf16 > 0 <=> int16 > 0
    const uint32_t hi = (int16_t)(mw[q] >> 16) > 0 ? 0xFFFF0000u : 0u;
    vw[q] &= (lo | hi);
  }
  return make_uint4(vw[0], vw[1], vw[2], vw[3]);
}

// Loads 8 consecutive channels [c0, c0 + 8) of pixel (n, y, x) from a
// two-source channel concatenation; zero outside the image or beyond the
// channel count.  mask (optional, same layout as the concatenation) zeroes
// elements whose mask is <= 0.
__device__ __forceinline__ uint4 load8(const ActView& a, const ActView& b, const ActView& m,
                                       int64_t pix, bool inb, int c0) {
  uint4 v = make_uint4(0, 0, 0, 0);
  if (!inb) return v;
  const ActView* s = &a;
  int c = c0;
  if (c0 >= a.c) {
    s = &b;
    c = c0 - a.c;
  }
  if (s->p == nullptr || c >= s->c) return v;
  v = *reinterpret_cast<const uint4*>(s->p + pix * s->stride + s->offset + c);
  if (m.p) {
    const uint4 mk = *reinterpret_cast<const uint4*>(m.p + pix * m.stride + m.offset + c0);
    v = apply_mask8(v, mk);
  }
  return v;
}

// Output tile of BMT pixels x BNT output channels; each of the four
// wavefronts computes a (16 IM) x 32 block (IM x 2 MFMA tiles of 16 x 16).
// K runs over 9 taps x cin in steps of BK = 32 channels; the next step's
// global loads are issued before this step's MFMAs, so their latency hides
// behind them.
template <int BMT, int BNT, int IM>
__global__ __launch_bounds__(256) void conv3x3_kernel(
    ActView x1, ActView x2, ActView mask, int N, int H, int W, const uint16_t* __restrict__ wk,
    int cout, int cin, const float* __restrict__ bias, int relu, uint16_t* __restrict__ y,
    int y_stride, int y_offset, float* __restrict__ yf, int yf_stride) {
  static_assert(BMT * BNT == 4 * 16 * IM * 32 && BNT % 32 == 0 && BMT % 64 == 0,
                "four (16 IM) x 32 wavefront tiles");
  constexpr int AR = BMT / 64;   // A rows (pixels) staged per thread
  __shared__ __attribute__((aligned(16))) uint16_t sA[BMT * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t sB[BNT * LDK];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t npix = (int64_t)N * H * W;
  const int64_t m0 = (int64_t)blockIdx.x * BMT;
  const int n0 = blockIdx.y * BNT;
  // loaders: thread t stages A rows (t / 4) + 64 u and B row t / 4 (when
  // below BNT), channels 8 (t % 4) .. +8 of the step
  const int lcol = (t & 3) * 8, lrow = t >> 2;
  int ly[AR], lx[AR], limg[AR];
  bool lok[AR];
#pragma unroll
  for (int u = 0; u < AR; ++u) {
    const int64_t lp = m0 + lrow + 64 * u;
    lok[u] = lp < npix;
    limg[u] = ly[u] = lx[u] = 0;
    if (lok[u]) {
      limg[u] = (int)(lp / ((int64_t)H * W));
      const int rem = (int)(lp - (int64_t)limg[u] * H * W);
      ly[u] = rem / W;
      lx[u] = rem - ly[u] * W;
    }
  }
  const bool bload = lrow < BNT;
  const int csteps = (cin + BK - 1) / BK;
  const int nsteps = 9 * csteps;
  // the mask (backward data: the ReLU of this layer's output) is loaded
  // beside the values and applied when the step is written to LDS, so the
  // prefetch does not wait for it
  const bool masked = mask.p != nullptr;
  const ActView none = {nullptr, 0, 0, 0};
  uint4 ra[AR], rm[AR], rb;
  auto fetch = [&](int step) {
    const int tap = step / csteps, c0 = (step - tap * csteps) * BK;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
    for (int u = 0; u < AR; ++u) {
      const int sy = ly[u] + dy, sx = lx[u] + dx;
      const bool inb = lok[u] && sy >= 0 && sy < H && sx >= 0 && sx < W;
      const int64_t pix = ((int64_t)limg[u] * H + sy) * W + sx;
      ra[u] = load8(x1, x2, none, pix, inb, c0 + lcol);
      if (masked) rm[u] = load8(mask, none, none, pix, inb, c0 + lcol);
    }
    rb = make_uint4(0, 0, 0, 0);
    const int co = n0 + lrow, ci = c0 + lcol;
    if (bload && co < cout && ci < cin)
      rb = *reinterpret_cast<const uint4*>(wk + ((int64_t)tap * cout + co) * cin + ci);
  };
  f32x4 acc[IM][2];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  constexpr int WN = BNT / 32;   // wavefronts across the channels
  const int wm = (wv % (4 / WN)) * 16 * IM, wn = (wv / (4 / WN)) * 32;
  fetch(0);
  for (int step = 0; step < nsteps; ++step) {
    __syncthreads();   // the previous step's fragments have been read
#pragma unroll
    for (int u = 0; u < AR; ++u)
      *reinterpret_cast<uint4*>(&sA[(lrow + 64 * u) * LDK + lcol]) =
          masked ? apply_mask8(ra[u], rm[u]) : ra[u];
    if (bload) *reinterpret_cast<uint4*>(&sB[lrow * LDK + lcol]) = rb;
    __syncthreads();
    if (step + 1 < nsteps) fetch(step + 1);
    bf16x8 a[IM], b[2];
#pragma unroll
    for (int i = 0; i < IM; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(&sA[(wm + i * 16 + (lane & 15)) * LDK + 8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(&sB[(wn + j * 16 + (lane & 15)) * LDK + 8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  // epilogue: bias, ReLU, bf16 (or float32) store
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int co = n0 + wn + j * 16 + (lane & 15);
      if (co >= cout) continue;
      const float bco = bias ? bias[co] : 0.f;
      for (int r = 0; r < 4; ++r) {
        const int64_t p = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        if (p >= npix) continue;
        float v = acc[i][j][r] + bco;
        if (relu) v = fmaxf(v, 0.f);
        if (y) y[p * y_stride + y_offset + co] = f2bf(v);
        if (yf) yf[p * yf_stride + co] = v;
      }
    }
}

// Direct 3x3 convolution on spatial tiles.  A workgroup computes 16 x 16
// pixel tiles of one image for BNT output channels; wavefront w computes
// output rows 4w .. 4w + 3 (each a 16-pixel MFMA row block) for all BNT
// channels.  Input channels go in chunks of 32: the chunk's 18 x 18 input
// patch (the tile and its one-pixel halo; zero outside the image) and its
// 9 x BNT x 32 weights are staged in LDS once, and every tap's A fragments
// are read from the patch at the tap's offset, so each input value is loaded
// from memory about 1.3 times instead of nine.  Workgroups are persistent:
// workgroup b takes tiles b, b + gridDim.x, ..., and the next (tile, chunk)
// pair's patch and weights are loaded into registers while this pair's
// 9 x 4 x BNT/16 MFMAs per wavefront run, so a layer with a single chunk
// overlaps the next tile's loads with this tile's products and stores.  With
// a single chunk the weights stay in LDS for all of a workgroup's tiles.
constexpr int PT = 16;                  // output tile side
constexpr int PP = PT + 2;              // patch side (with halo)
constexpr int PCC = 32;                 // input channels per chunk
constexpr int PPITCH = PCC + 8;         // LDS pitch in bf16 (80 bytes: 16-byte rows, spread banks)
constexpr int PATCH_CHUNKS = PP * PP * (PCC / 8);   // 16-byte pieces of a patch (1,296)

// MASKED: the input is multiplied by a ReLU mask (mask > 0) as it is staged.
template <int BNT, bool MASKED>
__global__ __launch_bounds__(256, BNT == 32 ? 3 : 2) void conv3x3_patch_kernel(
    ActView x1, ActView x2, ActView mask, int N, int H, int W, const uint16_t* __restrict__ wk,
    int cout, int cin, const float* __restrict__ bias, int relu, uint16_t* __restrict__ y,
    int y_stride, int y_offset, float* __restrict__ yf, int yf_stride) {
  constexpr int JN = BNT / 16;
  constexpr int W_CHUNKS = 9 * BNT * (PCC / 8);     // 16-byte pieces of a chunk's weights
  constexpr int PA = (PATCH_CHUNKS + 255) / 256;    // per thread
  constexpr int PB = (W_CHUNKS + 255) / 256;
  __shared__ __attribute__((aligned(16))) uint16_t sP[PP * PP * PPITCH];
  __shared__ __attribute__((aligned(16))) uint16_t sW[9 * BNT * PPITCH];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int tiles_x = (W + PT - 1) / PT, tiles_y = (H + PT - 1) / PT;
  const int n_tiles = N * tiles_x * tiles_y;
  const int n0 = blockIdx.y * BNT;
  const int nchunks = (cin + PCC - 1) / PCC;
  const bool w_resident = nchunks == 1;   // the weights are loaded once per workgroup
  const ActView none = {nullptr, 0, 0, 0};
  uint4 ra[PA], rm[MASKED ? PA : 1], rb[PB];
  auto fetch = [&](int tile, int chunk, bool weights) {
    const int img = tile / (tiles_x * tiles_y);
    const int trem = tile - img * tiles_x * tiles_y;
    const int ty0 = (trem / tiles_x) * PT, tx0 = (trem % tiles_x) * PT;
    const int c0 = chunk * PCC;
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      const int q = t + 256 * u;            // piece q: patch pixel q / 4, channels 8 (q % 4)
      const int pp = q >> 2, cc = (q & 3) * 8;
      const int py = pp / PP, px = pp - py * PP;
      const int sy = ty0 + py - 1, sx = tx0 + px - 1;
      const bool inb = q < PATCH_CHUNKS && sy >= 0 && sy < H && sx >= 0 && sx < W &&
                       c0 + cc < cin;
      const int64_t pix = ((int64_t)img * H + sy) * W + sx;
      ra[u] = load8(x1, x2, none, pix, inb, c0 + cc);
      if constexpr (MASKED) rm[u] = load8(mask, none, none, pix, inb, c0 + cc);
    }
    if (!weights) return;
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int q = t + 256 * u;            // piece q: (tap, channel n) = q / 4, inputs 8 (q % 4)
      const int tn = q >> 2, cc = (q & 3) * 8;
      const int tap = tn / BNT, co = n0 + (tn - tap * BNT);
      rb[u] = make_uint4(0, 0, 0, 0);
      if (q < W_CHUNKS && co < cout && c0 + cc < cin)
        rb[u] = *reinterpret_cast<const uint4*>(wk + ((int64_t)tap * cout + co) * cin + c0 + cc);
    }
  };
  f32x4 acc[4][JN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  // registers -> LDS: the patch, and the weights when they are (re)loaded
  auto stage = [&](bool weights) {
#pragma unroll
    for (int u = 0; u < PA; ++u) {
      const int q = t + 256 * u;
      if (q < PATCH_CHUNKS) {
        uint4 v = ra[u];
        if constexpr (MASKED) v = apply_mask8(v, rm[u]);
        *reinterpret_cast<uint4*>(&sP[(q >> 2) * PPITCH + (q & 3) * 8]) = v;
      }
    }
    if (!weights) return;
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const int q = t + 256 * u;
      if (q < W_CHUNKS) *reinterpret_cast<uint4*>(&sW[(q >> 2) * PPITCH + (q & 3) * 8]) = rb[u];
    }
  };
  auto multiply = [&]() {
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;   // patch offsets of the tap (0 .. 2)
      bf16x8 a[4], b[JN];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(
            &sP[((4 * wv + i + dy) * PP + (lane & 15) + dx) * PPITCH + 8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < JN; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(
            &sW[(tap * BNT + j * 16 + (lane & 15)) * PPITCH + 8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };
  // bias, ReLU, bf16 (or float32) store, accumulators cleared; acc[i][j][r] is
  // output row 4 wv + i, column 4 (lane / 16) + r, channel n0 + 16 j + lane % 16
  auto epilogue = [&](int tile) {
    const int img = tile / (tiles_x * tiles_y);
    const int trem = tile - img * tiles_x * tiles_y;
    const int ty0 = (trem / tiles_x) * PT, tx0 = (trem % tiles_x) * PT;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int oy = ty0 + 4 * wv + i;
#pragma unroll
      for (int j = 0; j < JN; ++j) {
        const int co = n0 + j * 16 + (lane & 15);
        if (oy < H && co < cout) {
          const float bco = bias ? bias[co] : 0.f;
          for (int r = 0; r < 4; ++r) {
            const int ox = tx0 + 4 * (lane >> 4) + r;
            if (ox >= W) continue;
            const int64_t p = ((int64_t)img * H + oy) * W + ox;
            float v = acc[i][j][r] + bco;
            if (relu) v = fmaxf(v, 0.f);
            if (y) y[p * y_stride + y_offset + co] = f2bf(v);
            if (yf) yf[p * yf_stride + co] = v;
          }
        }
        acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
      }
    }
  };
  int tile = blockIdx.x;
  if (tile >= n_tiles) return;   // the grid never exceeds the tiles; uniform over the workgroup
  fetch(tile, 0, true);
  if constexpr (MASKED) {
    // one tile per workgroup: the next chunk's loads overlap this chunk's products
    for (int chunk = 0; chunk < nchunks; ++chunk) {
      __syncthreads();   // the previous chunk's fragments have been read
      stage(true);
      __syncthreads();
      if (chunk + 1 < nchunks) fetch(tile, chunk + 1, true);
      multiply();
    }
    epilogue(tile);
  } else {
    int chunk = 0;
    for (bool first = true;; first = false) {
      __syncthreads();   // the previous pair's fragments have been read
      stage(first || !w_resident);
      __syncthreads();
      // the next (tile, chunk) pair, loaded while this one is multiplied
      int next_tile = tile, next_chunk = chunk + 1;
      if (next_chunk == nchunks) {
        next_chunk = 0;
        next_tile = tile + (int)gridDim.x;
      }
      const bool more = next_tile < n_tiles;
      if (more) fetch(next_tile, next_chunk, !w_resident);
      multiply();
      if (chunk == nchunks - 1) epilogue(tile);
      if (!more) break;
      tile = next_tile;
      chunk = next_chunk;
    }
  }
}

// Weight-gradient tile: 64 output channels x 64 input channels for one row
// of three taps (dy fixed, dx = -1, 0, 1: one load of dz serves three taps),
// pixels [kbeg, kbeg + kchunk) of the K dimension.  Each stage covers 64
// pixels: thread t loads pixels 2 (t % 32) and 2 (t % 32) + 1, channels
// 8 (t / 32) .. +8, of both dz (output-channel tile) and the tap-shifted
// inputs (input-channel tile) with 16-byte loads, and writes them transposed
// ([channel][pixel], two pixels per 32-bit write) into LDS; each wavefront
// then issues two K steps of four MFMAs per tap.
constexpr int WBK = 64;              // pixels per stage
constexpr int WLDK = WBK + 8;        // LDS row pitch in bf16 (16-byte aligned rows)
constexpr int kWgradBlocks = 512;    // pixel chunks are sized for about this many workgroups
constexpr int kWgrad32Blocks = 512;  // the narrow kernel: two resident workgroups per CU


__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(
    ActView x1, ActView x2, ActView dz, ActView mask, int N, int H, int W, int cout, int cin,
    int64_t kchunk, float* __restrict__ dw, float* __restrict__ dbias) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[BM * WLDK];   // [co][pixel]
  __shared__ __attribute__((aligned(16))) uint16_t sB[3][BN * WLDK];   // per tap [ci][pixel]
  __shared__ float s_bias[BM][33];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t npix = (int64_t)N * H * W;
  const int co0 = blockIdx.x * BM;
  const int row = blockIdx.y % 3;
  const int ci0 = (blockIdx.y / 3) * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = min(npix, kbeg + kchunk);
  const int dy = row - 1;
  f32x4 acc[3][2][2];
  for (int u = 0; u < 3; ++u)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[u][i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const bool do_bias = dbias != nullptr && row == 1 && ci0 == 0;
  float bacc[8];
  for (int q = 0; q < 8; ++q) bacc[q] = 0.f;
  const int wm = (wv & 1) * 32, wn = (wv >> 1) * 32;
  // this thread stages pixels k0 + 2 pp and k0 + 2 pp + 1, channels 8 cg .. +8
  const int pp = t & 31, cg = t >> 5;
  const ActView none = {nullptr, 0, 0, 0};
  // image coordinates of the first pixel, advanced by WBK pixels per stage
  int64_t p0 = kbeg + 2 * pp;
  int img = 0, py = 0, px = 0;
  if (p0 < npix) {
    img = (int)(p0 / ((int64_t)H * W));
    const int rem = (int)(p0 - (int64_t)img * H * W);
    py = rem / W;
    px = rem - py * W;
  }
  // loads of the stage at p0 (the thread's two pixels: (img, py, px) and the
  // next one); issued one stage ahead, before the MFMAs of the current one
  // the mask is applied when the stage is written to LDS, so no load waits on another
  const bool masked = mask.p != nullptr;
  uint4 z0, z1, m0, m1, xa[3], xb[3];
  auto fetch = [&]() {
    int img1 = img, py1 = py, px1 = px + 1;
    if (px1 == W) {
      px1 = 0;
      if (++py1 == H) {
        py1 = 0;
        ++img1;
      }
    }
    const bool v0 = p0 < kend, v1 = p0 + 1 < kend;
    z0 = load8(dz, none, none, p0, v0, co0 + 8 * cg);
    z1 = load8(dz, none, none, p0 + 1, v1, co0 + 8 * cg);
    if (masked) {
      m0 = load8(mask, none, none, p0, v0, co0 + 8 * cg);
      m1 = load8(mask, none, none, p0 + 1, v1, co0 + 8 * cg);
    }
    const int sy0 = py + dy, sy1 = py1 + dy;
    const bool r0 = v0 && sy0 >= 0 && sy0 < H, r1 = v1 && sy1 >= 0 && sy1 < H;
    const int64_t row0 = ((int64_t)img * H + sy0) * W, row1 = ((int64_t)img1 * H + sy1) * W;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int sx0 = px + u - 1, sx1 = px1 + u - 1;
      xa[u] = load8(x1, x2, none, row0 + sx0, r0 && sx0 >= 0 && sx0 < W, ci0 + 8 * cg);
      xb[u] = load8(x1, x2, none, row1 + sx1, r1 && sx1 >= 0 && sx1 < W, ci0 + 8 * cg);
    }
    // advance to the next stage (WBK pixels on; rows may be narrower)
    p0 += WBK;
    px += WBK;
    while (px >= W) {
      px -= W;
      if (++py == H) {
        py = 0;
        ++img;
      }
    }
  };
  fetch();
  for (int64_t k0 = kbeg; k0 < kend; k0 += WBK) {
    const uint4 zz0 = masked ? apply_mask8(z0, m0) : z0, zz1 = masked ? apply_mask8(z1, m1) : z1;
    const uint32_t za[4] = {zz0.x, zz0.y, zz0.z, zz0.w}, zb[4] = {zz1.x, zz1.y, zz1.z, zz1.w};
    __syncthreads();
    // transposed into [channel][pixel], two pixels per 32-bit write
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sh = 16 * (q & 1);
      const uint32_t lo_z = (za[q >> 1] >> sh) & 0xFFFFu, hi_z = (zb[q >> 1] >> sh) & 0xFFFFu;
      *reinterpret_cast<uint32_t*>(&sA[(8 * cg + q) * WLDK + 2 * pp]) = lo_z | (hi_z << 16);
      if (do_bias) bacc[q] += bf2f((uint16_t)lo_z) + bf2f((uint16_t)hi_z);
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const uint32_t xw0[4] = {xa[u].x, xa[u].y, xa[u].z, xa[u].w};
      const uint32_t xw1[4] = {xb[u].x, xb[u].y, xb[u].z, xb[u].w};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int sh = 16 * (q & 1);
        const uint32_t lo_x = (xw0[q >> 1] >> sh) & 0xFFFFu, hi_x = (xw1[q >> 1] >> sh) & 0xFFFFu;
        *reinterpret_cast<uint32_t*>(&sB[u][(8 * cg + q) * WLDK + 2 * pp]) = lo_x | (hi_x << 16);
      }
    }
    __syncthreads();
    if (k0 + WBK < kend) fetch();
#pragma unroll
    for (int ks = 0; ks < WBK / 32; ++ks) {
      bf16x8 a[2];
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(
            &sA[(wm + i * 16 + (lane & 15)) * WLDK + 32 * ks + 8 * (lane >> 4)]);
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        bf16x8 b[2];
        for (int j = 0; j < 2; ++j)
          b[j] = *reinterpret_cast<const bf16x8*>(
              &sB[u][(wn + j * 16 + (lane & 15)) * WLDK + 32 * ks + 8 * (lane >> 4)]);
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            acc[u][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[u][i][j], 0, 0, 0);
      }
    }
  }
  for (int u = 0; u < 3; ++u)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        const int ci = ci0 + wn + j * 16 + (lane & 15);
        if (ci >= cin) continue;
        for (int r = 0; r < 4; ++r) {
          const int co = co0 + wm + i * 16 + 4 * (lane >> 4) + r;
          if (co >= cout) continue;
          unsafeAtomicAdd(&dw[((int64_t)(3 * row + u) * cout + co) * cin + ci], acc[u][i][j][r]);
        }
      }
  if (do_bias) {   // block-uniform
    for (int q = 0; q < 8; ++q) s_bias[8 * cg + q][pp] = bacc[q];
    __syncthreads();
    if (t < BM && co0 + t < cout) {
      float sum = 0.f;
      for (int k = 0; k < 32; ++k) sum += s_bias[t][k];
      unsafeAtomicAdd(&dbias[co0 + t], sum);
    }
  }
}

// Weight gradient on spatial tiles: dW[tap][co][ci] = sum over pixels p of
// dz[p][co] x[p + tap][ci] (dz masked by the ReLU of the layer's output).  A
// workgroup owns COB output and 32 input channels and all nine taps, and
// walks a run of 8 x 16-pixel tiles.  Per tile it stages dz transposed to
// [channel][pixel] and the tile's 10 x 18 input patch transposed to
// [channel][row][column] in three copies shifted by 0, 1 and 2 columns, so
// that every tap's operand (8 consecutive pixels of one row per lane) is an
// aligned 16-byte LDS read; the K dimension of the MFMAs is the tile's 128
// pixels.  Wavefront w computes input-channel block w % 2 against output
// blocks (w / 2) and (w / 2) + 2 (COB 64) or block w / 2 (COB 32), for the
// nine taps.  Partial sums go to dW (and dbias) by float atomics at the end.
constexpr int WT_H = 8, WT_W = 16, WT_PX = WT_H * WT_W;   // pixels of a tile
constexpr int WX_H = WT_H + 2, WX_W = WT_W + 2;           // input patch
constexpr int WZ_PITCH = WT_PX + 8;                       // dz^T row pitch (bf16)
constexpr int WX_PITCH = WX_H * WT_W + 8;                 // per-channel pitch of a shifted copy

template <int COB>
__global__ __launch_bounds__(256) void conv3x3_wgrad_patch_kernel(
    ActView x1, ActView x2, ActView dz, ActView mask, int N, int H, int W, int cout, int cin,
    int tiles_per_wg, float* __restrict__ dw, float* __restrict__ dbias) {
  constexpr int NCO = COB / 32;                      // output 16-blocks per wavefront
  // staging items: two horizontally adjacent pixels x 8 channels, so that
  // the transposed LDS writes are 32-bit words, consecutive across a wave
  constexpr int ZI = (COB / 8) * (WT_PX / 2);        // dz items of a tile
  constexpr int ZIT = ZI / 256;                      // per thread
  constexpr int XROW = WX_W / 2;                     // pixel pairs per patch row (9)
  constexpr int XI = 4 * WX_H * XROW;                // input items (32 channels)
  constexpr int XIT = (XI + 255) / 256;
  __shared__ __attribute__((aligned(16))) uint16_t sZ[COB * WZ_PITCH];
  __shared__ __attribute__((aligned(16))) uint16_t sX[3 * 32 * WX_PITCH];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int tiles_x = (W + WT_W - 1) / WT_W, tiles_y = (H + WT_H - 1) / WT_H;
  const int64_t ntiles = (int64_t)N * tiles_x * tiles_y;
  const int co0 = blockIdx.y * COB, ci0 = blockIdx.z * 32;
  const bool do_bias = dbias != nullptr && blockIdx.z == 0;
  const bool masked = mask.p != nullptr;
  const ActView none = {nullptr, 0, 0, 0};
  const int ci_sub = wv & 1, co_blk = wv >> 1;
  f32x4 acc[NCO][9];
#pragma unroll
  for (int c = 0; c < NCO; ++c)
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[c][u] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;   // thread t < COB: bias gradient of output channel co0 + t
  uint4 rz[ZIT][2], rm[ZIT][2], rx[XIT][2];
  auto fetch = [&](int64_t tile) {
    const int img = (int)(tile / (tiles_x * tiles_y));
    const int trem = (int)(tile - (int64_t)img * tiles_x * tiles_y);
    const int ty0 = (trem / tiles_x) * WT_H, tx0 = (trem % tiles_x) * WT_W;
#pragma unroll
    for (int u = 0; u < ZIT; ++u) {            // item: channels 8 (i / 64), pixels 2 (i % 64) + 0, 1
      const int i = t + 256 * u;
      const int cg = i >> 6, p = 2 * (i & 63);
      const int oy = ty0 + p / WT_W, ox = tx0 + p % WT_W;
      const int64_t pix = ((int64_t)img * H + oy) * W + ox;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool inb = oy < H && ox + h < W;
        rz[u][h] = load8(dz, none, none, pix + h, inb, co0 + 8 * cg);
        if (masked) rm[u][h] = load8(mask, none, none, pix + h, inb, co0 + 8 * cg);
      }
    }
#pragma unroll
    for (int u = 0; u < XIT; ++u) {            // item: channels 8 (i / 90), patch row, pixel pair
      const int i = t + 256 * u;
      const int cg = i / (WX_H * XROW), pr = i % (WX_H * XROW);
      const int py = pr / XROW, px = 2 * (pr % XROW);
      const int sy = ty0 + py - 1, sx = tx0 + px - 1;
      const int64_t pix = ((int64_t)img * H + sy) * W + sx;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool inb = i < XI && sy >= 0 && sy < H && sx + h >= 0 && sx + h < W;
        rx[u][h] = load8(x1, x2, none, pix + h, inb, ci0 + 8 * cg);
      }
    }
  };
  // 32-bit word e of two pixels' 8-channel pieces: (pixel 0, pixel 1) of channel e
  auto pair_word = [](const uint4& a, const uint4& b, int e) -> uint32_t {
    const uint32_t wa[4] = {a.x, a.y, a.z, a.w}, wb[4] = {b.x, b.y, b.z, b.w};
    const uint32_t lo = (wa[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
    const uint32_t hi = (wb[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
    return lo | (hi << 16);
  };
  const int64_t t_beg = (int64_t)blockIdx.x * tiles_per_wg;
  const int64_t t_end = min(ntiles, t_beg + tiles_per_wg);
  if (t_beg < t_end) fetch(t_beg);
  for (int64_t tile = t_beg; tile < t_end; ++tile) {
    __syncthreads();   // the previous tile's fragments have been read
#pragma unroll
    for (int u = 0; u < ZIT; ++u) {
      const int i = t + 256 * u;
      const int cg = i >> 6, p = 2 * (i & 63);
      const uint4 v0 = masked ? apply_mask8(rz[u][0], rm[u][0]) : rz[u][0];
      const uint4 v1 = masked ? apply_mask8(rz[u][1], rm[u][1]) : rz[u][1];
#pragma unroll
      for (int e = 0; e < 8; ++e)
        *reinterpret_cast<uint32_t*>(&sZ[(8 * cg + e) * WZ_PITCH + p]) = pair_word(v0, v1, e);
    }
#pragma unroll
    for (int u = 0; u < XIT; ++u) {
      const int i = t + 256 * u;
      if (i >= XI) continue;
      const int cg = i / (WX_H * XROW), pr = i % (WX_H * XROW);
      const int py = pr / XROW, px = 2 * (pr % XROW);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t wd = pair_word(rx[u][0], rx[u][1], e);
        uint16_t* row0 = &sX[(0 * 32 + 8 * cg + e) * WX_PITCH + py * WT_W];
        uint16_t* row1 = &sX[(1 * 32 + 8 * cg + e) * WX_PITCH + py * WT_W];
        uint16_t* row2 = &sX[(2 * 32 + 8 * cg + e) * WX_PITCH + py * WT_W];
        // copy dx holds patch column c + dx at column c: the pair (px, px + 1)
        // lands at columns px, px + 1 (dx 0), px - 2, px - 1 (dx 2) as one
        // word, and at px - 1, px (dx 1) as two halves
        if (px + 1 < WT_W) *reinterpret_cast<uint32_t*>(row0 + px) = wd;
        if (px >= 2) *reinterpret_cast<uint32_t*>(row2 + px - 2) = wd;
        if (px >= 1) row1[px - 1] = (uint16_t)wd;
        if (px < WT_W) row1[px] = (uint16_t)(wd >> 16);
      }
    }
    __syncthreads();
    if (tile + 1 < t_end) fetch(tile + 1);
    if (do_bias && t < COB) {   // the row of dz^T of channel t (zero outside the image)
#pragma unroll 4
      for (int k = 0; k < WT_PX; k += 8) {
        const uint4 v = *reinterpret_cast<const uint4*>(&sZ[t * WZ_PITCH + k]);
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) bacc += bf2f((uint16_t)(w4[e >> 1] >> (16 * (e & 1))));
      }
    }
#pragma unroll
    for (int ks = 0; ks < WT_PX / 32; ++ks) {
      // this lane's 8 pixels of the K step: tile row r, columns c0 .. c0 + 7
      const int p = 32 * ks + 8 * (lane >> 4);
      const int r = p / WT_W, c0 = p % WT_W;
      bf16x8 a[NCO];
#pragma unroll
      for (int c = 0; c < NCO; ++c)
        a[c] = *reinterpret_cast<const bf16x8*>(
            &sZ[((co_blk + 2 * c) * 16 + (lane & 15)) * WZ_PITCH + p]);
#pragma unroll
      for (int u = 0; u < 9; ++u) {
        const int dy = u / 3, dx = u % 3;
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(
            &sX[(dx * 32 + ci_sub * 16 + (lane & 15)) * WX_PITCH + (r + dy) * WT_W + c0]);
#pragma unroll
        for (int c = 0; c < NCO; ++c)
          acc[c][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b, acc[c][u], 0, 0, 0);
      }
    }
  }
  // dW[tap][co][ci]: acc[c][u][r] is output channel (co_blk + 2 c) 16 +
  // 4 (lane / 16) + r, input channel ci_sub 16 + lane % 16
#pragma unroll
  for (int c = 0; c < NCO; ++c)
#pragma unroll
    for (int u = 0; u < 9; ++u) {
      const int ci = ci0 + ci_sub * 16 + (lane & 15);
      if (ci >= cin) continue;
      for (int r = 0; r < 4; ++r) {
        const int co = co0 + (co_blk + 2 * c) * 16 + 4 * (lane >> 4) + r;
        if (co < cout) unsafeAtomicAdd(&dw[((int64_t)u * cout + co) * cin + ci], acc[c][u][r]);
      }
    }
  if (do_bias && t < COB && co0 + t < cout) unsafeAtomicAdd(&dbias[co0 + t], bacc);
}

// Narrow weight gradient (cout <= 32): a 32 x 32 channel tile for one row
// of three taps (dy fixed, dx = -1, 0, 1), so each stage's dz and mask loads
// serve three taps.  The four wavefronts split the workgroup's pixels (wave
// w takes every fourth 64-pixel stage), each staging through its own LDS
// region, so only wave-level ordering is needed; the four partial tiles are
// summed once at the end.  Lane l stages pixels 2 (l % 32), 2 (l % 32) + 1
// and channel groups (l / 32) + 2 g, g = 0, 1, of dz and of the three
// shifted inputs.
__global__ __launch_bounds__(256) void conv3x3_wgrad32_kernel(
    ActView x1, ActView x2, ActView dz, ActView mask, int N, int H, int W, int cout, int cin,
    int64_t kchunk, float* __restrict__ dw, float* __restrict__ dbias) {
  __shared__ __attribute__((aligned(16))) union {
    struct {
      uint16_t a[4][32 * WLDK];      // per wave [co][pixel]
      uint16_t b[4][3][32 * WLDK];   // per wave and tap [ci][pixel]
    } st;
    float red[4][3][32][33];         // after the pixel loop: the four waves' tiles
  } sm;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t npix = (int64_t)N * H * W;
  const int row = blockIdx.y % 3;
  const int ci0 = (blockIdx.y / 3) * 32;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = min(npix, kbeg + kchunk);
  const int dy = row - 1;
  const bool do_bias = dbias != nullptr && row == 1 && ci0 == 0;
  const int pp = lane & 31, gh = lane >> 5;
  const ActView none = {nullptr, 0, 0, 0};
  f32x4 acc[3][2][2];
  for (int u = 0; u < 3; ++u)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[u][i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float bacc[16];
  for (int q = 0; q < 16; ++q) bacc[q] = 0.f;
  uint16_t* a_s = sm.st.a[wv];
  const bool masked = mask.p != nullptr;
  // image coordinates of the lane's first pixel, advanced by 4 WBK pixels
  // per stage (the stride of one wavefront)
  int64_t p0 = kbeg + (int64_t)wv * WBK + 2 * pp;
  int img = 0, py = 0, px = 0;
  if (p0 < npix) {
    img = (int)(p0 / ((int64_t)H * W));
    const int rem = (int)(p0 - (int64_t)img * H * W);
    py = rem / W;
    px = rem - py * W;
  }
  // [pixel][group] ([tap][pixel][group] for the input), loaded one stage
  // ahead; the mask is applied when the stage is written to LDS, so no load
  // waits on another
  uint4 z[2][2], zm[2][2], xv[3][2][2];
  auto fetch = [&]() {
    int img1 = img, py1 = py, px1 = px + 1;
    if (px1 == W) {
      px1 = 0;
      if (++py1 == H) {
        py1 = 0;
        ++img1;
      }
    }
    const bool v0 = p0 < kend, v1 = p0 + 1 < kend;
    const int sy0 = py + dy, sy1 = py1 + dy;
    const bool r0 = v0 && sy0 >= 0 && sy0 < H, r1 = v1 && sy1 >= 0 && sy1 < H;
    const int64_t row0 = ((int64_t)img * H + sy0) * W, row1 = ((int64_t)img1 * H + sy1) * W;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int cg = gh + 2 * g;   // channel group 0..3
      z[0][g] = load8(dz, none, none, p0, v0, 8 * cg);
      z[1][g] = load8(dz, none, none, p0 + 1, v1, 8 * cg);
      if (masked) {
        zm[0][g] = load8(mask, none, none, p0, v0, 8 * cg);
        zm[1][g] = load8(mask, none, none, p0 + 1, v1, 8 * cg);
      }
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int sx0 = px + u - 1, sx1 = px1 + u - 1;
        xv[u][0][g] = load8(x1, x2, none, row0 + sx0, r0 && sx0 >= 0 && sx0 < W, ci0 + 8 * cg);
        xv[u][1][g] = load8(x1, x2, none, row1 + sx1, r1 && sx1 >= 0 && sx1 < W, ci0 + 8 * cg);
      }
    }
    p0 += 4 * WBK;
    px += 4 * WBK;
    while (px >= W) {
      px -= W;
      if (++py == H) {
        py = 0;
        ++img;
      }
    }
  };
  fetch();
  for (int64_t k0 = kbeg + (int64_t)wv * WBK; k0 < kend; k0 += 4 * WBK) {
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int cg = gh + 2 * g;
      const uint4 z0 = masked ? apply_mask8(z[0][g], zm[0][g]) : z[0][g];
      const uint4 z1 = masked ? apply_mask8(z[1][g], zm[1][g]) : z[1][g];
      const uint32_t za[4] = {z0.x, z0.y, z0.z, z0.w};
      const uint32_t zb[4] = {z1.x, z1.y, z1.z, z1.w};
      // transposed into [channel][pixel], two pixels per 32-bit write
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int sh = 16 * (q & 1);
        const uint32_t lo_z = (za[q >> 1] >> sh) & 0xFFFFu, hi_z = (zb[q >> 1] >> sh) & 0xFFFFu;
        *reinterpret_cast<uint32_t*>(&a_s[(8 * cg + q) * WLDK + 2 * pp]) = lo_z | (hi_z << 16);
        if (do_bias) bacc[8 * g + q] += bf2f((uint16_t)lo_z) + bf2f((uint16_t)hi_z);
      }
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const uint32_t xa[4] = {xv[u][0][g].x, xv[u][0][g].y, xv[u][0][g].z, xv[u][0][g].w};
        const uint32_t xb[4] = {xv[u][1][g].x, xv[u][1][g].y, xv[u][1][g].z, xv[u][1][g].w};
        uint16_t* b_s = sm.st.b[wv][u];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int sh = 16 * (q & 1);
          const uint32_t lo_x = (xa[q >> 1] >> sh) & 0xFFFFu, hi_x = (xb[q >> 1] >> sh) & 0xFFFFu;
          *reinterpret_cast<uint32_t*>(&b_s[(8 * cg + q) * WLDK + 2 * pp]) = lo_x | (hi_x << 16);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (k0 + 4 * WBK < kend) fetch();
#pragma unroll
    for (int ks = 0; ks < WBK / 32; ++ks) {
      bf16x8 a[2];
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(&a_s[(i * 16 + (lane & 15)) * WLDK + 32 * ks + 8 * (lane >> 4)]);
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const uint16_t* b_s = sm.st.b[wv][u];
        bf16x8 b[2];
        for (int j = 0; j < 2; ++j)
          b[j] = *reinterpret_cast<const bf16x8*>(&b_s[(j * 16 + (lane & 15)) * WLDK + 32 * ks + 8 * (lane >> 4)]);
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j)
            acc[u][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[u][i][j], 0, 0, 0);
      }
    }
    __builtin_amdgcn_wave_barrier();   // fragments read before the next stage's writes
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
  // sum the four wavefronts' tiles: red[w][u][co][ci] (over the staging buffers)
  __syncthreads();
  float(*s_red)[3][32][33] = sm.red;
  for (int u = 0; u < 3; ++u)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int r = 0; r < 4; ++r)
          s_red[wv][u][i * 16 + 4 * (lane >> 4) + r][j * 16 + (lane & 15)] = acc[u][i][j][r];
  __syncthreads();
  for (int e = t; e < 3 * 32 * 32; e += 256) {
    const int u = e >> 10, co = (e >> 5) & 31, ci = e & 31;
    if (co >= cout || ci0 + ci >= cin) continue;
    const float v = s_red[0][u][co][ci] + s_red[1][u][co][ci] + s_red[2][u][co][ci] + s_red[3][u][co][ci];
    unsafeAtomicAdd(&dw[((int64_t)(3 * row + u) * cout + co) * cin + ci0 + ci], v);
  }
  if (do_bias) {   // block-uniform
    __syncthreads();   // s_red is reused for the per-wave channel sums
    float* sb = &s_red[0][0][0][0];
    for (int q = 0; q < 16; ++q) {
      float v = bacc[q];
      for (int d = 1; d < 32; d <<= 1) v += __shfl_xor(v, d, 64);   // over the 32 pixel pairs
      bacc[q] = v;
    }
    if (pp == 0)
      for (int g = 0; g < 2; ++g)
        for (int q = 0; q < 8; ++q) sb[wv * 32 + 8 * (gh + 2 * g) + q] = bacc[8 * g + q];
    __syncthreads();
    if (t < 32 && t < cout)
      unsafeAtomicAdd(&dbias[t], sb[t] + sb[32 + t] + sb[64 + t] + sb[96 + t]);
  }
}

// w [9][cout][cin] -> wt [9][cin][cout] with taps mirrored (backward data)
__global__ void flip_weights_kernel(const uint16_t* __restrict__ w, int cout, int cin,
                                    uint16_t* __restrict__ wt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = 9LL * cout * cin;
  if (i >= total) return;
  const int tap = (int)(i / ((int64_t)cout * cin));
  const int rem = (int)(i - (int64_t)tap * cout * cin);
  const int co = rem / cin, ci = rem % cin;
  wt[((int64_t)(8 - tap) * cin + ci) * cout + co] = w[i];
}

__device__ __forceinline__ void unpack8(uint4 u, float* v) {
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
  for (int k = 0; k < 4; ++k) {
    v[2 * k] = bf2f((uint16_t)(w[k] & 0xFFFFu));
    v[2 * k + 1] = bf2f((uint16_t)(w[k] >> 16));
  }
}

__device__ __forceinline__ uint4 pack8(const float* v) {
  uint32_t w[4];
  for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf(v[2 * k]) | ((uint32_t)f2bf(v[2 * k + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// 8 channels per thread (channel counts, strides and offsets are multiples of 8)
__global__ void avgpool2_kernel(ActView x, int N, int H, int W, uint16_t* __restrict__ y,
                                int y_stride) {
  const int Ho = H / 2, Wo = W / 2;
  const int c8n = x.c / 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * Ho * Wo * c8n;
  if (i >= total) return;
  const int c = (int)(i % c8n) * 8;
  const int64_t q = i / c8n;
  const int n = (int)(q / ((int64_t)Ho * Wo));
  const int r = (int)(q - (int64_t)n * Ho * Wo);
  const int yo = r / Wo, xo = r % Wo;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int64_t p = ((int64_t)n * H + 2 * yo + a) * W + 2 * xo + b;
      float v[8];
      unpack8(*reinterpret_cast<const uint4*>(x.p + p * x.stride + x.offset + c), v);
      for (int k = 0; k < 8; ++k) s[k] += v[k];
    }
  for (int k = 0; k < 8; ++k) s[k] *= 0.25f;
  *reinterpret_cast<uint4*>(y + q * y_stride + c) = pack8(s);
}

// dx[p][c] (+)= dy[pool(p)][c] / 4 (dx may be a channel slice; accumulate adds)
// 8 channels per thread (see upsample2_kernel)
__global__ void avgpool2_bwd_kernel(ActView dy, int N, int H, int W, uint16_t* __restrict__ dx,
                                    int dx_stride, int dx_offset, int accumulate,
                                    const uint16_t* __restrict__ add_src, int add_stride,
                                    int add_offset) {
  const int c8n = dy.c / 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * H * W * c8n;
  if (i >= total) return;
  const int c = (int)(i % c8n) * 8;
  const int64_t p = i / c8n;
  const int n = (int)(p / ((int64_t)H * W));
  const int r = (int)(p - (int64_t)n * H * W);
  const int yy = r / W, xx = r % W;
  const int Ho = H / 2, Wo = W / 2;
  float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (yy / 2 < Ho && xx / 2 < Wo) {
    const int64_t q = ((int64_t)n * Ho + yy / 2) * Wo + xx / 2;
    unpack8(*reinterpret_cast<const uint4*>(dy.p + q * dy.stride + dy.offset + c), v);
    for (int k = 0; k < 8; ++k) v[k] *= 0.25f;
  }
  if (add_src) {
    float a[8];
    unpack8(*reinterpret_cast<const uint4*>(add_src + p * add_stride + add_offset + c), a);
    for (int k = 0; k < 8; ++k) v[k] += a[k];
  }
  uint4* o = reinterpret_cast<uint4*>(dx + p * dx_stride + dx_offset + c);
  if (accumulate) {
    float cur[8];
    unpack8(*o, cur);
    for (int k = 0; k < 8; ++k) v[k] = cur[k] + v[k];
  }
  *o = pack8(v);
}

// 8 channels (16 bytes) per thread; channel counts, strides and offsets are
// multiples of 8.
__global__ void upsample2_kernel(ActView x, int N, int H, int W, uint16_t* __restrict__ y,
                                 int y_stride, int y_offset) {
  // x is (H/2) x (W/2); y is H x W
  const int c8n = x.c / 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * H * W * c8n;
  if (i >= total) return;
  const int c = (int)(i % c8n) * 8;
  const int64_t p = i / c8n;
  const int n = (int)(p / ((int64_t)H * W));
  const int r = (int)(p - (int64_t)n * H * W);
  const int yy = r / W, xx = r % W;
  const int64_t q = ((int64_t)n * (H / 2) + yy / 2) * (W / 2) + xx / 2;
  *reinterpret_cast<uint4*>(y + p * y_stride + y_offset + c) =
      *reinterpret_cast<const uint4*>(x.p + q * x.stride + x.offset + c);
}

// 8 channels per thread (see avgpool2_kernel)
__global__ void upsample2_bwd_kernel(ActView dy, int N, int H, int W, uint16_t* __restrict__ dx,
                                     int dx_stride) {
  // dy is H x W, dx is (H/2) x (W/2): dx = sum of the 2x2 block
  const int Ho = H / 2, Wo = W / 2;
  const int c8n = dy.c / 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * Ho * Wo * c8n;
  if (i >= total) return;
  const int c = (int)(i % c8n) * 8;
  const int64_t q = i / c8n;
  const int n = (int)(q / ((int64_t)Ho * Wo));
  const int r = (int)(q - (int64_t)n * Ho * Wo);
  const int yo = r / Wo, xo = r % Wo;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int64_t p = ((int64_t)n * H + 2 * yo + a) * W + 2 * xo + b;
      float v[8];
      unpack8(*reinterpret_cast<const uint4*>(dy.p + p * dy.stride + dy.offset + c), v);
      for (int k = 0; k < 8; ++k) s[k] += v[k];
    }
  *reinterpret_cast<uint4*>(dx + q * dx_stride + c) = pack8(s);
}

// planar float32 RGB [N][3][H][W] -> NHWC bf16 with `stride` channels (zero padded)
__global__ void rgb_to_nhwc_kernel(const float* __restrict__ rgb, int N, int H, int W,
                                   uint16_t* __restrict__ x, int stride) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)N * H * W;
  if (p >= npix) return;
  const int n = (int)(p / ((int64_t)H * W));
  const int64_t r = p - (int64_t)n * H * W;
  for (int c = 0; c < stride; ++c)
    x[p * stride + c] = c < 3 ? f2bf(rgb[((int64_t)n * 3 + c) * H * W + r]) : (uint16_t)0;
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = f2bf(src[i]);
}

// Per-pixel head on float32 features [p][2] (a 1x1 conv already applied by
// conv3x3 with a 1x1 kernel would waste 8/9 of the work; the head is a 1x1
// conv): out[n][k][y][x] = b[k] + sum_c w[k][c] f[p][c].
__global__ void head_fwd_kernel(ActView f, int N, int H, int W, const float* __restrict__ w,
                                const float* __restrict__ b, float* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)N * H * W;
  if (p >= npix) return;
  float o0 = b[0], o1 = b[1];
  for (int c = 0; c < f.c; ++c) {
    const float v = bf2f(f.p[p * f.stride + f.offset + c]);
    o0 += w[c] * v;
    o1 += w[f.c + c] * v;
  }
  const int n = (int)(p / ((int64_t)H * W));
  const int64_t r = p - (int64_t)n * H * W;
  out[((int64_t)n * 2 + 0) * H * W + r] = o0;
  out[((int64_t)n * 2 + 1) * H * W + r] = o1;
}

// The same with 16-byte loads when the channels come in whole groups of 8
// (count, stride and offset multiples of 8): a thread reads its pixel's
// features 8 at a time, the sums run over the channels in the same order.
__global__ __launch_bounds__(256) void head_fwd8_kernel(ActView f, int N, int H, int W,
                                                        const float* __restrict__ w,
                                                        const float* __restrict__ b,
                                                        float* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)N * H * W;
  if (p >= npix) return;
  const uint16_t* src = f.p + p * f.stride + f.offset;
  float o0 = b[0], o1 = b[1];
  for (int c = 0; c < f.c; c += 8) {
    const uint4 v = *reinterpret_cast<const uint4*>(src + c);
    const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float lo = __uint_as_float(wd[i] << 16), hi = __uint_as_float(wd[i] & 0xFFFF0000u);
      o0 += w[c + 2 * i] * lo;
      o1 += w[f.c + c + 2 * i] * lo;
      o0 += w[c + 2 * i + 1] * hi;
      o1 += w[f.c + c + 2 * i + 1] * hi;
    }
  }
  const int n = (int)(p / ((int64_t)H * W));
  const int64_t r = p - (int64_t)n * H * W;
  out[((int64_t)n * 2 + 0) * H * W + r] = o0;
  out[((int64_t)n * 2 + 1) * H * W + r] = o1;
}

// Head backward: dF[p][c] = sum_k w[k][c] dout[k][p] masked by the feature's
// ReLU (f > 0); dW, db accumulated with per-block reductions and atomics.
// Threads (channel lane t % 32, pixel group t / 32): each thread walks every
// eighth pixel of the workgroup's 256-pixel chunks (grid-stride), handling
// channels t % 32 + 32 k; the weight and bias partials stay in registers and
// are reduced over the eight groups once per workgroup.
constexpr int kHeadMaxSlots = 2;   // channels per thread: up to 64 feature channels (the C ABI limit)

__global__ __launch_bounds__(256) void head_bwd_kernel(ActView f, int N, int H, int W,
                                                       const float* __restrict__ w,
                                                       const float* __restrict__ dout,
                                                       uint16_t* __restrict__ df, int df_stride,
                                                       float* __restrict__ dw,
                                                       float* __restrict__ db) {
  __shared__ float s_red[8][2 * 32 * kHeadMaxSlots + 2];
  const int t = threadIdx.x, cl = t & 31, pg = t >> 5;
  const int64_t npix = (int64_t)N * H * W;
  const int64_t hw = (int64_t)H * W;
  const int slots = (f.c + 31) / 32;
  float a0[kHeadMaxSlots], a1[kHeadMaxSlots], w0[kHeadMaxSlots], w1[kHeadMaxSlots];
  for (int k = 0; k < kHeadMaxSlots; ++k) {
    a0[k] = a1[k] = 0.f;
    const int c = cl + 32 * k;
    w0[k] = (k < slots && c < f.c) ? w[c] : 0.f;
    w1[k] = (k < slots && c < f.c) ? w[f.c + c] : 0.f;
  }
  float b0 = 0.f, b1 = 0.f;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < npix; base += (int64_t)gridDim.x * 256) {
    for (int j = pg; j < 256; j += 8) {
      const int64_t p = base + j;
      if (p >= npix) break;
      const int n = (int)(p / hw);
      const int64_t r = p - (int64_t)n * hw;
      const float g0 = dout[((int64_t)n * 2 + 0) * hw + r];
      const float g1 = dout[((int64_t)n * 2 + 1) * hw + r];
      if (cl == 0) {
        b0 += g0;
        b1 += g1;
      }
      for (int k = 0; k < kHeadMaxSlots; ++k) {
        const int c = cl + 32 * k;
        if (k >= slots || c >= f.c) break;
        const float v = bf2f(f.p[p * f.stride + f.offset + c]);
        a0[k] += g0 * v;
        a1[k] += g1 * v;
        df[p * df_stride + c] = f2bf(v > 0.f ? (w0[k] * g0 + w1[k] * g1) : 0.f);
      }
    }
  }
  for (int k = 0; k < kHeadMaxSlots; ++k) {
    s_red[pg][32 * k + cl] = a0[k];
    s_red[pg][32 * kHeadMaxSlots + 32 * k + cl] = a1[k];
  }
  if (cl == 0) {
    s_red[pg][64 * kHeadMaxSlots] = b0;
    s_red[pg][64 * kHeadMaxSlots + 1] = b1;
  }
  __syncthreads();
  for (int k = t; k < 2 * f.c + 2; k += 256) {
    // k < f.c: dw row 0; f.c <= k < 2 f.c: dw row 1; then the two biases
    const int col = k < f.c ? k : k < 2 * f.c ? 32 * kHeadMaxSlots + (k - f.c)
                                              : 64 * kHeadMaxSlots + (k - 2 * f.c);
    float sum = 0.f;
    for (int g = 0; g < 8; ++g) sum += s_red[g][col];
    if (k < 2 * f.c)
      unsafeAtomicAdd(&dw[k], sum);
    else
      unsafeAtomicAdd(&db[k - 2 * f.c], sum);
  }
}

// Head backward with 16-byte accesses (channel counts, strides and offsets
// multiples of 8): thread t owns channel group t % G (8 channels, G = C / 8)
// of pixel t / G of each 256 / G-pixel step (grid-stride), loads and stores
// its 8 features and gradients at once, and keeps 16 weight partials in
// registers; the partials of a group are summed over the workgroup in LDS
// once, then added with one atomic per weight.
constexpr int kHead8Groups = 8;   // up to 64 channels

__global__ __launch_bounds__(256) void head_bwd8_kernel(ActView f, int N, int H, int W,
                                                        const float* __restrict__ w,
                                                        const float* __restrict__ dout,
                                                        uint16_t* __restrict__ df, int df_stride,
                                                        float* __restrict__ dw,
                                                        float* __restrict__ db) {
  __shared__ float s_red[256][19];
  const int t = threadIdx.x;
  const int G = f.c / 8;
  const int per = 256 / G;          // pixels per step
  const int cg = t % G, pix = t / G;
  const bool active = pix < per;    // 256 not a multiple of G: the last threads idle
  const int64_t npix = (int64_t)N * H * W;
  const int64_t hw = (int64_t)H * W;
  float w0[8], w1[8], a0[8], a1[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    w0[i] = w[8 * cg + i];
    w1[i] = w[f.c + 8 * cg + i];
    a0[i] = a1[i] = 0.f;
  }
  float b0 = 0.f, b1 = 0.f;
  if (active) {
    for (int64_t p = (int64_t)blockIdx.x * per + pix; p < npix; p += (int64_t)gridDim.x * per) {
      const int n = (int)(p / hw);
      const int64_t r = p - (int64_t)n * hw;
      const float g0 = dout[((int64_t)n * 2 + 0) * hw + r];
      const float g1 = dout[((int64_t)n * 2 + 1) * hw + r];
      if (cg == 0) {
        b0 += g0;
        b1 += g1;
      }
      const uint4 v = *reinterpret_cast<const uint4*>(f.p + p * f.stride + f.offset + 8 * cg);
      const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
      uint32_t od[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float lo = __uint_as_float(wd[i] << 16), hi = __uint_as_float(wd[i] & 0xFFFF0000u);
        a0[2 * i] += g0 * lo;
        a1[2 * i] += g1 * lo;
        a0[2 * i + 1] += g0 * hi;
        a1[2 * i + 1] += g1 * hi;
        const uint16_t dlo = f2bf(lo > 0.f ? (w0[2 * i] * g0 + w1[2 * i] * g1) : 0.f);
        const uint16_t dhi = f2bf(hi > 0.f ? (w0[2 * i + 1] * g0 + w1[2 * i + 1] * g1) : 0.f);
        od[i] = (uint32_t)dlo | ((uint32_t)dhi << 16);
      }
      *reinterpret_cast<uint4*>(df + p * df_stride + 8 * cg) = make_uint4(od[0], od[1], od[2], od[3]);
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    s_red[t][i] = a0[i];
    s_red[t][8 + i] = a1[i];
  }
  s_red[t][16] = b0;   // nonzero in the group-0 threads only
  s_red[t][17] = b1;
  __syncthreads();
  // weight (row, channel 8 g + i): the sum over the threads of group g;
  // bias k: the sum over the group-0 threads
  for (int k = t; k < 2 * f.c + 2; k += 256) {
    float sum = 0.f;
    if (k < 2 * f.c) {
      const int row = k / f.c, c = k - row * f.c, g = c / 8, i = c % 8;
      for (int u = g; u < per * G; u += G) sum += s_red[u][8 * row + i];
      unsafeAtomicAdd(&dw[k], sum);
    } else {
      for (int u = 0; u < per * G; u += G) sum += s_red[u][16 + (k - 2 * f.c)];
      unsafeAtomicAdd(&db[k - 2 * f.c], sum);
    }
  }
}

// Depth supervision: pred [N][2][H][W] = (log depth, log scale); target depth
// [N][H][W] (<= 0 marks invalid); log-scale target log(depth / fx).
// loss = mean over valid of |pred0 - log d| + |pred1 - log(d / fx)|.
__global__ __launch_bounds__(256) void depth_loss_kernel(const float* __restrict__ pred,
                                                         const float* __restrict__ depth, int N,
                                                         int H, int W, float fx,
                                                         const int* __restrict__ count,
                                                         float* __restrict__ dpred,
                                                         double* __restrict__ loss) {
  __shared__ float s_acc[4];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npix = (int64_t)N * H * W;
  float l = 0.f;
  if (p < npix) {
    const int n = (int)(p / ((int64_t)H * W));
    const int64_t r = p - (int64_t)n * H * W;
    const float d = depth[p];
    const float inv = 1.0f / (float)max(*count, 1);
    float g0 = 0.f, g1 = 0.f;
    if (d > 0.f) {
      const float ld = logf(d), ls = logf(d / fx);
      const float e0 = pred[((int64_t)n * 2 + 0) * H * W + r] - ld;
      const float e1 = pred[((int64_t)n * 2 + 1) * H * W + r] - ls;
      l = (fabsf(e0) + fabsf(e1)) * inv;
      g0 = e0 > 0.f ? inv : (e0 < 0.f ? -inv : 0.f);
      g1 = e1 > 0.f ? inv : (e1 < 0.f ? -inv : 0.f);
    }
    dpred[((int64_t)n * 2 + 0) * H * W + r] = g0;
    dpred[((int64_t)n * 2 + 1) * H * W + r] = g1;
  }
  for (int d = 32; d > 0; d >>= 1) l += __shfl_xor(l, d, 64);
  if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, (double)(s_acc[0] + s_acc[1] + s_acc[2] + s_acc[3]));
}

__global__ void count_valid_kernel(const float* __restrict__ depth, int64_t n,
                                   int* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = (i < n && depth[i] > 0.f) ? 1 : 0;
  for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

__global__ void zero_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

ActView view(const gs_act* a) {
  ActView v{nullptr, 0, 0, 0};
  if (a) {
    v.p = static_cast<const uint16_t*>(a->data);
    v.c = a->c;
    v.stride = a->stride;
    v.offset = a->offset;
  }
  return v;
}

unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// The unmasked patch convolution is persistent: as many workgroups as the
// device holds at once (split over the channel tiles), never more than there
// are tiles.
template <int BNT, bool MASKED>
hipError_t launch_patch(ActView x1, ActView x2, ActView mask, int n, int h, int w,
                        const uint16_t* wp, int cout, int cin, const float* bias, int relu,
                        uint16_t* yp, int ys, int yo, float* yf, int yf_stride, unsigned tiles,
                        hipStream_t s) {
  const unsigned gy = (unsigned)((cout + BNT - 1) / BNT);
  const int resident = resident_workgroups((const void*)conv3x3_patch_kernel<BNT, MASKED>, 256);
  unsigned gx = tiles;   // masked calls: one tile per workgroup
  if (!MASKED && resident > 0)
    gx = std::min(tiles, std::max(1u, ((unsigned)resident + gy - 1) / gy));
  hipLaunchKernelGGL((conv3x3_patch_kernel<BNT, MASKED>), dim3(gx, gy), dim3(256), 0, s, x1, x2,
                     mask, n, h, w, wp, cout, cin, bias, relu, yp, ys, yo, yf, yf_stride);
  return hipGetLastError();
}

}  // namespace

hipError_t nn_conv3x3(const gs_act* x1, const gs_act* x2, const gs_act* mask, const void* w,
                      int cout, const float* bias, int relu, gs_act* y, float* yf, int yf_stride,
                      hipStream_t s) {
  const int cin = x1->c + (x2 ? x2->c : 0);
  const int64_t npix = (int64_t)x1->n * x1->h * x1->w;
  // Tiles: up to 32 output channels, 32-channel tiles (a 64-channel tile
  // would spend half its MFMAs on channels that do not exist); 64 x 32
  // wavefront blocks while that still gives about 1,024 workgroups, else
  // 32 x 32 ones (twice the workgroups for the small deep layers).
  auto* yp = y ? static_cast<uint16_t*>(y->data) : nullptr;
  const int ys = y ? y->stride : 0, yo = y ? y->offset : 0;
  const auto* wp = static_cast<const uint16_t*>(w);
  if (cin % 8 == 0 && x1->c % 8 == 0) {
    const unsigned tiles = (unsigned)(x1->n * ((x1->h + PT - 1) / PT) * ((x1->w + PT - 1) / PT));
    // 32 output channels per workgroup up to 32 channels, for an odd number
    // of 32-channel groups (96 channels in 64-channel tiles would waste a
    // quarter of the products), and also where 64-channel workgroups would
    // number fewer than 1,024: twice the workgroups, and at 49 KB of LDS three
    // fit a CU (72 KB: two); measured 3% faster on the forward pass of four
    // 640x480 images, and the 96-channel backward-data call 2% of the backward
    const bool narrow =
        cout <= 32 || cout % 64 == 32 || tiles * (unsigned)((cout + 63) / 64) < 1024u;
#define GS_PATCH(B, M)                                                                     \
  launch_patch<B, M>(view(x1), view(x2), view(mask), x1->n, x1->h, x1->w, wp, cout, cin, bias, \
                     relu, yp, ys, yo, yf, yf_stride, tiles, s)
    if (narrow) return mask ? GS_PATCH(32, true) : GS_PATCH(32, false);
    return mask ? GS_PATCH(64, true) : GS_PATCH(64, false);
#undef GS_PATCH
  }
  const unsigned ntile = (unsigned)((cout + 63) / 64);
  // (the masked backward-data calls measured faster without the large tiles)
  const bool narrow = cout <= 32;
  const bool big = mask == nullptr &&
                   (int64_t)blocks(npix, narrow ? 256 : 128) * (narrow ? 1 : ntile) >= 1024;
  if (narrow && big)
    hipLaunchKernelGGL((conv3x3_kernel<256, 32, 4>), dim3(blocks(npix, 256), 1), dim3(256), 0, s,
                       view(x1), view(x2), view(mask), x1->n, x1->h, x1->w, wp, cout, cin, bias,
                       relu, yp, ys, yo, yf, yf_stride);
  else if (narrow)
    hipLaunchKernelGGL((conv3x3_kernel<128, 32, 2>), dim3(blocks(npix, 128), 1), dim3(256), 0, s,
                       view(x1), view(x2), view(mask), x1->n, x1->h, x1->w, wp, cout, cin, bias,
                       relu, yp, ys, yo, yf, yf_stride);
  else if (big)
    hipLaunchKernelGGL((conv3x3_kernel<128, 64, 4>), dim3(blocks(npix, 128), ntile), dim3(256), 0,
                       s, view(x1), view(x2), view(mask), x1->n, x1->h, x1->w, wp, cout, cin, bias,
                       relu, yp, ys, yo, yf, yf_stride);
  else
    hipLaunchKernelGGL((conv3x3_kernel<64, 64, 2>), dim3(blocks(npix, 64), ntile), dim3(256), 0,
                       s, view(x1), view(x2), view(mask), x1->n, x1->h, x1->w, wp, cout, cin, bias,
                       relu, yp, ys, yo, yf, yf_stride);
  return hipGetLastError();
}

hipError_t nn_conv3x3_wgrad(const gs_act* x1, const gs_act* x2, const gs_act* dz,
                            const gs_act* mask, float* dw, float* dbias, hipStream_t s) {
  const int cin = x1->c + (x2 ? x2->c : 0);
  const int cout = dz->c;
  const int64_t npix = (int64_t)x1->n * x1->h * x1->w;
  if (cout <= 32 && cin % 8 == 0 && x1->c % 8 == 0 && cout % 8 == 0) {
    // narrow layers (the full-resolution ones): spatial tiles; for wider
    // layers the 64 x 64 channel tiles below measured faster (their MFMA
    // work per staged byte is larger, and the tile kernel at 64 output
    // channels holds two workgroups per CU)
    const int64_t ntiles = (int64_t)x1->n * ((x1->h + WT_H - 1) / WT_H) * ((x1->w + WT_W - 1) / WT_W);
    const int64_t blocks_ch = (cin + 31) / 32;
    // runs of tiles: about 1,024 workgroups, each long enough that its
    // 9 x 32 x 32 closing atomics are few next to its MFMA work
    const int64_t per = std::max<int64_t>(4, (ntiles * blocks_ch + 1023) / 1024);
    const dim3 grid((unsigned)((ntiles + per - 1) / per), 1u, (unsigned)blocks_ch);
    hipLaunchKernelGGL(conv3x3_wgrad_patch_kernel<32>, grid, dim3(256), 0, s, view(x1), view(x2),
                       view(dz), view(mask), x1->n, x1->h, x1->w, cout, cin, (int)per, dw, dbias);
    return hipGetLastError();
  }
  // pixel chunks: enough workgroups to fill the chip, each long enough that
  // its 4096 atomic adds into dw are few next to its MFMA work
  if (cout <= 32) {   // 32 x 32 channel tiles, a row of taps each (see conv3x3_wgrad32_kernel)
    const int64_t tiles = 3 * (int64_t)((cin + 31) / 32);
    const int64_t nk = std::max<int64_t>(1, kWgrad32Blocks / tiles);
    int64_t kchunk = (npix + nk - 1) / nk;
    kchunk = std::max<int64_t>(4 * WBK, (kchunk + 4 * WBK - 1) / (4 * WBK) * (4 * WBK));
    const dim3 grid(1, (unsigned)(3 * ((cin + 31) / 32)), (unsigned)((npix + kchunk - 1) / kchunk));
    hipLaunchKernelGGL(conv3x3_wgrad32_kernel, grid, dim3(256), 0, s, view(x1), view(x2),
                       view(dz), view(mask), x1->n, x1->h, x1->w, cout, cin, kchunk, dw, dbias);
    return hipGetLastError();
  }
  const int64_t tiles = (int64_t)((cout + BM - 1) / BM) * 3 * ((cin + BN - 1) / BN);
  const int64_t nk = std::max<int64_t>(1, kWgradBlocks / tiles);
  int64_t kchunk = (npix + nk - 1) / nk;
  kchunk = std::max<int64_t>(WBK, (kchunk + WBK - 1) / WBK * WBK);
  const dim3 grid((unsigned)((cout + BM - 1) / BM), (unsigned)(3 * ((cin + BN - 1) / BN)),
                  (unsigned)((npix + kchunk - 1) / kchunk));
  hipLaunchKernelGGL(conv3x3_wgrad_kernel, grid, dim3(256), 0, s, view(x1), view(x2), view(dz),
                     view(mask), x1->n, x1->h, x1->w, cout, cin, kchunk, dw, dbias);
  return hipGetLastError();
}

hipError_t nn_flip_weights(const void* w, int cout, int cin, void* wt, hipStream_t s) {
  hipLaunchKernelGGL(flip_weights_kernel, dim3(blocks(9LL * cout * cin)), dim3(256), 0, s,
                     static_cast<const uint16_t*>(w), cout, cin, static_cast<uint16_t*>(wt));
  return hipGetLastError();
}

hipError_t nn_avgpool2(const gs_act* x, gs_act* y, hipStream_t s) {
  const int64_t total = (int64_t)x->n * (x->h / 2) * (x->w / 2) * (x->c / 8);
  hipLaunchKernelGGL(avgpool2_kernel, dim3(blocks(total)), dim3(256), 0, s, view(x), x->n, x->h,
                     x->w, static_cast<uint16_t*>(y->data) + y->offset, y->stride);
  return hipGetLastError();
}

hipError_t nn_avgpool2_bwd(const gs_act* dy, const gs_act* add, gs_act* dx, int accumulate,
                           hipStream_t s) {
  const int64_t total = (int64_t)dx->n * dx->h * dx->w * (dy->c / 8);
  hipLaunchKernelGGL(avgpool2_bwd_kernel, dim3(blocks(total)), dim3(256), 0, s, view(dy), dx->n,
                     dx->h, dx->w, static_cast<uint16_t*>(dx->data), dx->stride, dx->offset,
                     accumulate, add ? static_cast<const uint16_t*>(add->data) : nullptr,
                     add ? add->stride : 0, add ? add->offset : 0);
  return hipGetLastError();
}

hipError_t nn_upsample2(const gs_act* x, gs_act* y, hipStream_t s) {
  const int64_t total = (int64_t)y->n * y->h * y->w * (x->c / 8);
  hipLaunchKernelGGL(upsample2_kernel, dim3(blocks(total)), dim3(256), 0, s, view(x), y->n, y->h,
                     y->w, static_cast<uint16_t*>(y->data), y->stride, y->offset);
  return hipGetLastError();
}

hipError_t nn_upsample2_bwd(const gs_act* dy, gs_act* dx, hipStream_t s) {
  const int64_t total = (int64_t)dx->n * dx->h * dx->w * (dy->c / 8);
  hipLaunchKernelGGL(upsample2_bwd_kernel, dim3(blocks(total)), dim3(256), 0, s, view(dy), dy->n,
                     dy->h, dy->w, static_cast<uint16_t*>(dx->data) + dx->offset, dx->stride);
  return hipGetLastError();
}

hipError_t nn_rgb_to_nhwc(const float* rgb, gs_act* x, hipStream_t s) {
  const int64_t npix = (int64_t)x->n * x->h * x->w;
  hipLaunchKernelGGL(rgb_to_nhwc_kernel, dim3(blocks(npix)), dim3(256), 0, s, rgb, x->n, x->h,
                     x->w, static_cast<uint16_t*>(x->data), x->stride);
  return hipGetLastError();
}

hipError_t nn_f32_to_bf16(const float* src, void* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks(n)), dim3(256), 0, s, src,
                     static_cast<uint16_t*>(dst), n);
  return hipGetLastError();
}

hipError_t nn_head(const gs_act* f, const float* w, const float* b, float* out, hipStream_t s) {
  const int64_t npix = (int64_t)f->n * f->h * f->w;
  if (f->c % 8 == 0 && f->stride % 8 == 0 && f->offset % 8 == 0)
    hipLaunchKernelGGL(head_fwd8_kernel, dim3(blocks(npix)), dim3(256), 0, s, view(f), f->n, f->h,
                       f->w, w, b, out);
  else
    hipLaunchKernelGGL(head_fwd_kernel, dim3(blocks(npix)), dim3(256), 0, s, view(f), f->n, f->h,
                       f->w, w, b, out);
  return hipGetLastError();
}

hipError_t nn_head_bwd(const gs_act* f, const float* w, const float* dout, gs_act* df, float* dw,
                       float* db, hipStream_t s) {
  const int64_t npix = (int64_t)f->n * f->h * f->w;
  if (f->c > 32 * kHeadMaxSlots) return hipErrorInvalidValue;
  if (f->c % 8 == 0 && f->c <= 8 * kHead8Groups && f->stride % 8 == 0 && f->offset % 8 == 0 &&
      df->stride % 8 == 0 && df->offset % 8 == 0) {
    const int per = 256 / (f->c / 8);
    const unsigned nb = (unsigned)std::min<int64_t>((npix + per - 1) / per, 2048);
    hipLaunchKernelGGL(head_bwd8_kernel, dim3(nb), dim3(256), 0, s, view(f), f->n, f->h, f->w, w,
                       dout, static_cast<uint16_t*>(df->data) + df->offset, df->stride, dw, db);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(head_bwd_kernel, dim3(std::min<unsigned>(blocks(npix), 1024u)), dim3(256), 0,
                     s, view(f), f->n, f->h,
                     f->w, w, dout, static_cast<uint16_t*>(df->data) + df->offset, df->stride, dw,
                     db);
  return hipGetLastError();
}

hipError_t nn_depth_loss(const float* pred, const float* depth, int N, int H, int W, float fx,
                         float* dpred, double* loss, int* count_ws, hipStream_t s) {
  const int64_t npix = (int64_t)N * H * W;
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(count_ws),
                     (int64_t)1);
  if (loss) hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s,
                               reinterpret_cast<uint32_t*>(loss), (int64_t)2);
  hipLaunchKernelGGL(count_valid_kernel, dim3(blocks(npix)), dim3(256), 0, s, depth, npix, count_ws);
  hipLaunchKernelGGL(depth_loss_kernel, dim3(blocks(npix)), dim3(256), 0, s, pred, depth, N, H, W,
                     fx, count_ws, dpred, loss);
  return hipGetLastError();
}

}  // namespace gsmi
