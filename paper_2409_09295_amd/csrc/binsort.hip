// gs_bin_sort: tile binning and (tile, depth) ordering of the splats.
//
//   count     one lane per (view, splat): tile rectangle (float64 from the
//             float32 centre) -> number of tiles, and whether it has any
//             (skipped when the projection stored the counts)
//   depth     the splats with tiles are compacted in entry order (by the
//             down-sweep of a scan of the flags) and sorted by their float32
//             depth bits with a
//             stable LSD radix sort, so equal depths keep entry order; this
//             sorts one item per visible splat instead of one per key
//   scan      device-wide exclusive scan of the tile counts in that order,
//             total in 64 bits (the key count)
//   emit      wave-cooperative emission in depth order: the 64 splats of a
//             wave own a contiguous key range; the wave walks that range 64
//             keys at a time and each lane finds its owner with a prefix
//             maximum over the splats' start marks, so stores are contiguous
//             and big rectangles do not serialise one lane
//   tile sort stable LSD radix sort of the keys on their tile bits only
//             (ceil(log2 tiles) bits): keys of a tile keep the depth order of
//             their emission, giving the (tile, depth, entry) order.  Per
//             pass: block histograms, a row scan of the digit-major
//             histogram, then a down-sweep that ranks keys within the block
//             with wave ballots (stable), stages them in LDS in digit order
//             and writes each digit run contiguously.  Without output keys
//             the passes carry 32-bit tile ids instead of 64-bit keys
//   ranges    [start, end) per global tile from tile boundaries in the
//             sorted keys
//   order     optional: the tiles stably sorted by list length group,
//             longest first (the launch order of the compositing grids)
#include "gs_internal.h"

namespace gsmi {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;   // 2048 (measured against 4096)
constexpr int kSortItems = 8;
constexpr int kSortChunk = 256 * kSortItems;            // 2048 keys per workgroup (tile passes)
// The depth passes sort only the binned splats (about a ninth of the
// entries): chunks of 1,024 keys put more workgroups in flight (measured
// against 2,048 and 512).
constexpr int kDepthItems = 4;

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

// Inclusive scan over the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over a 256-thread block; returns the
// exclusive prefix and writes the block total to *total (all threads).
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* s_wave, T& total) {
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const T inc = wave_inclusive_scan(x);
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  T pre = 0, tot = 0;
  for (uint32_t k = 0; k < 4; ++k) {
    const T s = s_wave[k];
    pre += (k < w) ? s : (T)0;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return pre + inc - x;
}

// ---------------------------------------------------------------------------
// generic exclusive scan of uint32 values (out may alias in)
// ---------------------------------------------------------------------------

// PRED: the scanned value is (in[i] != 0) instead of in[i].
template <bool PRED>
__device__ __forceinline__ uint32_t scan_in(const uint32_t* in, int64_t idx, int64_t n) {
  if (idx >= n) return 0u;
  const uint32_t x = in[idx];
  return PRED ? (x != 0u ? 1u : 0u) : x;
}

// n_dev (optional): a device-side count that bounds n further; blocks past it
// write a zero partial (reduce) or nothing (down-sweep).
__device__ __forceinline__ int64_t scan_bound(int64_t n, const uint32_t* n_dev) {
  return n_dev ? min(n, (int64_t)*n_dev) : n;
}

// Optional work folded into a scan's reduce kernel (saves a launch): clear
// ranges[n_tiles][2] and write the identity order (when order != nullptr).
struct ClearBins {
  uint32_t* ranges = nullptr;
  int n_tiles = 0;
  uint32_t* order = nullptr;
};

template <bool PRED>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                                   int64_t n,
                                                                   const uint32_t* __restrict__ n_dev,
                                                                   uint64_t* __restrict__ partial,
                                                                   ClearBins clr) {
  __shared__ uint64_t s_wave[4];
  for (int64_t t = (int64_t)blockIdx.x * kScanThreads + threadIdx.x; t < clr.n_tiles;
       t += (int64_t)gridDim.x * kScanThreads) {
    clr.ranges[2 * t] = 0u;
    clr.ranges[2 * t + 1] = 0u;
    if (clr.order) clr.order[t] = (uint32_t)t;
  }
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  n = scan_bound(n, n_dev);
  if (base >= n) {   // uniform over the block
    if (threadIdx.x == 0) partial[blockIdx.x] = 0;
    return;
  }
  uint64_t acc = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r)
    acc += scan_in<PRED>(in, base + r * kScanThreads + threadIdx.x, n);
  uint64_t tot;
  block_exclusive_scan<uint64_t>(acc, s_wave, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}


// Each wave scans kScanChunk / 4 consecutive values of the block's chunk as rows of
// 64 (coalesced), carrying the running total from row to row, so only the
// four wave totals need a block-level step.  out may alias in: every value is
// read before its position is written.
// Compacting form (Compact::on, with PRED): instead of the positions, the
// entries with in[i] != 0 are written in entry order as dkey[pos] = depth
// bits of rd[i], dval[pos] = i.
struct Compact {
  const float4* rd = nullptr;
  uint32_t* dkey = nullptr;
  uint32_t* dval = nullptr;
};

// partial: the reduce kernel's block sums; each block adds up those of the
// blocks before it (a few loads per thread), and the block holding the last
// value writes the total to *total and min(total, 2^32 - 1) to *n_keys.
template <bool PRED, bool COMPACT = false>
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(const uint32_t* in, int64_t n,
                                                                 const uint32_t* __restrict__ n_dev,
                                                                 const uint64_t* __restrict__ partial,
                                                                 uint32_t* out, Compact cp,
                                                                 uint64_t* __restrict__ total,
                                                                 uint32_t* __restrict__ n_keys) {
  static_assert(!COMPACT || PRED, "compaction scans the binned flags");
  __shared__ uint32_t s_wave[4];
  __shared__ uint64_t s_pre[4];
  constexpr int kRows = kScanChunk / kScanThreads;   // rows of 64 per wave
  n = scan_bound(n, n_dev);
  const int64_t bbase = (int64_t)blockIdx.x * kScanChunk;
  if (bbase >= n) {   // uniform over the block
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
      *total = 0;
      if (n_keys) *n_keys = 0;
    }
    return;
  }
  uint64_t pre = 0;
  for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanThreads) pre += partial[i];
  uint64_t block_pre;
  block_exclusive_scan<uint64_t>(pre, s_pre, block_pre);   // block_pre = sum over all threads
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)w * (64 * kRows) + lane;
  uint32_t x[kRows];
  uint32_t flags = 0;   // COMPACT: bit r set when row r's value is 1
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    x[r] = scan_in<PRED>(in, base + 64 * r, n);
    if (COMPACT) flags |= x[r] << r;
  }
  uint32_t run = 0;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const uint32_t inc = wave_inclusive_scan(x[r]);
    const uint32_t row_tot = __builtin_amdgcn_readlane(inc, 63);
    x[r] = run + inc - x[r];   // exclusive prefix within the wave's 1024 values
    run += row_tot;
  }
  if (lane == 0) s_wave[w] = run;
  __syncthreads();
  uint32_t carry = (uint32_t)block_pre;
  for (uint32_t k = 0; k < w; ++k) carry += s_wave[k];
  if (threadIdx.x == 0 && bbase + kScanChunk >= n) {   // the last block with values
    const uint64_t tot =
        block_pre + (uint64_t)s_wave[0] + s_wave[1] + (uint64_t)s_wave[2] + s_wave[3];
    *total = tot;
    if (n_keys) *n_keys = tot > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)tot;
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int64_t idx = base + 64 * r;
    if (COMPACT) {
      if ((flags >> r) & 1u) {
        const uint32_t j = carry + x[r];
        cp.dkey[j] = __float_as_uint(cp.rd[idx].w);
        cp.dval[j] = (uint32_t)idx;
      }
    } else if (idx < n) {
      out[idx] = carry + x[r];
    }
  }
}

// Exclusive scan of in[0, m) (of in[i] != 0 with PRED) into out, where
// m = min(n, *n_dev) when n_dev is given (out[m, n) is left untouched), else n;
// with COMPACT the scan compacts instead (see scan_down_kernel) and out is unused.
// The total goes to *total and, clamped to 32 bits, to *n_keys.  n > 0.
template <bool PRED = false, bool COMPACT = false>
void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* n_dev,
              uint64_t* partial, uint64_t* total, uint32_t* n_keys, hipStream_t s,
              Compact cp = Compact{}, ClearBins clr = ClearBins{}) {
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  if (nb > 0)
    hipLaunchKernelGGL(scan_reduce_kernel<PRED>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in,
                       n, n_dev, partial, clr);
  if (nb > 0)
    hipLaunchKernelGGL((scan_down_kernel<PRED, COMPACT>), dim3((unsigned)nb), dim3(kScanThreads), 0,
                       s, in, n, n_dev, partial, out, cp, total, n_keys);
}

// ---------------------------------------------------------------------------
// count / emit
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t value,
                                                       int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

__global__ __launch_bounds__(256) void count_kernel(const float2* __restrict__ xy,
                                                    const int32_t* __restrict__ radius,
                                                    int64_t n_entries, int64_t n, ViewTable vt,
                                                    uint32_t* __restrict__ counts) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_entries) return;
  const int v = (int)(e / n);
  const ViewInfo& vi = vt.v[v];
  Rect rc;
  const float2 c = xy[e];
  const bool ok = tile_rect(c.x, c.y, radius[e], vi.width, vi.height, rc);
  const uint32_t cnt = ok ? (uint32_t)((rc.x1 - rc.x0) * (rc.y1 - rc.y0)) : 0u;
  counts[e] = cnt;
}


// Inclusive prefix maximum over the 64 lanes of a wavefront (DPP row shifts,
// then the row broadcasts; lanes without a source see 0, the identity here).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, true);
}

__device__ __forceinline__ uint32_t wave_prefix_max(uint32_t x) {
  x = max(x, dpp_u32<0x111, 0xf>(x));   // row_shr:1
  x = max(x, dpp_u32<0x112, 0xf>(x));   // row_shr:2
  x = max(x, dpp_u32<0x114, 0xf>(x));   // row_shr:4
  x = max(x, dpp_u32<0x118, 0xf>(x));   // row_shr:8
  x = max(x, dpp_u32<0x142, 0xa>(x));   // row_bcast:15 into rows 1 and 3
  x = max(x, dpp_u32<0x143, 0xc>(x));   // row_bcast:31 into rows 2 and 3
  return x;
}

// Items j < *n_items are splats order[j] (depth order); item j's keys start at
// offsets[j].  A wavefront owns the contiguous key range of its 64 items and
// writes it 64 keys at a time: in each window of 64 positions, every item
// with keys marks where it starts, and a prefix maximum over the lanes gives
// each position its item (the item marked last at or before it).
// K = uint64_t: keys (tile << 32) | depth bits; K = uint32_t: the tile id
// alone (the keys are emitted in depth order, and the tile passes are
// stable, so the tile id is all the sort needs).
template <typename K>
__global__ __launch_bounds__(256) void emit_kernel(const float2* __restrict__ xy,
                                                   const int32_t* __restrict__ radius,
                                                   const float4* __restrict__ rd,
                                                   const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ n_items,
                                                   const uint32_t* __restrict__ offsets,
                                                   int64_t n, ViewTable vt,
                                                   const uint64_t* __restrict__ total,
                                                   int64_t capacity, K* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
  if (*total > (uint64_t)capacity) return;  // overflow: nothing is emitted
  __shared__ uint4 s_rect[4][64];    // start, first tile, rectangle width, tiles per row
  __shared__ uint2 s_val[4][64];     // depth bits, entry
  __shared__ uint32_t s_mark[4][64];
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = j < (int64_t)*n_items;
  uint32_t start = 0, cnt = 0, t0 = 0, rw = 1, tx = 1, db = 0, ent = 0;
  if (valid) {
    ent = order[j];
    const int v = (int)(ent / n);
    const ViewInfo& vi = vt.v[v];
    Rect rc;
    const float2 c = xy[ent];
    const bool ok = tile_rect(c.x, c.y, radius[ent], vi.width, vi.height, rc);
    start = offsets[j];
    if (ok) {
      cnt = (uint32_t)((rc.x1 - rc.x0) * (rc.y1 - rc.y0));
      t0 = (uint32_t)(vi.tile_base + rc.y0 * vi.tiles_x + rc.x0);
      rw = (uint32_t)(rc.x1 - rc.x0);
      tx = (uint32_t)vi.tiles_x;
      db = __float_as_uint(rd[ent].w);
    }
  }
  s_rect[w][lane] = make_uint4(start, t0, rw, tx);
  s_val[w][lane] = make_uint2(db, ent);
  // wave range [first start, last end); the items are contiguous from lane 0
  const uint64_t vmask = __ballot(valid);
  if (vmask == 0) return;
  const uint32_t wbase = __shfl(start, 0, 64);
  const uint32_t last = 63 - __clzll(vmask);
  const uint32_t wend = __shfl(start + cnt, last, 64);
  uint32_t carry = 0;   // 1 + item of the position before the window
  for (uint32_t w0 = wbase; w0 < wend; w0 += 64) {
    s_mark[w][lane] = 0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (cnt > 0 && start >= w0 && start - w0 < 64) s_mark[w][start - w0] = lane + 1;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t m = wave_prefix_max(max(s_mark[w][lane], carry));
    carry = (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
    const uint32_t pos = w0 + lane;
    if (pos < wend) {
      const uint4 r = s_rect[w][m - 1];
      const uint2 d = s_val[w][m - 1];
      const uint32_t jj = pos - r.x;
      const uint32_t row = jj / r.z;
      const uint32_t tile = r.y + row * r.w + (jj - row * r.z);
      if constexpr (sizeof(K) == 8)
        keys[pos] = ((uint64_t)tile << 32) | (uint64_t)d.x;
      else
        keys[pos] = tile;
      vals[pos] = d.y;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t valid_keys(const uint32_t* n_keys, int64_t capacity) {
  const uint32_t n = *n_keys;
  return ((int64_t)n <= capacity) ? n : 0u;
}

// ITEMS keys per thread: a workgroup sorts a chunk of 256 * ITEMS keys.
template <typename K, int ITEMS>
__global__ __launch_bounds__(256) void radix_upsweep_kernel(const K* __restrict__ keys,
                                                            const uint32_t* __restrict__ n_keys,
                                                            int64_t capacity, int shift,
                                                            uint32_t* __restrict__ hist,
                                                            uint32_t nblocks) {
  constexpr int kChunk = 256 * ITEMS;
  __shared__ uint32_t h[4][256];
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const uint32_t n = valid_keys(n_keys, capacity);
  if ((int64_t)blockIdx.x * kChunk >= (int64_t)n) return;   // past the keys: column unused
  for (int k = threadIdx.x; k < 4 * 256; k += 256) (&h[0][0])[k] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk + w * (kChunk / 4);
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    if (idx < n) atomicAdd(&h[w][(uint32_t)(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t t = threadIdx.x;
  hist[(int64_t)t * nblocks + blockIdx.x] = h[0][t] + h[1][t] + h[2][t] + h[3][t];
}

// Exclusive scan of each digit's row of per-block counts in the digit-major
// histogram [256][nblocks] (one workgroup per digit); row totals to tot[256].
// The down-sweep adds the exclusive prefix of the totals.
__global__ __launch_bounds__(256) void hist_row_scan_kernel(uint32_t* __restrict__ hist,
                                                            uint32_t nblocks, uint32_t chunk,
                                                            const uint32_t* __restrict__ n_keys,
                                                            int64_t capacity,
                                                            uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_wave[4];
  uint32_t* row = hist + (int64_t)blockIdx.x * nblocks;
  // columns of blocks past the keys are neither written nor read
  const uint32_t used = min(nblocks, (valid_keys(n_keys, capacity) + chunk - 1) / chunk);
  const uint32_t per = (used + 255) / 256;
  const uint32_t lo = min(used, threadIdx.x * per), hi = min(lo + per, used);
  uint32_t sum = 0;
  for (uint32_t k = lo; k < hi; ++k) sum += row[k];
  uint32_t total;
  uint32_t run = block_exclusive_scan<uint32_t>(sum, s_wave, total);
  for (uint32_t k = lo; k < hi; ++k) {
    const uint32_t x = row[k];
    row[k] = run;
    run += x;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// gather_in (optional): also writes gather_out[o] = gather_in[value] for the
// value placed at o (the tile counts of the splats, in the sorted order).
template <typename K, int ITEMS>
__global__ __launch_bounds__(256) void radix_downsweep_kernel(
    const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    K* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ n_keys, int64_t capacity, int shift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ digit_tot, uint32_t nblocks,
    const uint32_t* __restrict__ gather_in, uint32_t* __restrict__ gather_out) {
  constexpr int kChunk = 256 * ITEMS;
  __shared__ uint32_t s_wcnt[4][256];
  __shared__ uint32_t s_wpre[4][256];
  __shared__ uint32_t s_dstart[256];
  __shared__ uint32_t s_gbase[256];
  __shared__ uint32_t s_wave[4];
  __shared__ K s_keys[kChunk];
  __shared__ uint32_t s_vals[kChunk];
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const uint32_t n = valid_keys(n_keys, capacity);
  const int64_t bstart = (int64_t)blockIdx.x * kChunk;
  if (bstart >= (int64_t)n) return;   // no keys in this block
  for (int k = threadIdx.x; k < 4 * 256; k += 256) (&s_wcnt[0][0])[k] = 0;
  __syncthreads();
  const int64_t base = bstart + w * (kChunk / 4);
  K key[ITEMS];
  uint32_t val[ITEMS], rank[ITEMS], dig[ITEMS];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    const bool valid = idx < n;
    key[j] = valid ? keys_in[idx] : (K)0;
    val[j] = valid ? vals_in[idx] : 0u;
    const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
    dig[j] = d;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t r_in = (uint32_t)__popcll(peers & lt);
    uint32_t before = 0;
    if (valid) before = s_wcnt[w][d];
    __builtin_amdgcn_wave_barrier();
    if (valid && r_in == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    rank[j] = before + r_in;
  }
  __syncthreads();
  {
    const uint32_t t = threadIdx.x;
    const uint32_t c0 = s_wcnt[0][t], c1 = s_wcnt[1][t], c2 = s_wcnt[2][t], c3 = s_wcnt[3][t];
    s_wpre[0][t] = 0;
    s_wpre[1][t] = c0;
    s_wpre[2][t] = c0 + c1;
    s_wpre[3][t] = c0 + c1 + c2;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<uint32_t>(c0 + c1 + c2 + c3, s_wave, tot);
    s_dstart[t] = ex;
    const uint32_t dbase = block_exclusive_scan<uint32_t>(digit_tot[t], s_wave, tot);
    s_gbase[t] = hist[(int64_t)t * nblocks + blockIdx.x] + dbase;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t idx = base + j * 64 + lane;
    if (idx < n) {
      const uint32_t lp = s_dstart[dig[j]] + s_wpre[w][dig[j]] + rank[j];
      s_keys[lp] = key[j];
      s_vals[lp] = val[j];
    }
  }
  __syncthreads();
  const int64_t nb_valid = min((int64_t)kChunk, (int64_t)n - bstart);
#pragma unroll
  for (int q = 0; q < ITEMS; ++q) {
    const int pos = q * 256 + threadIdx.x;
    if (pos < nb_valid) {
      const K k = s_keys[pos];
      const uint32_t d = (uint32_t)(k >> shift) & 255u;
      const uint32_t o = s_gbase[d] + (uint32_t)pos - s_dstart[d];
      const uint32_t v = s_vals[pos];
      keys_out[o] = k;
      vals_out[o] = v;
      if (gather_in) gather_out[o] = gather_in[v];
    }
  }
}

__device__ __forceinline__ uint32_t key_tile(uint64_t k) { return (uint32_t)(k >> 32); }
__device__ __forceinline__ uint32_t key_tile(uint32_t k) { return k; }

template <typename K>
__global__ __launch_bounds__(256) void ranges_kernel(const K* __restrict__ keys,
                                                     const uint32_t* __restrict__ n_keys,
                                                     int64_t capacity, uint32_t* __restrict__ ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = valid_keys(n_keys, capacity);
  if (i >= n) return;
  const uint32_t tile = key_tile(keys[i]);
  if (i == 0 || key_tile(keys[i - 1]) != tile) ranges[2 * (int64_t)tile] = (uint32_t)i;
  if (i == (int64_t)n - 1 || key_tile(keys[i + 1]) != tile)
    ranges[2 * (int64_t)tile + 1] = (uint32_t)(i + 1);
}

// Tile order, longest lists first: a stable sort of the tiles by 32 list
// length groups (0, then half octaves), longest group first and ascending
// tile index within a group, so that tiles running side by side stay close
// in the image.  Three passes over blocks of kOrderBlock tiles: group counts
// per block, per-(block, group) output offsets, stable scatter.
constexpr int kOrderGroups = 32;
constexpr int kOrderBlock = 256;

__device__ __forceinline__ int length_group(uint32_t len) {   // ascending in len
  if (len == 0) return 0;
  const int lg = 31 - __clz(len);
  const int half = lg > 0 ? (int)((len >> (lg - 1)) & 1u) : 0;
  return min(kOrderGroups - 1, 1 + 2 * lg + half);
}

__device__ __forceinline__ int tile_group(const uint32_t* ranges, int t) {
  return length_group(ranges[2 * (int64_t)t + 1] - ranges[2 * (int64_t)t]);
}

// Group of this thread's tile (-1 past the end), its rank among the block's
// earlier tiles of the same group, and the block's count of every group.
__device__ __forceinline__ int block_group_ranks(const uint32_t* ranges, int n_tiles,
                                                 uint32_t* s_wcnt /* [4][32] */,
                                                 uint32_t* s_cnt /* [32] */, uint32_t& rank) {
  const int t = blockIdx.x * kOrderBlock + (int)threadIdx.x;
  const int g = t < n_tiles ? tile_group(ranges, t) : -1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint64_t peers = 0;
  for (int h = 0; h < kOrderGroups; ++h) {
    const uint64_t m = __ballot(g == h);
    if (g == h) peers = m;
    if (lane == 0) s_wcnt[wave * kOrderGroups + h] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < kOrderGroups) {
    uint32_t c = 0;
    for (int w = 0; w < kOrderBlock / 64; ++w) c += s_wcnt[w * kOrderGroups + threadIdx.x];
    s_cnt[threadIdx.x] = c;
  }
  rank = 0;
  if (g >= 0) {
    for (int w = 0; w < wave; ++w) rank += s_wcnt[w * kOrderGroups + g];
    rank += (uint32_t)__popcll(peers & ((uint64_t(1) << lane) - 1));
  }
  __syncthreads();
  return g;
}

__global__ __launch_bounds__(kOrderBlock) void order_count_kernel(
    const uint32_t* __restrict__ ranges, int n_tiles, uint32_t* __restrict__ blk) {
  __shared__ uint32_t s_wcnt[4 * kOrderGroups];
  __shared__ uint32_t s_cnt[kOrderGroups];
  uint32_t rank;
  block_group_ranks(ranges, n_tiles, s_wcnt, s_cnt, rank);
  if (threadIdx.x < kOrderGroups) blk[blockIdx.x * kOrderGroups + threadIdx.x] = s_cnt[threadIdx.x];
}

// One workgroup: blk[b][g] (counts) -> output offset of block b's group-g
// tiles.  Thread (g, j) owns the blocks of chunk j for group g.
__global__ __launch_bounds__(1024) void order_offsets_kernel(uint32_t* __restrict__ blk, int nblk) {
  __shared__ uint32_t s_part[kOrderGroups][33];
  __shared__ uint32_t s_start[kOrderGroups];
  const int g = threadIdx.x & 31, j = threadIdx.x >> 5;
  const int chunk = (nblk + 31) / 32;
  const int b0 = min(nblk, j * chunk), b1 = min(nblk, b0 + chunk);
  uint32_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += blk[b * kOrderGroups + g];
  s_part[g][j] = sum;
  __syncthreads();
  if (threadIdx.x < kOrderGroups) {   // chunk prefix per group, then group totals
    uint32_t run = 0;
    for (int k = 0; k < 32; ++k) {
      const uint32_t v = s_part[threadIdx.x][k];
      s_part[threadIdx.x][k] = run;
      run += v;
    }
    s_part[threadIdx.x][32] = run;
  }
  __syncthreads();
  if (threadIdx.x == 0) {   // longest group first
    uint32_t run = 0;
    for (int h = kOrderGroups - 1; h >= 0; --h) {
      s_start[h] = run;
      run += s_part[h][32];
    }
  }
  __syncthreads();
  uint32_t off = s_start[g] + s_part[g][j];
  for (int b = b0; b < b1; ++b) {
    const uint32_t c = blk[b * kOrderGroups + g];
    blk[b * kOrderGroups + g] = off;
    off += c;
  }
}

__global__ __launch_bounds__(kOrderBlock) void order_scatter_kernel(
    const uint32_t* __restrict__ ranges, int n_tiles, const uint32_t* __restrict__ blk,
    uint32_t* __restrict__ order) {
  __shared__ uint32_t s_wcnt[4 * kOrderGroups];
  __shared__ uint32_t s_cnt[kOrderGroups];
  uint32_t rank;
  const int g = block_group_ranks(ranges, n_tiles, s_wcnt, s_cnt, rank);
  if (g >= 0)
    order[blk[blockIdx.x * kOrderGroups + g] + rank] = (uint32_t)(blockIdx.x * kOrderBlock + threadIdx.x);
}

// Start of every call: all ranges empty and, when an order is requested, the
// identity order (so that bins.order is a permutation on every return path).
__global__ __launch_bounds__(256) void clear_bins_kernel(uint32_t* __restrict__ ranges, int n_tiles,
                                                         uint32_t* __restrict__ order) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  ranges[2 * (int64_t)t] = 0u;
  ranges[2 * (int64_t)t + 1] = 0u;
  if (order) order[t] = (uint32_t)t;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, value,
                     n);
  return hipGetLastError();
}

BinSortPlan make_bin_sort_plan(int64_t n, const ViewTable& vt, int64_t capacity) {
  BinSortPlan P{};
  P.n_entries = n * vt.n_views;
  P.capacity = capacity;
  P.n_tiles = vt.n_tiles;
  int tile_bits = 0;
  while ((int64_t(1) << tile_bits) < (int64_t)vt.n_tiles) ++tile_bits;
  P.passes = (tile_bits + 7) / 8;   // tile digits of the keys (depth is ordered beforehand)
  P.scan_blocks = (P.n_entries + kScanChunk - 1) / kScanChunk;
  P.sort_blocks = (capacity + kSortChunk - 1) / kSortChunk;
  const int64_t depth_chunk = 256 * kDepthItems;
  const int64_t depth_blocks = (P.n_entries + depth_chunk - 1) / depth_chunk;
  const int64_t hist_n = 256 * std::max<int64_t>(std::max(P.sort_blocks, depth_blocks), 1);
  const size_t ne = sizeof(uint32_t) * (size_t)P.n_entries;
  size_t off = 0;
  P.off_counts = off;    off += align_up(ne);
  P.off_offsets = off;   off += align_up(ne);   // key offsets in depth order
  P.off_dkey = off;      off += align_up(2 * ne);
  P.off_dval = off;      off += align_up(2 * ne);
  P.off_scan_part = off; off += align_up(sizeof(uint64_t) * (P.scan_blocks + 1));
  P.off_keys_alt = off;  off += align_up(sizeof(uint64_t) * capacity);
  P.off_vals_alt = off;  off += align_up(sizeof(uint32_t) * capacity);
  P.off_hist = off;      off += align_up(sizeof(uint32_t) * hist_n);
  P.off_hist_part = off; off += align_up(sizeof(uint32_t) * 256);   // digit totals
  P.off_flag = off;      off += align_up(sizeof(uint64_t) * 8);
  P.off_order = off;     // tile order: per-(block, group) counts, then offsets
  off += align_up(sizeof(uint32_t) * kOrderGroups * ((vt.n_tiles + kOrderBlock - 1) / kOrderBlock));
  P.total = off;
  return P;
}

// One LSD radix pass over n (device count, at most cap) keys of type K, in
// chunks of 256 * ITEMS keys.
template <typename K, int ITEMS>
void radix_pass(const K* kin, const uint32_t* vin, K* kout, uint32_t* vout, const uint32_t* n,
                int64_t cap, int shift, uint32_t* hist, uint32_t* digit_tot, hipStream_t s,
                const uint32_t* gather_in = nullptr, uint32_t* gather_out = nullptr) {
  constexpr int64_t chunk = 256 * ITEMS;
  const uint32_t nblocks = (uint32_t)((cap + chunk - 1) / chunk);
  hipLaunchKernelGGL((radix_upsweep_kernel<K, ITEMS>), dim3(nblocks), dim3(256), 0, s, kin, n, cap,
                     shift, hist, nblocks);
  hipLaunchKernelGGL(hist_row_scan_kernel, dim3(256), dim3(256), 0, s, hist, nblocks,
                     (uint32_t)chunk, n, cap, digit_tot);
  hipLaunchKernelGGL((radix_downsweep_kernel<K, ITEMS>), dim3(nblocks), dim3(256), 0, s, kin, vin,
                     kout, vout, n, cap, shift, hist, digit_tot, nblocks, gather_in, gather_out);
}

// Key emission in depth order, the stable passes over the tile bits (the
// first at bit tile_shift of K) and the ranges.  out/alt: the key buffers;
// after an even number of passes the sorted keys and values are in out and
// bins.values.
template <typename K>
void tile_sort(const gs_projected& p, int64_t n, const ViewTable& vt, const gs_bins& bins, K* out,
               K* alt, uint32_t* vals_alt, int tile_shift, const uint32_t* dval,
               const uint32_t* n_binned, const uint32_t* offsets, const uint64_t* flag,
               int64_t n_sort, uint32_t* hist, uint32_t* digit_tot, const BinSortPlan& P,
               hipStream_t s) {
  const auto* xy = reinterpret_cast<const float2*>(p.xy);
  const auto* rd = reinterpret_cast<const float4*>(p.rgb_depth);
  const unsigned eblocks = (unsigned)((P.n_entries + 255) / 256);
  K* kA = (P.passes % 2 == 0) ? out : alt;
  uint32_t* vA = (P.passes % 2 == 0) ? bins.values : vals_alt;
  K* kB = (P.passes % 2 == 0) ? alt : out;
  uint32_t* vB = (P.passes % 2 == 0) ? vals_alt : bins.values;
  hipLaunchKernelGGL((emit_kernel<K>), dim3(eblocks), dim3(256), 0, s, xy, p.radius, rd, dval,
                     n_binned, offsets, n, vt, flag, P.capacity, kA, vA);
  for (int pass = 0; pass < P.passes; ++pass) {
    radix_pass<K, kSortItems>(kA, vA, kB, vB, bins.n_keys, std::min<int64_t>(n_sort, P.capacity),
                              tile_shift + 8 * pass, hist, digit_tot, s);
    std::swap(kA, kB);
    std::swap(vA, vB);
  }
  hipLaunchKernelGGL((ranges_kernel<K>), dim3((unsigned)((n_sort + 255) / 256)), dim3(256), 0, s,
                     kA, bins.n_keys, P.capacity, bins.ranges);
}

int run_bin_sort(const gs_projected& p, int64_t n, const ViewTable& vt, const gs_bins& bins,
                 uint32_t* n_keys_host, char* ws, const BinSortPlan& P, hipStream_t s) {
  auto* counts = reinterpret_cast<uint32_t*>(ws + P.off_counts);
  auto* offsets = reinterpret_cast<uint32_t*>(ws + P.off_offsets);
  auto* dkey = reinterpret_cast<uint32_t*>(ws + P.off_dkey);
  auto* dval = reinterpret_cast<uint32_t*>(ws + P.off_dval);
  auto* part = reinterpret_cast<uint64_t*>(ws + P.off_scan_part);
  auto* keys_alt = reinterpret_cast<uint64_t*>(ws + P.off_keys_alt);
  auto* vals_alt = reinterpret_cast<uint32_t*>(ws + P.off_vals_alt);
  auto* hist = reinterpret_cast<uint32_t*>(ws + P.off_hist);
  auto* digit_tot = reinterpret_cast<uint32_t*>(ws + P.off_hist_part);
  auto* flag = reinterpret_cast<uint64_t*>(ws + P.off_flag);   // [0] keys, [1] binned splats
  auto* n_binned = reinterpret_cast<uint32_t*>(flag + 2);
  auto* order_blk = reinterpret_cast<uint32_t*>(ws + P.off_order);
  const auto* xy = reinterpret_cast<const float2*>(p.xy);
  const auto* rd = reinterpret_cast<const float4*>(p.rgb_depth);
  const int64_t ne = P.n_entries;
  const unsigned eblocks = (unsigned)((ne + 255) / 256);
  hipError_t e;

  kernel_event_start(GS_KERNEL_BIN_SORT, s);
  // all ranges empty and the identity order first (so that both are valid on
  // every return path): folded into the first scan, or a kernel of its own
  ClearBins clr;
  clr.ranges = bins.ranges;
  clr.n_tiles = vt.n_tiles;
  clr.order = bins.order;
  if (ne == 0 && vt.n_tiles > 0)
    hipLaunchKernelGGL(clear_bins_kernel, dim3((unsigned)((vt.n_tiles + 255) / 256)), dim3(256), 0,
                       s, bins.ranges, vt.n_tiles, bins.order);
  // 1. tiles per splat (from the projection when it stored them); binned
  // splats compacted in entry order with their depth
  if (ne > 0) {
    // (the scan's down-sweep writes the compacted depth keys and entries)
    const uint32_t* tiles = p.tiles;
    if (!tiles) {
      hipLaunchKernelGGL(count_kernel, dim3(eblocks), dim3(256), 0, s, xy, p.radius, ne, n, vt,
                         counts);
      tiles = counts;
    }
    Compact cp;
    cp.rd = rd;
    cp.dkey = dkey;
    cp.dval = dval;
    scan_u32<true, true>(tiles, nullptr, ne, nullptr, part, flag + 1, n_binned, s, cp, clr);
    // 2. stable sort of the binned splats by depth (ties keep entry order)
    uint32_t *ka = dkey, *va = dval, *kb = dkey + ne, *vb = dval + ne;
    // (the last pass also writes each splat's tile count in the sorted order)
    for (int pass = 0; pass < 4; ++pass) {
      radix_pass<uint32_t, kDepthItems>(ka, va, kb, vb, n_binned, ne, 8 * pass, hist, digit_tot, s,
                                        pass == 3 ? tiles : nullptr,
                                        pass == 3 ? offsets : nullptr);
      std::swap(ka, kb);
      std::swap(va, vb);
    }
    // ka/va (= dkey/dval after an even number of passes) hold the depth order
    // 3. key offsets in depth order (an in-place scan of those counts); their
    // total is the key count.  Positions past the binned splats are neither
    // written nor read.
    scan_u32(offsets, offsets, ne, n_binned, part, flag, bins.n_keys, s);
  } else {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, s,
                       reinterpret_cast<uint32_t*>(flag), 0u, (int64_t)16);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, s, bins.n_keys, 0u, (int64_t)1);
  }
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "count/depth-order launch");

  int64_t n_sort = P.capacity;   // keys the sort grid covers
  if (n_keys_host) {
    uint64_t total = 0;
    if ((e = hipMemcpyAsync(&total, flag, sizeof(uint64_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(e, "read key count");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "synchronise key count");
    *n_keys_host = total > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)total;
    if (total > (uint64_t)P.capacity) {
      set_error("gs_bin_sort: %llu keys exceed capacity %lld", (unsigned long long)total,
                (long long)P.capacity);
      return GS_ERR_CAPACITY;
    }
    n_sort = (int64_t)total;
  }
  if (n_sort == 0 || ne == 0) {
    kernel_event_stop(GS_KERNEL_BIN_SORT, s);
    return GS_OK;
  }

  // 4. keys emitted in depth order, then a stable sort on the tile bits only
  // (with bins.keys == NULL on 32-bit tile ids held in the workspace)
  if (bins.keys)
    tile_sort<uint64_t>(p, n, vt, bins, bins.keys, reinterpret_cast<uint64_t*>(keys_alt), vals_alt,
                        32, dval, n_binned, offsets, flag, n_sort, hist, digit_tot, P, s);
  else
    tile_sort<uint32_t>(p, n, vt, bins, reinterpret_cast<uint32_t*>(keys_alt),
                        reinterpret_cast<uint32_t*>(keys_alt) + P.capacity, vals_alt, 0, dval,
                        n_binned, offsets, flag, n_sort, hist, digit_tot, P, s);
  if (bins.order && vt.n_tiles > 0) {
    const int nblk = (vt.n_tiles + kOrderBlock - 1) / kOrderBlock;
    hipLaunchKernelGGL(order_count_kernel, dim3((unsigned)nblk), dim3(kOrderBlock), 0, s,
                       bins.ranges, vt.n_tiles, order_blk);
    hipLaunchKernelGGL(order_offsets_kernel, dim3(1), dim3(1024), 0, s, order_blk, nblk);
    hipLaunchKernelGGL(order_scatter_kernel, dim3((unsigned)nblk), dim3(kOrderBlock), 0, s,
                       bins.ranges, vt.n_tiles, order_blk, bins.order);
  }
  kernel_event_stop(GS_KERNEL_BIN_SORT, s);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "bin sort launch");
  return GS_OK;
}

}  // namespace gsmi
