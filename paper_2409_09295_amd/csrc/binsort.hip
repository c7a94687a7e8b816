// gs_bin_sort: tile binning and (tile, depth) ordering of the splats.
//
// The order wanted is, per global tile, the splats whose rectangles cover it
// by ascending (float32 depth bits, entry).  It is built as a counting sort
// on the tile (the tiles are few: 38,400 for 32 views at 640x480) followed by
// a sort of each tile's own short list.  No step uses global atomics on the
// tile counters, which contend badly on tiles many splats cover:
//
//   compact   the splats of each view that touch a tile are appended to a
//             per-view list as {u, v, radius, depth} records (one global
//             atomic per workgroup of 1,024 entries); the walks below read
//             only these (a tenth of the entries in a mapping batch)
//   hist      each workgroup of 512 threads takes chunks of 1,024 listed
//             splats of one view and counts, in an LDS histogram over that
//             view's tiles, the keys they emit (each splat's tile rectangle
//             in float64 from its float32 centre), then stores the whole
//             histogram as row `chunk` of a dense chunk x tile matrix.
//             Splats with large rectangles do not serialise one lane: a
//             wavefront walks its 64 splats' keys 64 at a time, each lane
//             finding its splat by a prefix maximum over start marks.
//   column    per tile, an exclusive scan down its matrix column (each
//             chunk's first slot within the tile's segment) and the total
//   scan      exclusive scan of the per-tile totals: every tile's [start,
//             end) in the sorted keys, and the key count (in 64 bits)
//   emit      the same walk per chunk places each key's (depth bits,
//             entry) pair in its tile's segment, at the chunk's slots
//             (LDS atomics hand out the slots within a chunk)
//   segment   one wavefront per tile sorts its segment by (depth bits,
//             entry) with a bitonic network in registers (lists of up to
//             kSegShort pairs) and writes the entries (and keys); in the
//             same launch, the first workgroups sort the longer lists with
//             all their wavefronts (registers and LDS), or, beyond kSegLong
//             pairs, by a stable LSD radix sort over the 64-bit pair
//   order     optional: the tiles stably sorted by list length group,
//             longest first (the launch order of the compositing grids)
//
// Views with more tiles than the LDS histogram holds are processed in tile
// windows (one walk per window).  Nothing here needs a host synchronisation
// unless the caller asks for the key count.
#include "gs_internal.h"

namespace gsmi {

namespace {

constexpr int kBinThreads = 512;                         // threads of a binning workgroup
constexpr int kBinWaves = kBinThreads / 64;
constexpr int kWalkBatch = 2;                            // splats per binning thread
constexpr int kBinChunk = kBinThreads * kWalkBatch;      // splats per binning chunk
constexpr int kBinGrid = 32;                             // binning workgroups per view
constexpr int kLdsTiles = 8192;                          // largest LDS histogram (tiles)
constexpr int kSegShort = 1024;                          // longest list of the wavefront sort
constexpr int kSegLong = 4096;                           // longest list of the workgroup sort
constexpr int kSortThreads = 512;                        // threads of a sort workgroup
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kLongSlots = 256;                          // sort workgroups that take the long lists

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

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

// ---------------------------------------------------------------------------
// the key walk
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t value,
                                                       int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
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

// Inclusive prefix sum over the 64 lanes (the same DPP pattern).
__device__ __forceinline__ uint32_t wave_prefix_sum(uint32_t x) {
  x += dpp_u32<0x111, 0xf>(x);
  x += dpp_u32<0x112, 0xf>(x);
  x += dpp_u32<0x114, 0xf>(x);
  x += dpp_u32<0x118, 0xf>(x);
  x += dpp_u32<0x142, 0xa>(x);
  x += dpp_u32<0x143, 0xc>(x);
  return x;
}

// Per wavefront: its 64 entries' key ranges and rectangles while it walks them.
struct WalkLds {
  uint4 rect[kBinWaves][64];   // first key in the wave's run, first tile (view-local), width, tiles per row
  uint32_t ent[kBinWaves][64];
  uint32_t dep[kBinWaves][64];   // float32 depth bits (emission only)
  uint32_t mark[kBinWaves][64];
};

// q = jj / w for jj < 2^20 and 1 <= w < 2^11: a float reciprocal estimate
// corrected by one step either way (exact: the estimate is within one).
__device__ __forceinline__ uint32_t div_small(uint32_t jj, uint32_t w) {
  uint32_t q = (uint32_t)((float)jj * __builtin_amdgcn_rcpf((float)w));
  if (q * w > jj) --q;
  else if ((q + 1) * w <= jj) ++q;
  return q;
}

// Calls op(view-local tile, entry, depth bits) once for every key that the
// splats j0 .. j0 + kBinChunk of a view's compacted list (count splats in
// all) emit.  Each thread takes kWalkBatch splats (stride kBinThreads) and
// issues their loads together; then, per splat slot, each wavefront walks
// its 64 splats' keys 64 at a time, every lane taking the key at its
// position and finding the splat that owns it as the last splat whose first
// key is at or before it (a prefix maximum over start marks), so large
// rectangles spread over the lanes.
template <bool kDepth, typename Op>
__device__ __forceinline__ void walk_keys(const uint4* __restrict__ rec,
                                          const uint32_t* __restrict__ ids, uint32_t count,
                                          uint32_t j0, const ViewInfo& vi, WalkLds& L, Op op) {
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  // all loads of the batch first, from clamped indices (no branches between
  // them, so they are in flight together); slots past the list get radius 0
  uint4 c[kWalkBatch];
  uint32_t id[kWalkBatch];
#pragma unroll
  for (int q = 0; q < kWalkBatch; ++q) {
    const uint32_t j = j0 + q * kBinThreads + threadIdx.x;
    const uint32_t jc = j < count ? j : count - 1;
    c[q] = rec[jc];
    if constexpr (kDepth) id[q] = ids[jc];
    if (j >= count) c[q].z = 0u;
  }
  // per entry: key count, and first tile | rectangle width << 21 (a view
  // has at most 2^20 tiles, a rectangle at most 1,024 columns)
  uint32_t cnt[kWalkBatch], rect[kWalkBatch], dep[kWalkBatch];
#pragma unroll
  for (int q = 0; q < kWalkBatch; ++q) {
    Rect rc;
    cnt[q] = 0;
    rect[q] = 1u << 21;
    dep[q] = 0;
    if (tile_rect(__uint_as_float(c[q].x), __uint_as_float(c[q].y), (int32_t)c[q].z, vi.width,
                  vi.height, rc)) {
      cnt[q] = (uint32_t)((rc.x1 - rc.x0) * (rc.y1 - rc.y0));
      rect[q] = (uint32_t)(rc.y0 * vi.tiles_x + rc.x0) | ((uint32_t)(rc.x1 - rc.x0) << 21);
      if constexpr (kDepth) dep[q] = c[q].w;
    }
  }
#pragma unroll
  for (int q = 0; q < kWalkBatch; ++q) {
    const uint32_t inc = wave_prefix_sum(cnt[q]);
    const uint32_t start = inc - cnt[q];
    const uint32_t wend = __builtin_amdgcn_readlane(inc, 63);
    if (wend == 0) continue;   // uniform within the wavefront
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    L.rect[w][lane] = make_uint4(start, rect[q] & 0x1FFFFFu, rect[q] >> 21, (uint32_t)vi.tiles_x);
    if constexpr (kDepth) {
      L.ent[w][lane] = id[q];
      L.dep[w][lane] = dep[q];
    }
    uint32_t carry = 0;   // 1 + lane of the entry owning the position before the window
    for (uint32_t w0 = 0; w0 < wend; w0 += 64) {
      L.mark[w][lane] = 0;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      if (cnt[q] > 0 && start >= w0 && start - w0 < 64) L.mark[w][start - w0] = lane + 1;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
      const uint32_t m = wave_prefix_max(max(L.mark[w][lane], carry));
      carry = (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
      const uint32_t pos = w0 + lane;
      if (pos < wend) {   // then m >= 1: the owner's first key is at or before pos
        const uint4 rc = L.rect[w][m - 1];
        const uint32_t jj = pos - rc.x;
        const uint32_t row = div_small(jj, rc.z);
        if constexpr (kDepth)
          op(rc.y + row * rc.w + (jj - row * rc.z), L.ent[w][m - 1], L.dep[w][m - 1]);
        else
          op(rc.y + row * rc.w + (jj - row * rc.z), 0u, 0u);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
    }
  }
}

// ---------------------------------------------------------------------------
// compaction, counts: chunk x tile matrix, column scan
// ---------------------------------------------------------------------------

constexpr int kCompactItems = 4;                 // entries per thread (256 threads)
constexpr int kCompactChunk = 256 * kCompactItems;

// Grid (entries / kCompactChunk, views): the splats of view v that touch a
// tile (stored count > 0, or radius > 0 when counts are not stored) are
// appended to the view's list, [v n, v n + list_count[v]), as {u, v, radius,
// depth bits} records with their entries (v n + i) beside them.  One global
// atomic per workgroup reserves its run; the list order is the order of the
// reservations, which the per-tile sort makes irrelevant.
__global__ __launch_bounds__(256) void bin_compact_kernel(const float2* __restrict__ xy,
                                                          const int32_t* __restrict__ radius,
                                                          const float4* __restrict__ rd,
                                                          const uint32_t* __restrict__ stored,
                                                          int64_t n,
                                                          uint32_t* __restrict__ list_count,
                                                          uint4* __restrict__ rec,
                                                          uint32_t* __restrict__ ids) {
  __shared__ uint32_t s_wave[4];
  __shared__ uint32_t s_base;
  const int v = blockIdx.y;
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * kCompactChunk;
  bool keep[kCompactItems];
  uint32_t mine = 0;
#pragma unroll
  for (int q = 0; q < kCompactItems; ++q) {
    const int64_t i = i0 + q * 256 + threadIdx.x;
    const int64_t e = (int64_t)v * n + (i < n ? i : n - 1);
    const uint32_t x = stored ? stored[e] : (uint32_t)max(radius[e], 0);
    keep[q] = i < n && x > 0u;
    mine += keep[q] ? 1u : 0u;
  }
  // the kept splats' data, loaded while the run is reserved (entries not
  // kept read the view's first entry instead, one cached line)
  float2 c[kCompactItems];
  int32_t r[kCompactItems];
  float z[kCompactItems];
#pragma unroll
  for (int q = 0; q < kCompactItems; ++q) {
    const int64_t e = (int64_t)v * n + (keep[q] ? i0 + q * 256 + threadIdx.x : 0);
    c[q] = xy[e];
    r[q] = radius[e];
    z[q] = rd[e].w;
  }
  const uint32_t inc = wave_prefix_sum(mine);
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t tot = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    s_base = tot ? atomicAdd(&list_count[v], tot) : 0u;
  }
  __syncthreads();
  uint32_t pos = s_base + inc - mine;
  for (uint32_t k = 0; k < w; ++k) pos += s_wave[k];
  uint4* vrec = rec + (int64_t)v * n;
  uint32_t* vids = ids + (int64_t)v * n;
#pragma unroll
  for (int q = 0; q < kCompactItems; ++q) {
    if (keep[q]) {
      vrec[pos] = make_uint4(__float_as_uint(c[q].x), __float_as_uint(c[q].y), (uint32_t)r[q],
                             __float_as_uint(z[q]));
      vids[pos] = (uint32_t)((int64_t)v * n + i0 + q * 256 + threadIdx.x);
      ++pos;
    }
  }
}

__device__ __forceinline__ uint32_t list_chunks(uint32_t count) {
  return (count + kBinChunk - 1) / kBinChunk;
}

// Grid (kBinGrid, views): workgroup x takes chunks x, x + kBinGrid, ... of
// view y's list; row `chunk` of `matrix` ([chunks][n_tiles]), over the
// view's columns, receives the keys the chunk emits per tile.
__global__ __launch_bounds__(kBinThreads) void bin_hist_kernel(const uint4* __restrict__ rec,
                                                               const uint32_t* __restrict__ list_count,
                                                               int64_t n, ViewTable vt,
                                                               int lds_tiles,
                                                               uint32_t* __restrict__ matrix) {
  extern __shared__ uint32_t s_hist[];
  __shared__ WalkLds L;
  const int v = blockIdx.y;
  const ViewInfo& vi = vt.v[v];
  const uint32_t count = list_count[v];
  const int vtiles = vi.tiles_x * vi.tiles_y;
  const uint4* vrec = rec + (int64_t)v * n;
  for (uint32_t ch = blockIdx.x; ch < list_chunks(count); ch += gridDim.x) {
    uint32_t* row = matrix + (int64_t)ch * vt.n_tiles + vi.tile_base;
    for (int tw = 0; tw < vtiles; tw += lds_tiles) {   // tile windows (one unless the view is huge)
      const uint32_t span = (uint32_t)min(lds_tiles, vtiles - tw);
      for (uint32_t t = threadIdx.x; t < span; t += kBinThreads) s_hist[t] = 0u;
      __syncthreads();
      walk_keys<false>(vrec, nullptr, count, ch * kBinChunk, vi, L,
                       [&](uint32_t tile, uint32_t, uint32_t) {
                         const uint32_t k = tile - (uint32_t)tw;
                         if (k < span) atomicAdd(&s_hist[k], 1u);
                       });
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < span; t += kBinThreads) row[tw + t] = s_hist[t];
      __syncthreads();
    }
  }
}

// Grid (view tiles / 256, views), one thread per tile: exclusive scan down
// its column over the view's chunks (in place) and the column total.
__global__ __launch_bounds__(256) void bin_column_kernel(uint32_t* __restrict__ matrix,
                                                         const uint32_t* __restrict__ list_count,
                                                         ViewTable vt,
                                                         uint32_t* __restrict__ counts) {
  const int v = blockIdx.y;
  const ViewInfo& vi = vt.v[v];
  const int tl = blockIdx.x * 256 + threadIdx.x;
  if (tl >= vi.tiles_x * vi.tiles_y) return;
  const int64_t T = vt.n_tiles;
  const int t = vi.tile_base + tl;
  const int chunks = (int)list_chunks(list_count[v]);
  uint32_t run = 0;
  int c = 0;
  for (; c + 8 <= chunks; c += 8) {
    uint32_t x[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = matrix[(int64_t)(c + q) * T + t];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      matrix[(int64_t)(c + q) * T + t] = run;
      run += x[q];
    }
  }
  for (; c < chunks; ++c) {
    const uint32_t x = matrix[(int64_t)c * T + t];
    matrix[(int64_t)c * T + t] = run;
    run += x;
  }
  counts[t] = run;
}

// ---------------------------------------------------------------------------
// exclusive scan of the per-tile counts: segments, key count
// ---------------------------------------------------------------------------

constexpr int kScanBlock = 1024;   // tiles per scan workgroup (256 threads x 4)

__global__ __launch_bounds__(256) void bin_scan_reduce_kernel(const uint32_t* __restrict__ counts,
                                                              int n_tiles,
                                                              uint64_t* __restrict__ partial,
                                                              uint32_t* __restrict__ n_long,
                                                              uint32_t* __restrict__ queue) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_long = 0u;   // the down-sweep queues long lists
  // the compositing calls' tile counters start from zero
  if (queue && blockIdx.x == 0)
    for (int w = threadIdx.x; w < GS_QUEUE_WORDS; w += 256) queue[w] = 0u;
  __shared__ uint64_t s_wave[4];
  const int base = blockIdx.x * kScanBlock + threadIdx.x;
  uint64_t acc = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc += base + q * 256 < n_tiles ? counts[base + q * 256] : 0u;
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if (lane_id() == 0) s_wave[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
}

// Each workgroup adds the totals of the blocks before it and scans its own
// 1,024 tiles (4 consecutive per thread): ranges [start, end) ([0, 0) for an
// empty tile, and for all on overflow) and every tile's first slot, and
// queues the tiles with more than kSegShort keys; block 0 also writes the
// key count in 64 bits and its 32-bit clamp.
__global__ __launch_bounds__(256) void bin_scan_down_kernel(const uint32_t* __restrict__ counts,
                                                            int n_tiles,
                                                            const uint64_t* __restrict__ partial,
                                                            int n_blocks, int64_t capacity,
                                                            uint32_t* __restrict__ ranges,
                                                            uint32_t* __restrict__ starts,
                                                            uint64_t* __restrict__ total,
                                                            uint32_t* __restrict__ n_keys,
                                                            uint32_t* __restrict__ long_list,
                                                            uint32_t* __restrict__ n_long) {
  __shared__ uint64_t s_red[2][4];
  __shared__ uint32_t s_wave[4];
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  uint64_t pre = 0, tot = 0;
  for (int b = threadIdx.x; b < n_blocks; b += 256) {
    const uint64_t x = partial[b];
    tot += x;
    pre += b < (int)blockIdx.x ? x : 0u;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    pre += __shfl_xor(pre, d, 64);
    tot += __shfl_xor(tot, d, 64);
  }
  if (lane == 0) {
    s_red[0][w] = pre;
    s_red[1][w] = tot;
  }
  const int t0 = blockIdx.x * kScanBlock + 4 * threadIdx.x;
  uint32_t c[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) c[q] = t0 + q < n_tiles ? counts[t0 + q] : 0u;
  const uint32_t mine = c[0] + c[1] + c[2] + c[3];
  const uint32_t inc = wave_inclusive_scan(mine);
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  pre = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
  tot = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
  const bool ok = tot <= (uint64_t)capacity;
  uint32_t st = (uint32_t)pre + inc - mine;   // exact whenever ok
  for (uint32_t k = 0; k < w; ++k) st += s_wave[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *total = tot;
    *n_keys = tot > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)tot;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = t0 + q;
    if (t < n_tiles) {
      const bool used = ok && c[q] > 0;
      ranges[2 * (int64_t)t] = used ? st : 0u;
      ranges[2 * (int64_t)t + 1] = used ? st + c[q] : 0u;
      starts[t] = st;
    }
    st += c[q];
  }
  // queue the long lists: one atomic per wavefront and item; lane 0's
  // reservation reaches the other lanes through LDS (every lane reads what
  // lane 0 wrote, whatever the compiler does with the lanes' control flow)
  __shared__ uint32_t s_qbase[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = t0 + q;
    const bool lng = ok && t < n_tiles && c[q] > (uint32_t)kSegShort;
    const uint64_t m = __ballot(lng);
    if (m) {
      if (lane == 0) s_qbase[w] = atomicAdd(n_long, (uint32_t)__popcll(m));
      const uint32_t base = s_qbase[w];
      if (lng) long_list[base + (uint32_t)__popcll(m & ((uint64_t(1) << lane) - 1))] = (uint32_t)t;
    }
  }
}

// ---------------------------------------------------------------------------
// emission
// ---------------------------------------------------------------------------

// Grid (kBinGrid, views), chunks as in the histogram: every key's (depth
// bits, entry) pair goes to its tile's segment at slot start + (the chunk's
// offset in the column) + (its rank among the chunk's keys of that tile, in
// no particular order).  Nothing on overflow.
__global__ __launch_bounds__(kBinThreads) void bin_emit_kernel(
    const uint4* __restrict__ rec, const uint32_t* __restrict__ ids,
    const uint32_t* __restrict__ list_count, int64_t n, ViewTable vt, int lds_tiles,
    const uint32_t* __restrict__ matrix, const uint32_t* __restrict__ starts,
    const uint64_t* __restrict__ total, int64_t capacity, uint64_t* __restrict__ staged) {
  extern __shared__ uint32_t s_slot[];
  __shared__ WalkLds L;
  if (*total > (uint64_t)capacity) return;
  const int v = blockIdx.y;
  const ViewInfo& vi = vt.v[v];
  const uint32_t count = list_count[v];
  const int vtiles = vi.tiles_x * vi.tiles_y;
  const uint4* vrec = rec + (int64_t)v * n;
  const uint32_t* vids = ids + (int64_t)v * n;
  const uint32_t* st = starts + vi.tile_base;
  for (uint32_t ch = blockIdx.x; ch < list_chunks(count); ch += gridDim.x) {
    const uint32_t* row = matrix + (int64_t)ch * vt.n_tiles + vi.tile_base;
    for (int tw = 0; tw < vtiles; tw += lds_tiles) {
      const uint32_t span = (uint32_t)min(lds_tiles, vtiles - tw);
      for (uint32_t t = threadIdx.x; t < span; t += kBinThreads) s_slot[t] = st[tw + t] + row[tw + t];
      __syncthreads();
      walk_keys<true>(vrec, vids, count, ch * kBinChunk, vi, L,
                      [&](uint32_t tile, uint32_t ent, uint32_t dep) {
                        const uint32_t k = tile - (uint32_t)tw;
                        if (k < span) staged[atomicAdd(&s_slot[k], 1u)] = ((uint64_t)dep << 32) | ent;
                      });
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// per-tile sort by (depth bits, entry)
// ---------------------------------------------------------------------------

template <typename K>
__device__ __forceinline__ void seg_store(K* keys, uint32_t* vals, int64_t pos, uint32_t tile,
                                          uint64_t k) {
  vals[pos] = (uint32_t)k;
  if constexpr (sizeof(K) == 8) {
    if (keys) keys[pos] = ((uint64_t)tile << 32) | (k >> 32);
  }
}

// The value of lane (this lane ^ jl), 64 bits: DPP quad permutations for 1
// and 2, a row rotation by 8 for 8, a lane permute otherwise.
__device__ __forceinline__ uint64_t lane_xor(uint64_t x, int jl) {
  const int lo = (int)(uint32_t)x, hi = (int)(uint32_t)(x >> 32);
  int a, b;
  switch (jl) {
    case 1:   // quad_perm [1, 0, 3, 2]
      a = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xf, 0xf, true);
      b = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xf, 0xf, true);
      break;
    case 2:   // quad_perm [2, 3, 0, 1]
      a = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xf, 0xf, true);
      b = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xf, 0xf, true);
      break;
    case 8:   // row_ror:8
      a = __builtin_amdgcn_update_dpp(0, lo, 0x128, 0xf, 0xf, true);
      b = __builtin_amdgcn_update_dpp(0, hi, 0x128, 0xf, 0xf, true);
      break;
    default:
      a = __shfl_xor(lo, jl, 64);
      b = __shfl_xor(hi, jl, 64);
      break;
  }
  return ((uint64_t)(uint32_t)b << 32) | (uint32_t)a;
}

// One stage (block size kk, partner distance j) of an ascending bitonic sort
// of the pairs whose indices are gbase + lane R + k, held in x[k] (R
// consecutive pairs per lane).  Partners closer than R are in the same lane;
// partners up to 64 R apart are exchanged across lanes.
template <int R>
__device__ __forceinline__ void bitonic_stage_wave(uint64_t (&x)[R], uint32_t lane, uint32_t gbase,
                                                   int kk, int j) {
  if (j < R) {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if ((k & j) == 0) {
        const bool up = ((gbase + lane * R + k) & kk) == 0;
        const uint64_t a = x[k], b = x[k + j];
        const bool sw = (b < a) == up;
        x[k] = sw ? b : a;
        x[k + j] = sw ? a : b;
      }
    }
  } else {
    const int jl = j / R;
    const bool up = ((gbase + lane * R) & kk) == 0;
    const bool keep_min = up == ((lane & jl) == 0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint64_t y = lane_xor(x[k], jl);
      x[k] = ((y < x[k]) == keep_min) ? y : x[k];
    }
  }
}

// One wavefront sorts a list of at most 64 R pairs in registers.
template <int R, typename K>
__device__ __forceinline__ void wave_segment_sort(const uint64_t* __restrict__ staged, uint32_t s,
                                                  int len, uint32_t tile, K* keys, uint32_t* vals) {
  const uint32_t lane = lane_id();
  uint64_t x[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = (int)lane * R + k;
    x[k] = i < len ? staged[s + i] : ~0ull;
  }
#pragma unroll
  for (int kk = 2; kk <= 64 * R; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) bitonic_stage_wave<R>(x, lane, 0u, kk, j);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = (int)lane * R + k;
    if (i < len) seg_store(keys, vals, (int64_t)s + i, tile, x[k]);
  }
}

// The kSortWaves wavefronts of a workgroup sort a list of at most
// kSortWaves 64 R pairs: wavefront w holds indices w 64 R + lane R + k;
// partners 64 R or more apart are exchanged through LDS (s_x).
template <int R, typename K>
__device__ __forceinline__ void block_segment_sort(const uint64_t* __restrict__ staged, uint32_t s,
                                                   int len, uint32_t tile, K* keys, uint32_t* vals,
                                                   uint64_t* s_x) {
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const uint32_t gbase = w * 64 * R;
  uint64_t x[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = (int)(gbase + lane * R) + k;
    x[k] = i < len ? staged[s + i] : ~0ull;
  }
#pragma unroll
  for (int kk = 2; kk <= kSortWaves * 64 * R; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j >= 64 * R) {
#pragma unroll
        for (int k = 0; k < R; ++k) s_x[gbase + lane * R + k] = x[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const uint32_t i = gbase + lane * R + k;
          const uint64_t y = s_x[i ^ (uint32_t)j];
          const bool keep_min = ((i & (uint32_t)kk) == 0) == ((i & (uint32_t)j) == 0);
          x[k] = ((y < x[k]) == keep_min) ? y : x[k];
        }
        __syncthreads();
      } else {
        bitonic_stage_wave<R>(x, lane, gbase, kk, j);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = (int)(gbase + lane * R) + k;
    if (i < len) seg_store(keys, vals, (int64_t)s + i, tile, x[k]);
  }
}

// Stable LSD radix sort of a long segment by its 64-bit (depth, entry) pair,
// one workgroup, 8 passes of 8 bits between buffers a and b (an even number:
// the result ends in a).  Per kSortThreads-key round, keys are ranked within
// their wavefront by match masks of equal digits and across wavefronts by
// their digit counts, which keeps equal digits in input order.
__device__ void radix_segment_sort(uint64_t* a, uint64_t* b, int64_t len, uint32_t* s_cnt,
                                   uint32_t* s_wdig /* [kSortWaves][256] */) {
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 8 * pass;
    if (threadIdx.x < 256) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < len; i += kSortThreads)
      atomicAdd(&s_cnt[(uint32_t)(a[i] >> shift) & 255u], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {   // first output slot of every digit
      uint32_t run = 0;
      for (int d = 0; d < 256; ++d) {
        const uint32_t c = s_cnt[d];
        s_cnt[d] = run;
        run += c;
      }
    }
    __syncthreads();
    for (int64_t c0 = 0; c0 < len; c0 += kSortThreads) {
      const int64_t i = c0 + threadIdx.x;
      const bool valid = i < len;
      const uint64_t k = valid ? a[i] : 0ull;
      const uint32_t dig = valid ? (uint32_t)(k >> shift) & 255u : 0u;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const uint64_t m = __ballot((dig >> bit) & 1u);
        peers &= ((dig >> bit) & 1u) ? m : ~m;
      }
      const uint32_t below = (uint32_t)__popcll(peers & ((uint64_t(1) << lane) - 1));
      for (int d = threadIdx.x; d < kSortWaves * 256; d += kSortThreads) s_wdig[d] = 0u;
      __syncthreads();
      if (valid && below == 0) s_wdig[w * 256 + dig] = (uint32_t)__popcll(peers);
      __syncthreads();
      if (valid) {
        uint32_t off = s_cnt[dig] + below;
        for (uint32_t q = 0; q < w; ++q) off += s_wdig[q * 256 + dig];
        b[off] = k;
      }
      __syncthreads();
      if (threadIdx.x < 256) {
        uint32_t add = 0;
        for (int q = 0; q < kSortWaves; ++q) add += s_wdig[q * 256 + threadIdx.x];
        s_cnt[threadIdx.x] += add;
      }
      __syncthreads();
    }
    uint64_t* t = a;
    a = b;
    b = t;
    __syncthreads();
  }
}

// Grid kLongSlots + T / kSortWaves.  The first kLongSlots workgroups take
// the queued lists longer than kSegShort (all wavefronts of a workgroup up to
// kSegLong pairs, else the radix sort, whose pair buffers are `staged` itself
// and `spare`); they are dispatched first, so the long lists run beside the
// short ones.  In every later workgroup each wavefront sorts one tile's list
// of up to kSegShort pairs in registers.
template <typename K>
__global__ __launch_bounds__(kSortThreads) void seg_sort_kernel(const uint32_t* __restrict__ ranges,
                                                                int n_tiles,
                                                                uint64_t* __restrict__ staged,
                                                                uint64_t* __restrict__ spare,
                                                                K* __restrict__ keys,
                                                                uint32_t* __restrict__ vals,
                                                                const uint32_t* __restrict__ long_list,
                                                                const uint32_t* __restrict__ n_long) {
  __shared__ uint64_t s_mem[kSegLong + 128];   // pairs, or the radix sort's digit counts
  if (blockIdx.x < (unsigned)kLongSlots) {
    uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_mem + kSegLong);
    uint32_t* s_wdig = reinterpret_cast<uint32_t*>(s_mem);
    const uint32_t count = *n_long;
    for (uint32_t q = blockIdx.x; q < count; q += kLongSlots) {
      const uint32_t tile = long_list[q];
      const uint32_t s = ranges[2 * (int64_t)tile], e = ranges[2 * (int64_t)tile + 1];
      const int64_t len = (int64_t)e - (int64_t)s;
      if (len <= kSegLong / 2) {
        block_segment_sort<kSegLong / (2 * kSortThreads)>(staged, s, (int)len, tile, keys, vals, s_mem);
      } else if (len <= kSegLong) {
        block_segment_sort<kSegLong / kSortThreads>(staged, s, (int)len, tile, keys, vals, s_mem);
      } else {
        radix_segment_sort(staged + s, spare + s, len, s_cnt, s_wdig);
        for (int64_t i = threadIdx.x; i < len; i += kSortThreads)
          seg_store(keys, vals, (int64_t)s + i, tile, staged[s + i]);
      }
      __syncthreads();   // LDS reused by the next list
    }
    return;
  }
  const int tile = (int)(blockIdx.x - kLongSlots) * kSortWaves + (int)(threadIdx.x >> 6);
  if (tile >= n_tiles) return;
  const uint32_t s = ranges[2 * (int64_t)tile], e = ranges[2 * (int64_t)tile + 1];
  const int64_t len = (int64_t)e - (int64_t)s;   // 0 for every tile on overflow
  const uint32_t t = (uint32_t)tile;
  if (len <= 0 || len > kSegShort) return;
  if (len <= 64) wave_segment_sort<1>(staged, s, (int)len, t, keys, vals);
  else if (len <= 128) wave_segment_sort<2>(staged, s, (int)len, t, keys, vals);
  else if (len <= 256) wave_segment_sort<4>(staged, s, (int)len, t, keys, vals);
  else if (len <= 512) wave_segment_sort<8>(staged, s, (int)len, t, keys, vals);
  else wave_segment_sort<16>(staged, s, (int)len, t, keys, vals);
}

// Start of a call that ends before the segments exist: all ranges empty and,
// when an order is requested, the identity order.
__global__ __launch_bounds__(256) void clear_bins_kernel(uint32_t* __restrict__ ranges, int n_tiles,
                                                         uint32_t* __restrict__ order) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  ranges[2 * (int64_t)t] = 0u;
  ranges[2 * (int64_t)t + 1] = 0u;
  if (order) order[t] = (uint32_t)t;
}

// ---------------------------------------------------------------------------
// tile order, longest lists first
// ---------------------------------------------------------------------------

// A stable sort of the tiles by 32 list length groups (0, then half
// octaves), longest group first and ascending tile index within a group, so
// that tiles running side by side stay close in the image.  Three passes over
// blocks of kOrderBlock tiles: group counts per block, per-(block, group)
// output offsets, stable scatter.
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

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t bin_chunks(int64_t n) { return (n + kBinChunk - 1) / kBinChunk; }   // at most

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
  P.chunks = bin_chunks(n);
  P.lds_tiles = 1;
  P.max_view_tiles = 1;
  for (int v = 0; v < vt.n_views; ++v) {
    P.max_view_tiles = std::max(P.max_view_tiles, vt.v[v].tiles_x * vt.v[v].tiles_y);
    P.lds_tiles = std::max(P.lds_tiles, std::min(kLdsTiles, vt.v[v].tiles_x * vt.v[v].tiles_y));
  }
  const size_t nt = sizeof(uint32_t) * (size_t)std::max(vt.n_tiles, 1);
  size_t off = 0;
  P.off_matrix = off;    off += align_up(sizeof(uint32_t) * (size_t)P.chunks * (size_t)vt.n_tiles);
  P.off_list = off;      off += align_up(sizeof(uint4) * (size_t)P.n_entries);      // compacted splats
  P.off_ids = off;       off += align_up(sizeof(uint32_t) * (size_t)P.n_entries);   // their entries
  P.off_list_count = off; off += align_up(sizeof(uint32_t) * GS_MAX_VIEWS);
  P.off_counts = off;    off += align_up(nt);   // keys per tile
  P.off_starts = off;    off += align_up(nt);   // first slot of every tile's segment
  P.off_long = off;      off += align_up(nt);   // tiles whose lists the long grid sorts
  P.off_flag = off;      off += align_up(sizeof(uint64_t) * 2);   // key count, long-list count
  P.off_partial = off;   // per scan block: its tiles' key count
  off += align_up(sizeof(uint64_t) * (size_t)std::max(1, (vt.n_tiles + kScanBlock - 1) / kScanBlock));
  P.off_order = off;     // tile order: per-(block, group) counts, then offsets
  off += align_up(sizeof(uint32_t) * kOrderGroups * ((vt.n_tiles + kOrderBlock - 1) / kOrderBlock));
  P.off_staged = off;    off += align_up(sizeof(uint64_t) * (size_t)capacity);   // (depth, entry) pairs
  P.off_spare = off;     off += align_up(sizeof(uint64_t) * (size_t)capacity);   // radix partner
  P.total = off;
  return P;
}

int run_bin_sort(const gs_projected& p, int64_t n, const ViewTable& vt, const gs_bins& bins,
                 uint32_t* n_keys_host, char* ws, const BinSortPlan& P, hipStream_t s) {
  auto* matrix = reinterpret_cast<uint32_t*>(ws + P.off_matrix);
  auto* list = reinterpret_cast<uint4*>(ws + P.off_list);
  auto* ids = reinterpret_cast<uint32_t*>(ws + P.off_ids);
  auto* list_count = reinterpret_cast<uint32_t*>(ws + P.off_list_count);
  auto* counts = reinterpret_cast<uint32_t*>(ws + P.off_counts);
  auto* starts = reinterpret_cast<uint32_t*>(ws + P.off_starts);
  auto* long_list = reinterpret_cast<uint32_t*>(ws + P.off_long);
  auto* total = reinterpret_cast<uint64_t*>(ws + P.off_flag);
  auto* n_long = reinterpret_cast<uint32_t*>(ws + P.off_flag + sizeof(uint64_t));
  auto* partial = reinterpret_cast<uint64_t*>(ws + P.off_partial);
  auto* order_blk = reinterpret_cast<uint32_t*>(ws + P.off_order);
  auto* staged = reinterpret_cast<uint64_t*>(ws + P.off_staged);
  auto* spare = reinterpret_cast<uint64_t*>(ws + P.off_spare);
  const auto* xy = reinterpret_cast<const float2*>(p.xy);
  const auto* rd = reinterpret_cast<const float4*>(p.rgb_depth);
  const int T = vt.n_tiles;
  const size_t lds = sizeof(uint32_t) * (size_t)P.lds_tiles;
  hipError_t e;

  kernel_event_start(GS_KERNEL_BIN_SORT, s);
  if (T == 0) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, s, bins.n_keys, 0u, (int64_t)1);
    if (bins.queue)
      hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, s, bins.queue, 0u,
                         (int64_t)GS_QUEUE_WORDS);
    kernel_event_stop(GS_KERNEL_BIN_SORT, s);
    return (e = hipGetLastError()) == hipSuccess ? GS_OK : hip_fail(e, "bin sort launch");
  }
  const unsigned tblocks = (unsigned)((T + 255) / 256);
  const dim3 bin_grid((unsigned)std::min<int64_t>(kBinGrid, std::max<int64_t>(P.chunks, 1)),
                      (unsigned)vt.n_views);
  // 1. the splats that touch a tile, per view; keys per (chunk, tile), per
  // tile, the segments and the key count
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, s, list_count, 0u,
                     (int64_t)vt.n_views);
  if (n > 0) {
    hipLaunchKernelGGL(bin_compact_kernel, dim3((unsigned)((n + kCompactChunk - 1) / kCompactChunk),
                       (unsigned)vt.n_views), dim3(256), 0, s, xy, p.radius, rd, p.tiles, n,
                       list_count, list, ids);
    hipLaunchKernelGGL(bin_hist_kernel, bin_grid, dim3(kBinThreads), lds, s, list, list_count, n,
                       vt, P.lds_tiles, matrix);
  }
  hipLaunchKernelGGL(bin_column_kernel, dim3((unsigned)((P.max_view_tiles + 255) / 256),
                     (unsigned)vt.n_views), dim3(256), 0, s, matrix, list_count, vt, counts);
  const int nsb = (T + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(bin_scan_reduce_kernel, dim3((unsigned)nsb), dim3(256), 0, s, counts, T,
                     partial, n_long, bins.queue);
  hipLaunchKernelGGL(bin_scan_down_kernel, dim3((unsigned)nsb), dim3(256), 0, s, counts, T,
                     partial, nsb, P.capacity, bins.ranges, starts, total, bins.n_keys, long_list,
                     n_long);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "bin count launch");

  bool empty = false;
  if (n_keys_host) {
    uint64_t tot = 0;
    if ((e = hipMemcpyAsync(&tot, total, sizeof(uint64_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return hip_fail(e, "read key count");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "synchronise key count");
    *n_keys_host = tot > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)tot;
    if (tot > (uint64_t)P.capacity) {
      if (bins.order)   // ranges are all empty: the identity is the order
        hipLaunchKernelGGL(clear_bins_kernel, dim3(tblocks), dim3(256), 0, s, bins.ranges, T,
                           bins.order);
      kernel_event_stop(GS_KERNEL_BIN_SORT, s);
      set_error("gs_bin_sort: %llu keys exceed capacity %lld", (unsigned long long)tot,
                (long long)P.capacity);
      return GS_ERR_CAPACITY;
    }
    empty = tot == 0;
  }
  // 2. placement into the segments, then each segment sorted by (depth, entry)
  if (n > 0 && !empty) {
    hipLaunchKernelGGL(bin_emit_kernel, bin_grid, dim3(kBinThreads), lds, s, list, ids, list_count,
                       n, vt, P.lds_tiles, matrix, starts, total, P.capacity, staged);
    const unsigned sblocks = (unsigned)(kLongSlots + (T + kSortWaves - 1) / kSortWaves);
    if (bins.keys)
      hipLaunchKernelGGL(seg_sort_kernel<uint64_t>, dim3(sblocks), dim3(kSortThreads), 0, s,
                         bins.ranges, T, staged, spare, bins.keys, bins.values, long_list, n_long);
    else
      hipLaunchKernelGGL(seg_sort_kernel<uint32_t>, dim3(sblocks), dim3(kSortThreads), 0, s,
                         bins.ranges, T, staged, spare, (uint32_t*)nullptr, bins.values, long_list,
                         n_long);
  }
  // 3. launch order of the compositing grids (from the ranges; on overflow
  // they are all empty and this is the identity)
  if (bins.order) {
    const int nblk = (T + kOrderBlock - 1) / kOrderBlock;
    hipLaunchKernelGGL(order_count_kernel, dim3((unsigned)nblk), dim3(kOrderBlock), 0, s,
                       bins.ranges, T, order_blk);
    hipLaunchKernelGGL(order_offsets_kernel, dim3(1), dim3(1024), 0, s, order_blk, nblk);
    hipLaunchKernelGGL(order_scatter_kernel, dim3((unsigned)nblk), dim3(kOrderBlock), 0, s,
                       bins.ranges, T, order_blk, bins.order);
  }
  kernel_event_stop(GS_KERNEL_BIN_SORT, s);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "bin sort launch");
  return GS_OK;
}

}  // namespace gsmi
