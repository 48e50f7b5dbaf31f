// Binning kernels: stream compaction of visible (view, Gaussian) slots, device-wide scans, an
// LDS-staged wavefront LSD radix sort, range detection and the row binning.
//
// Binning follows the tile-based rasterizer the paper adopts (Sec. 3.2): every splat is
// listed in each screen tile its reach ellipse touches, and each tile's list is ordered by
// camera depth, front to back (Sec. 3.1 composites the splats in depth order).  Here the
// depth order is made once per visible splat (a 32-bit depth sort of the compacted slots); the
// splats' runs of tiles per tile row are then emitted in depth order, sorted stably by tile
// row alone and expanded into the tile lists, so each tile's list inherits the depth order
// (ties keep the slot order, i.e. the Gaussian index).
#include <hip/hip_runtime.h>
#include <algorithm>

#include "g4d_internal.h"

namespace g4d {
namespace {

constexpr int kThreads = kSortThreads;          // 4 waves of 64
constexpr int kItems = kScanItems;              // 16 items per thread
constexpr int kPerThread = kItems / kThreads;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
// Items per workgroup of a radix pass (a multiple of 4 x 64).  Measured on the 300k/16-view
// workload with 32-bit tile keys (35.7M pairs, 14-bit tile ids): 4096 sorts the tiles in
// 0.632 ms, 2048 in 0.649, 8192 in 0.797 (two workgroups per CU for its 70 KB of LDS);
// splitting the 14 bits evenly (7 + 7) instead of 8 + 6 gains nothing (0.636).  With 16-bit
// keys (26.1M pairs, 15-bit ids): 4096 in 0.398 ms, 2048 in 0.422, 8192 in 0.513; the depth
// sort (1.8M slots, 32-bit keys) takes 0.149, 0.143 and 0.201 ms.
#ifndef G4D_RADIX_ITEMS
#define G4D_RADIX_ITEMS 4096
#endif
constexpr int kRadixItems = G4D_RADIX_ITEMS;
constexpr int kRadixPerThread = kRadixItems / kThreads;
static_assert(kRadixItems % (4 * 64) == 0, "radix items per workgroup");

// Orders a wave's LDS writes before its later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}


// Exclusive scan of one value per thread over a 256-thread block; also returns the total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t& total, uint32_t* lds4) {
  const uint32_t inc = wave_incl_scan(x);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) lds4[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t s = lds4[k];
    pre += (k < w) ? s : 0u;
    total += s;
  }
  __syncthreads();
  return pre + inc - x;
}

// ------------------------------------------------------------------------------------------
// Generic three-phase exclusive scan: per-block sums, a one-block scan of the sums, and a
// per-block scan that hands (index, exclusive prefix, value) to an output functor.
// ------------------------------------------------------------------------------------------
struct InFlag {
  const uint32_t* p;
  __device__ uint32_t operator()(int64_t i) const { return p[i] > 0u ? 1u : 0u; }
};
// Gathers cnt[idx[i]] and keeps it at keep[i], so that a second pass over the same items
// reads them contiguously instead of gathering again (each gather costs a cache line).
struct InGatherKeep {
  const uint32_t* cnt;
  const uint32_t* idx;
  uint32_t* keep;
  __device__ uint32_t operator()(int64_t i) const {
    const uint32_t c = cnt[idx[i]];
    keep[i] = c;
    return c;
  }
};
struct InPlain {
  const uint32_t* p;
  __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct OutStore {
  uint32_t* out;
  __device__ void operator()(int64_t i, uint32_t excl, uint32_t) const { out[i] = excl; }
};
struct OutCompact {
  const uint32_t* dkey;
  uint32_t* okey;
  uint32_t* oval;
  __device__ void operator()(int64_t i, uint32_t excl, uint32_t v) const {
    if (v) {
      okey[excl] = dkey[i];
      oval[excl] = (uint32_t)i;
    }
  }
};

__device__ __forceinline__ int64_t count_of(const uint32_t* n_dev, int64_t n_host) {
  return n_dev ? (int64_t)*n_dev : n_host;
}

template <class In>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(In in, const uint32_t* n_dev,
                                                          int64_t n_host, uint32_t* sums) {
  __shared__ uint32_t lds[4];
  const int64_t n = count_of(n_dev, n_host);
  const int64_t base = (int64_t)blockIdx.x * kItems;
  uint32_t acc = 0;
  if (base < n) {
    // all of the thread's loads are issued before any is used (a gathered input costs two
    // dependent memory round trips per block, not two per row)
    uint32_t v[kPerThread];
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
      const int64_t i = base + r * kThreads + threadIdx.x;
      v[r] = (i < n) ? in(i) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) acc += v[r];
  }
  uint32_t total;
  block_excl_scan(acc, total, lds);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block: exclusive scan of `count` sums in place; writes the grand total.
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t* sums, int count, uint32_t* total) {
  __shared__ uint32_t lds[16];
  uint32_t carry = 0;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int base = 0; base < count; base += 1024) {
    const int i = base + threadIdx.x;
    const uint32_t x = (i < count) ? sums[i] : 0u;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      pre += (k < w) ? lds[k] : 0u;
      tot += lds[k];
    }
    if (i < count) sums[i] = carry + pre + inc - x;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// Row r of a block holds items base + r * kThreads + t.  Every row is loaded first, each is
// scanned within its wave, and one barrier publishes the per-(row, wave) totals from which
// each item's block prefix follows.  With kOwnPrefix the block adds up the totals of the
// blocks before it (`sums` as the reduce pass left them) instead of reading a prefix scanned
// by k_scan_sums, and the block holding the last item writes the grand total.
template <class In, class Out, bool kOwnPrefix>
__global__ __launch_bounds__(kThreads) void k_scan_apply(In in, Out out, const uint32_t* n_dev,
                                                         int64_t n_host, const uint32_t* sums,
                                                         uint32_t* total) {
  __shared__ uint4 lds[kPerThread];  // [row] -> totals of the 4 waves
  __shared__ uint32_t lds_pre[4];
  const int64_t n = count_of(n_dev, n_host);
  const int64_t base = (int64_t)blockIdx.x * kItems;
  if (base >= n) {
    if (kOwnPrefix && blockIdx.x == 0 && threadIdx.x == 0 && total) *total = 0u;
    return;
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t v[kPerThread], inc[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t i = base + r * kThreads + threadIdx.x;
    v[r] = (i < n) ? in(i) : 0u;
  }
  if (kOwnPrefix) {
    uint32_t part = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kThreads) part += sums[k];
    part = wave_incl_scan(part);
    if (lane == 63) lds_pre[w] = part;
  }
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    inc[r] = wave_incl_scan(v[r]);
    if (lane == 63) reinterpret_cast<uint32_t*>(&lds[r])[w] = inc[r];
  }
  __syncthreads();
  uint32_t carry =
      kOwnPrefix ? lds_pre[0] + lds_pre[1] + lds_pre[2] + lds_pre[3] : sums[blockIdx.x];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const uint4 t = lds[r];
    const uint32_t pre = (w > 0 ? t.x : 0u) + (w > 1 ? t.y : 0u) + (w > 2 ? t.z : 0u);
    const int64_t i = base + r * kThreads + threadIdx.x;
    if (i < n) out(i, carry + pre + inc[r] - v[r], v[r]);
    carry += t.x + t.y + t.z + t.w;
  }
  if (kOwnPrefix && total && threadIdx.x == 0 && base + kItems >= n) *total = carry;
}

// Up to this many blocks each apply block sums the totals before it (at most 8 KB of reads
// from L2 per block), which saves the one-block k_scan_sums launch.
constexpr int64_t kOwnPrefixBlocks = 2048;

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v);

// The reduce pass reads items through `in_sum`, the apply pass through `in`; both must yield
// the same values.
template <class InSum, class In, class Out>
void scan_generic(InSum in_sum, In in, Out out, const uint32_t* n_dev, int64_t n_cap,
                  uint32_t* total, void* scratch, hipStream_t st) {
  const int64_t blocks = (n_cap + kItems - 1) / kItems;
  if (blocks == 0) {
    if (total) fill_u32(total, 1, 0u, st);
    return;
  }
  uint32_t* sums = static_cast<uint32_t*>(scratch);
  hipLaunchKernelGGL(k_scan_reduce<InSum>, dim3((unsigned)blocks), dim3(kThreads), 0, st, in_sum,
                     n_dev, n_cap, sums);
  if (blocks <= kOwnPrefixBlocks) {
    hipLaunchKernelGGL((k_scan_apply<In, Out, true>), dim3((unsigned)blocks), dim3(kThreads), 0,
                       st, in, out, n_dev, n_cap, sums, total);
    return;
  }
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, sums, (int)blocks, total);
  hipLaunchKernelGGL((k_scan_apply<In, Out, false>), dim3((unsigned)blocks), dim3(kThreads), 0,
                     st, in, out, n_dev, n_cap, sums, nullptr);
}

// ------------------------------------------------------------------------------------------
// Radix sort pass: digit histogram per block, scan of the (digit, block) table, and a
// stable scatter.  Each wave owns a contiguous 1024-item run of its block; ranks inside a
// wave come from ballot-based digit matching, so equal digits keep their input order.
// ------------------------------------------------------------------------------------------
// NT threads per workgroup, 16 items per thread: 256 (4096 items), or 512 for long sorts, whose
// scatter then writes runs of one digit about twice as long (8192 items over 256 digits) with
// two workgroups still resident per CU.  Tile sort of the 300k-Gaussian, 16-view workload
// (26.1M pairs, 16-bit keys): 0.399 ms at 256 threads, 0.368-0.375 at 512, 0.477 at 384
// (three workgroups per CU, shorter runs), 0.442 at 768 and 0.399 at 1024 (one workgroup per
// CU, which serializes its load, rank and write phases).
#ifndef G4D_WIDE_THREADS
#define G4D_WIDE_THREADS 512
#endif
constexpr int kWideThreads = G4D_WIDE_THREADS;

template <typename K, int NT>
__global__ __launch_bounds__(NT) void k_radix_hist(const K* __restrict__ key,
                                                   const uint32_t* n_dev, int shift,
                                                   uint32_t mask, uint32_t* hist, int nblocks) {
  constexpr int NW = NT / 64, ITEMS = NT * kRadixPerThread;
  __shared__ uint32_t wh[NW][kRadix];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int d = threadIdx.x; d < NW * kRadix; d += NT) (&wh[0][0])[d] = 0;
  __syncthreads();
  const int64_t n = *n_dev;
  const int64_t base = (int64_t)blockIdx.x * ITEMS + w * (ITEMS / NW);
#pragma unroll 4
  for (int r = 0; r < kRadixPerThread; ++r) {
    const int64_t i = base + r * 64 + lane;
    if (i < n) atomicAdd(&wh[w][((uint32_t)key[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += NT) {
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) t += wh[k][d];
    hist[(int64_t)d * nblocks + blockIdx.x] = t;
  }
}

__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
  uint64_t peers = valid;
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

template <typename K, int NT, typename V>
__global__ __launch_bounds__(NT) void k_radix_scatter(
    const K* __restrict__ kin, const V* __restrict__ vin, K* __restrict__ kout,
    V* __restrict__ vout, const uint32_t* n_dev, int shift, uint32_t mask,
    const uint32_t* __restrict__ hist, int nblocks) {
  constexpr int NW = NT / 64, ITEMS = NT * kRadixPerThread;
  static_assert(NT >= kRadix, "one thread per digit");
  __shared__ uint32_t wcount[NW][kRadix];
  __shared__ uint32_t bstart[kRadix];
  __shared__ uint32_t goff[kRadix];
  __shared__ K sk[ITEMS];
  __shared__ V sv[ITEMS];
  __shared__ uint32_t lds4[4];
  const int64_t n = *n_dev;
  const int64_t bbase = (int64_t)blockIdx.x * ITEMS;
  if (bbase >= n) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int d = threadIdx.x; d < NW * kRadix; d += NT) (&wcount[0][0])[d] = 0;
  __syncthreads();
  const int64_t base = bbase + w * (ITEMS / NW);
  const uint64_t lt = lanemask_lt();
  uint32_t k[kRadixPerThread], rank[kRadixPerThread];
  V v[kRadixPerThread];
#pragma unroll
  for (int r = 0; r < kRadixPerThread; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool valid = i < n;
    k[r] = valid ? (uint32_t)kin[i] : 0u;
    v[r] = valid ? vin[i] : V{};
    const uint32_t d = (k[r] >> shift) & mask;
    const uint64_t peers = match_digit(d, __ballot(valid));
    const uint32_t before = wcount[w][d];
    rank[r] = before + (uint32_t)__popcll(peers & lt);
    __builtin_amdgcn_wave_barrier();
    if (valid && (peers & lt) == 0ull) wcount[w][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // Per-digit totals, exclusive prefix over waves (in place) and over digits (bstart): the
  // first 256 threads hold one digit each.
  uint32_t tot = 0;
  if (threadIdx.x < kRadix) {
    const int d = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const uint32_t c = wcount[q][d];
      wcount[q][d] = tot;
      tot += c;
    }
    goff[d] = hist[(int64_t)d * nblocks + blockIdx.x];
  }
  const uint32_t inc = wave_incl_scan(tot);  // waves past the digits scan zeros
  if (lane == 63 && w < 4) lds4[w] = inc;
  __syncthreads();
  if (threadIdx.x < kRadix) {
    uint32_t pre = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) pre += (q < w) ? lds4[q] : 0u;
    bstart[threadIdx.x] = pre + inc - tot;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRadixPerThread; ++r) {
    const int64_t i = base + r * 64 + lane;
    if (i < n) {
      const uint32_t d = (k[r] >> shift) & mask;
      const uint32_t pos = bstart[d] + wcount[w][d] + rank[r];
      sk[pos] = (K)k[r];
      sv[pos] = v[r];
    }
  }
  __syncthreads();
  const int cnt = (int)((n - bbase) < ITEMS ? (n - bbase) : ITEMS);
  for (int p = threadIdx.x; p < cnt; p += NT) {
    const uint32_t kk = (uint32_t)sk[p];
    const uint32_t d = (kk >> shift) & mask;
    const uint32_t dst = goff[d] + ((uint32_t)p - bstart[d]);
    kout[dst] = (K)kk;
    vout[dst] = sv[p];
  }
}

// ------------------------------------------------------------------------------------------
// Row binning.  The tiles a splat is listed in are, in each tile row of its box, one run of
// columns (tile_row_span).  Instead of one (tile, splat) pair per tile, sorted by tile, the
// runs are emitted (one per box row, visible splats in depth order), sorted stably by their
// global tile row, and expanded: each row's runs are taken 64 at a time (a chunk, one wave), a
// count pass tallies how many runs of the chunk cover each column, an exclusive scan over
// (tile, chunk) in tile order gives every chunk its place in each tile's list, and a write
// pass lays the slots down.  A tile's list so holds its splats in depth order (the runs enter
// the stable row sort in depth order), exactly as a stable sort of the individual pairs by
// tile would leave them; the sort moves one item per run instead of one per pair.
// ------------------------------------------------------------------------------------------

// One run per box row of every visible splat, in depth order: each wave takes 64 consecutive
// visible entries, numbers their rows with a wave scan and deals them out 64 per round; the
// run of row k lands at roff[first] + k.  rkey = global tile row, rval = (slot, span) with
// span = (first column << 16) | last, or ~0u for a row the ellipse misses.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_rowgen(
    const float* __restrict__ rec, const uint32_t* __restrict__ vval,
    const uint32_t* __restrict__ roff, const uint32_t* n_vis_dev, const uint32_t* n_rows_dev,
    int64_t row_cap, int n_per_view, const DView* __restrict__ views, DSettings S,
    K* __restrict__ rkey, uint2* __restrict__ rval, uint32_t* flag) {
  __shared__ uint32_t s_rows[4][64];
  __shared__ float s_u[4][64], s_v[4][64], s_a[4][64], s_b[4][64], s_c[4][64];
  __shared__ float s_ex[4][64], s_ey[4][64], s_lim[4][64];
  __shared__ int32_t s_x0[4][64], s_x1[4][64], s_y0[4][64], s_w[4][64], s_h[4][64], s_rb[4][64];
  __shared__ uint32_t s_slot[4][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t n_vis = *n_vis_dev;
  const int64_t first = ((int64_t)blockIdx.x * 4 + w) * 64;
  if (first >= n_vis) return;
  const int64_t r = first + lane;
  const int64_t last = (n_vis - first < 64 ? n_vis : first + 64) - 1;
  const uint32_t off0 = roff[first];
  const uint32_t off_end = (last + 1 < n_vis) ? roff[last + 1] : *n_rows_dev;
  uint32_t rows = 0;
  if (r < n_vis) {
    const uint32_t slot = vval[r];
    const DView& V = views[(int)(slot / (uint32_t)n_per_view)];
    const float* p = rec + (size_t)slot * kRec;
    int x0, x1, y0, y1;
    if (tile_rect(p[R_U], p[R_V], p[R_EX], p[R_EY], V, S.tile_shift, x0, x1, y0, y1))
      rows = (uint32_t)(y1 - y0 + 1);
    s_u[w][lane] = p[R_U];
    s_v[w][lane] = p[R_V];
    s_a[w][lane] = p[R_A];
    s_b[w][lane] = p[R_B];
    s_c[w][lane] = p[R_C];
    s_ex[w][lane] = p[R_EX];
    s_ey[w][lane] = p[R_EY];
    s_lim[w][lane] = coverage_limit(p[R_OPT], S);
    s_x0[w][lane] = x0;
    s_x1[w][lane] = x1;
    s_y0[w][lane] = y0;
    s_w[w][lane] = V.width;
    s_h[w][lane] = V.height;
    s_rb[w][lane] = V.row_base;
    s_slot[w][lane] = slot;
  }
  uint32_t n_rows;
  const uint32_t row0 = wave_excl_scan(rows, n_rows);
  s_rows[w][lane] = (r < n_vis) ? row0 : n_rows;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // the row offsets were scanned from the same boxes; a disagreement is reported and nothing
  // is written past this wave's share
  if (off0 + n_rows != off_end && lane == 0) *flag = 2u;
  for (uint32_t k0 = 0; k0 < n_rows; k0 += 64) {
    const uint32_t k = k0 + lane;
    if (k >= n_rows) continue;
    int lo = 0, hi = 63;  // the last lane whose rows start at or before k owns row k
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_rows[w][mid] <= k) lo = mid; else hi = mid - 1;
    }
    const int ty = s_y0[w][lo] + (int)(k - s_rows[w][lo]);
    const int span = tile_row_span(s_u[w][lo], s_v[w][lo], s_a[w][lo], s_b[w][lo], s_c[w][lo],
                                   s_lim[w][lo], s_ex[w][lo], s_ey[w][lo], ty, S.tile_shift,
                                   s_w[w][lo], s_h[w][lo], s_x0[w][lo], s_x1[w][lo]);
    const uint32_t pos = off0 + k;
    if (pos < off_end && (int64_t)pos < row_cap) {
      rkey[pos] = (K)(s_rb[w][lo] + ty);
      rval[pos] = make_uint2(s_slot[w][lo], span >= 0 ? (uint32_t)span : ~0u);
    } else if ((int64_t)pos >= row_cap) {
      *flag = 1u;
    }
  }
}

// The chunks of tile row r are expanded on XCD r % 8 (workgroup b runs on XCD b % 8): a row's
// pairs then fill whole cache lines in one L2 before they are written back, instead of
// reaching memory as partial lines from several XCDs.
constexpr int kXcds = 8;

// Per tile row r (one workgroup walks all rows): its runs [lo, lo + len) in the sorted run
// list, its chunks of 64 runs and the index of its first chunk among the chunks of its XCD,
// and the base of its (column, chunk) count table: rinfo[2r] = (lo, len, first chunk, table
// base), rinfo[2r + 1] = (chunks, tiles_x, first tile id, 0).  totals = (chunks of XCD 0..7,
// table entries).
__global__ __launch_bounds__(1024) void k_row_table(const uint2* __restrict__ rrange, int n_rows,
                                                    const DView* __restrict__ views, int n_views,
                                                    uint4* __restrict__ rinfo, uint32_t hist_cap,
                                                    uint32_t* totals) {
  __shared__ uint32_t s_c[16][kXcds], s_h[16];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int x = threadIdx.x % kXcds;  // every 1024-row group starts at a multiple of 8
  uint32_t carry_c = 0, carry_h = 0;
  for (int base = 0; base < n_rows; base += 1024) {
    const int r = base + threadIdx.x;
    uint32_t lo = 0, len = 0, nch = 0, nx = 0, tile0 = 0;
    if (r < n_rows) {
      int a = 0, b = n_views - 1;  // the last view whose rows start at or before r
      while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (views[m].row_base <= r) a = m; else b = m - 1;
      }
      const DView& V = views[a];
      nx = (uint32_t)V.tiles_x;
      tile0 = (uint32_t)(V.tile_base + (r - V.row_base) * V.tiles_x);
      const uint2 g = rrange[r];
      lo = g.x;
      len = g.y - g.x;
      nch = (len + 63u) >> 6;
    }
    const uint32_t hs = nch * nx;
    // chunks: inclusive scan over the lanes of the same XCD (stride 8); table: over all lanes
    uint32_t ic = nch;
#pragma unroll
    for (int o = kXcds; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(ic, o, 64);
      if (lane >= o) ic += y;
    }
    const uint32_t ih = wave_incl_scan(hs);
    if (lane >= 64 - kXcds) s_c[w][x] = ic;
    if (lane == 63) s_h[w] = ih;
    __syncthreads();
    uint32_t pc = 0, ph = 0, tc = 0, th = 0;
    for (int k = 0; k < 16; ++k) {
      pc += (k < w) ? s_c[k][x] : 0u;
      ph += (k < w) ? s_h[k] : 0u;
      tc += s_c[k][x];
      th += s_h[k];
    }
    if (r < n_rows) {
      rinfo[2 * r] = make_uint4(lo, len, carry_c + pc + ic - nch, carry_h + ph + ih - hs);
      rinfo[2 * r + 1] = make_uint4(nch, nx, tile0, 0u);
    }
    carry_c += tc;
    carry_h += th;
    __syncthreads();
  }
  // (the table capacity covers every run list the row capacity admits; the clamp only keeps
  // a broken count from taking the scan past it)
  if (threadIdx.x < kXcds) totals[threadIdx.x] = carry_c;
  if (threadIdx.x == 0) totals[kXcds] = min(carry_h, hist_cap);
}

// crow[XCD][chunk] = the tile row of each chunk (one workgroup per row); each XCD's list
// holds up to chunk_cap entries.
__global__ void k_chunk_rows(const uint4* __restrict__ rinfo, int64_t chunk_cap,
                             uint32_t* __restrict__ crow) {
  const uint32_t r = blockIdx.x;
  const uint32_t first = rinfo[2 * r].z, nch = rinfo[2 * r + 1].x;
  uint32_t* out = crow + (size_t)(r % kXcds) * chunk_cap;
  for (uint32_t k = threadIdx.x; k < nch && (int64_t)(first + k) < chunk_cap; k += blockDim.x)
    out[first + k] = r;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, (uint32_t)__shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor(x, o, 64));
  return x;
}

// A chunk's runs as column bounds [x0, x1] (x0 > x1: empty), and the wave's column range.
// A run covers columns x0 .. x0 + w (an empty run: x0 = ~0u, w = 0, which no column
// reaches, since column - x0 is then column + 1 > 0).
struct Chunk {
  uint4 a, b;    // rinfo of the row
  uint32_t c;    // chunk within the row
  uint32_t x0, w, cmin, cmax, slot;
};

// Chunk g of the XCD's list (crow is that XCD's row map; wave-uniform values are kept
// scalar, so that the row and its table entries come through scalar loads).
__device__ __forceinline__ void load_chunk(const uint4* __restrict__ rinfo,
                                           const uint32_t* __restrict__ crow, uint32_t g,
                                           const uint2* __restrict__ runs, Chunk& ck) {
  const int lane = threadIdx.x & 63;
  const uint32_t r = __builtin_amdgcn_readfirstlane(crow[g]);
  ck.a = rinfo[2 * r];
  ck.b = rinfo[2 * r + 1];
  ck.c = g - ck.a.z;
  const uint32_t e = ck.c * 64u + (uint32_t)lane;
  ck.x0 = ~0u;
  ck.w = 0u;
  ck.slot = 0u;
  uint32_t x1 = 0u;
  if (e < ck.a.y) {
    const uint2 sv = runs[ck.a.x + e];
    ck.slot = sv.x;
    if (sv.y != ~0u) {
      ck.x0 = sv.y >> 16;
      x1 = sv.y & 0xFFFFu;
      ck.w = x1 - ck.x0;
    }
  }
  ck.cmin = __builtin_amdgcn_readfirstlane(wave_min_u32(ck.x0));
  ck.cmax = __builtin_amdgcn_readfirstlane(wave_max_u32(x1));
}

// Chunks of this workgroup's XCD, 4 per workgroup (one per wave), striding over the grid's
// share of that XCD; the loop ends for every wave once the list is exhausted.
#define FOR_EACH_CHUNK(counts, chunk_cap, crow_base, crow_x, g)                                 \
  const uint32_t xcd_ = blockIdx.x % kXcds;                                                    \
  const uint32_t* crow_x = (crow_base) + (size_t)xcd_ * (chunk_cap);                           \
  const uint32_t n_x_ = (uint32_t)min((int64_t)(counts)[xcd_], (int64_t)(chunk_cap));          \
  const uint32_t step_ = (gridDim.x / kXcds) * 4u;                                             \
  for (uint32_t g = __builtin_amdgcn_readfirstlane((blockIdx.x / kXcds) * 4u + (threadIdx.x >> 6)); \
       g < n_x_; g += step_)

// Count pass: hist[table base + column * chunks + chunk] = runs of the chunk covering the
// column (tile-major, so that one scan over the whole table yields positions in tile order).
// Each wave adds +1 at its runs' first and -1 past their last column in an LDS difference
// array of 256 columns; a prefix sum over it (four columns per lane) gives the counts.
constexpr int kCountCols = 256;
__global__ __launch_bounds__(256) void k_expand_count(const uint4* __restrict__ rinfo,
                                                      const uint32_t* __restrict__ crow,
                                                      int64_t chunk_cap,
                                                      const uint32_t* __restrict__ counts,
                                                      const uint2* __restrict__ runs,
                                                      uint32_t* __restrict__ hist,
                                                      int64_t hist_cap) {
  __shared__ int4 s_diff[4][kCountCols / 4 + 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int* diff = reinterpret_cast<int*>(&s_diff[w][0]);
  FOR_EACH_CHUNK(counts, chunk_cap, crow, crow_x, g) {
    Chunk ck;
    load_chunk(rinfo, crow_x, g, runs, ck);
    const uint32_t nch = ck.b.x, nx = ck.b.y;
    for (uint32_t c0 = 0; c0 < nx; c0 += kCountCols) {
      s_diff[w][lane] = make_int4(0, 0, 0, 0);
      if (lane == 0) s_diff[w][kCountCols / 4] = make_int4(0, 0, 0, 0);
      wave_lds_sync();
      if (ck.x0 != ~0u) {
        const int lo = max((int)ck.x0 - (int)c0, 0);
        const int hi = min((int)(ck.x0 + ck.w) - (int)c0, kCountCols - 1);
        if (lo <= hi) {
          atomicAdd(&diff[lo], 1);
          atomicSub(&diff[hi + 1], 1);
        }
      }
      wave_lds_sync();
      const int4 d = s_diff[w][lane];
      const int p0 = d.x, p1 = p0 + d.y, p2 = p1 + d.z, p3 = p2 + d.w;
      const int base = (int)wave_incl_scan((uint32_t)p3) - p3;
      const int v[4] = {base + p0, base + p1, base + p2, base + p3};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t col = c0 + 4u * (uint32_t)lane + (uint32_t)k;
        const int64_t at = (int64_t)ck.a.w + ck.c + (int64_t)col * nch;
        if (col < nx && at < hist_cap) hist[at] = (uint32_t)v[k];
      }
      wave_lds_sync();  // the next window clears the array
    }
  }
}

// Tile ranges from the scanned table: [start of (tile, chunk 0), start of the next tile), both
// clamped to the pair capacity; an empty tile gets (0, 0).
__global__ void k_expand_ranges(const uint4* __restrict__ rinfo, const DView* __restrict__ views,
                                int n_views, const uint32_t* __restrict__ scanned,
                                const uint32_t* n_hist_dev, const uint32_t* total_dev,
                                const uint32_t* n_pairs_dev, int64_t n_tiles, uint32_t pair_cap,
                                uint2* __restrict__ ranges, uint32_t* flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  // more pairs than the list holds is a capacity overflow; otherwise the preprocess counted the
  // pairs the expansion lays down, and a disagreement is reported (unless a capacity overflow,
  // which clips the runs, already was)
  if (t == 0) {
    if (*total_dev > pair_cap) *flag = 1u;
    else if (*total_dev != *n_pairs_dev && *flag == 0u) *flag = 2u;
  }
  int a = 0, b = n_views - 1;  // the last view whose tiles start at or before t
  while (a < b) {
    const int m = (a + b + 1) >> 1;
    if (views[m].tile_base <= t) a = m; else b = m - 1;
  }
  const DView& V = views[a];
  const int local = (int)(t - V.tile_base);
  const int ty = local / V.tiles_x, tx = local - ty * V.tiles_x;
  const int r = V.row_base + ty;
  const uint4 ra = rinfo[2 * r], rb = rinfo[2 * r + 1];
  uint32_t lo = 0, hi = 0;
  if (rb.x > 0) {
    const uint32_t n_hist = *n_hist_dev;
    const uint32_t i0 = ra.w + (uint32_t)tx * rb.x, i1 = i0 + rb.x;
    lo = i0 < n_hist ? scanned[i0] : *total_dev;
    hi = i1 < n_hist ? scanned[i1] : *total_dev;
    lo = min(lo, pair_cap);
    hi = min(hi, pair_cap);
  }
  ranges[t] = hi > lo ? make_uint2(lo, hi) : make_uint2(0u, 0u);
}

// Write pass: the slots of the chunk's runs covering each column, at the column's scanned
// place plus their rank among the chunk's covering runs.  The places of 64 columns come in
// one load (lane j holds column t0 + j) and are read out per column with readlane; the
// stores go through a buffer resource over the pair list (32-bit offsets).
__global__ __launch_bounds__(256) void k_expand_write(const uint4* __restrict__ rinfo,
                                                      const uint32_t* __restrict__ crow,
                                                      int64_t chunk_cap,
                                                      const uint32_t* __restrict__ counts,
                                                      const uint2* __restrict__ runs,
                                                      const uint32_t* __restrict__ scanned,
                                                      int64_t hist_cap, uint32_t pair_cap,
                                                      uint32_t* __restrict__ pval, uint32_t* flag) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  // pair_cap is at most 2^29 here, so every offset below it fits the 32-bit range
  const __amdgpu_buffer_rsrc_t out =
      __builtin_amdgcn_make_buffer_rsrc(pval, 0, (int)(pair_cap * 4u), 0x00020000);
  FOR_EACH_CHUNK(counts, chunk_cap, crow, crow_x, g) {
    Chunk ck;
    load_chunk(rinfo, crow_x, g, runs, ck);
    const uint32_t nch = ck.b.x, nx = ck.b.y;
    const uint32_t last = min(ck.cmax, nx - 1u);
    bool bad = false;
    for (uint32_t t0 = ck.cmin & ~63u; ck.cmin <= last && t0 <= last && !bad; t0 += 64) {
      const uint32_t col = t0 + (uint32_t)lane;
      const int64_t at = (int64_t)ck.a.w + ck.c + (int64_t)col * nch;
      if (__ballot(col < nx && at >= hist_cap)) {  // never with a table sized for the runs
        if (lane == 0) *flag = 1u;
        bad = true;
        break;
      }
      const uint32_t loaded = (col < nx) ? scanned[at] : 0u;
      // A register move (a DPP identity, which the compiler keeps) takes the wait for the load
      // out of the loop: inside it, a wait for the loaded register would also wait for every
      // store the loop has issued (one counter covers both on this GPU).
      const uint32_t places = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)loaded, 0xE4, 0xF,
                                                                     0xF, false);
      const uint32_t j0 = ck.cmin > t0 ? ck.cmin : t0, j1 = min(last + 1u, t0 + 64u);
      for (uint32_t tx = j0; tx < j1; ++tx) {
        const bool cov = tx - ck.x0 <= ck.w;
        const uint64_t m = __ballot(cov);
        if (m == 0ull) continue;
        const uint32_t base = __builtin_amdgcn_readlane(places, (int)(tx - t0));
        const uint32_t pos = base + (uint32_t)__popcll(m & lt);
        if (cov && pos < pair_cap)
          __builtin_amdgcn_raw_buffer_store_b32(ck.slot, out, (int)(pos * 4u), 0, 0);
      }
    }
  }
}

// Tile id of every listed pair, from the ranges (a workgroup per tile, striding over them).
__global__ void k_tile_ids(const uint2* __restrict__ ranges, int64_t n_tiles, int64_t n,
                           uint32_t* __restrict__ ids) {
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const uint2 g = ranges[t];
    for (uint32_t i = g.x + threadIdx.x; i < g.y && (int64_t)i < n; i += blockDim.x)
      ids[i] = (uint32_t)t;
  }
}

// Tile boundaries in the sorted keys, four keys per thread (one 16-byte load; the neighbours
// on either side come from the caches).
// Four keys per thread (one 4-key vector load), compared with their neighbours.
template <typename K> struct Key4;
template <> struct Key4<uint32_t> { using T = uint4; };
template <> struct Key4<uint16_t> { using T = ushort4; };

template <typename K>
__global__ void k_ranges(const K* __restrict__ key, const uint32_t* n_dev, int64_t cap,
                         int64_t n_tiles, uint2* ranges) {
  const int64_t n = (int64_t)*n_dev < cap ? (int64_t)*n_dev : cap;
  const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (i0 >= n) return;
  uint32_t k[6];  // key[i0 - 1 .. i0 + 4]
  if (i0 + 4 <= n) {
    const typename Key4<K>::T q = *reinterpret_cast<const typename Key4<K>::T*>(key + i0);
    k[1] = q.x;
    k[2] = q.y;
    k[3] = q.z;
    k[4] = q.w;
  } else {
    for (int j = 0; j < 4; ++j) k[1 + j] = (i0 + j < n) ? (uint32_t)key[i0 + j] : 0u;
  }
  k[0] = i0 > 0 ? (uint32_t)key[i0 - 1] : 0u;
  k[5] = i0 + 4 < n ? (uint32_t)key[i0 + 4] : 0u;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t i = i0 + j;
    if (i >= n) break;
    const uint32_t kk = k[1 + j];
    if ((int64_t)kk >= n_tiles) continue;  // dummy tile
    if (i == 0 || k[j] != kk) ranges[kk].x = (uint32_t)i;
    if (i == n - 1 || k[2 + j] != kk) ranges[kk].y = (uint32_t)(i + 1);
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_clamp_count(const uint32_t* n, uint32_t cap, uint32_t* out) {
  if (threadIdx.x == 0) *out = min(*n, cap);
}

__global__ void k_view_setup(DView* views, int n_views, float m) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_views) return;
  DView& V = views[v];
  for (int j = 0; j < 3; ++j)
    V.C[j] = -(V.W[j] * V.tau[0] + V.W[3 + j] * V.tau[1] + V.W[6 + j] * V.tau[2]);
  V.xlo = (-m * (float)V.width - V.cx) / V.fx;
  V.xhi = ((1.f + m) * (float)V.width - V.cx) / V.fx;
  V.ylo = (-m * (float)V.height - V.cy) / V.fy;
  V.yhi = ((1.f + m) * (float)V.height - V.cy) / V.fy;
}

}  // namespace

// Plain fill kernel (used instead of memset nodes so that the sequence can be graph-captured).
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

size_t scan_scratch_bytes(int64_t n) {
  return sizeof(uint32_t) * (size_t)((n + kItems - 1) / kItems + 1);
}

void compact_visible(const uint32_t* tiles, const uint32_t* dkey, int64_t n_slots,
                     uint32_t* out_key, uint32_t* out_val, uint32_t* n_out, void* scratch,
                     hipStream_t st) {
  scan_generic(InFlag{tiles}, InFlag{tiles}, OutCompact{dkey, out_key, out_val}, nullptr, n_slots,
               n_out, scratch, st);
}

void pair_total(const uint32_t* tiles, int64_t n, uint32_t* total, void* scratch,
                hipStream_t st) {
  const int64_t blocks = (n + kItems - 1) / kItems;
  if (blocks == 0) {
    fill_u32(total, 1, 0u, st);
    return;
  }
  // block sums, then one block adds them up
  uint32_t* sums = static_cast<uint32_t*>(scratch);
  hipLaunchKernelGGL(k_scan_reduce<InPlain>, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                     InPlain{tiles}, nullptr, n, sums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, sums, (int)blocks, total);
}

void row_offsets(const uint32_t* nrows, const uint32_t* vval, const uint32_t* n_vis,
                 int64_t n_cap, uint32_t* roff, uint32_t* total, void* scratch, hipStream_t st) {
  // the reduce pass leaves each entry's row count in `roff`; the apply pass scans it in place
  scan_generic(InGatherKeep{nrows, vval, roff}, InPlain{roff}, OutStore{roff}, n_vis, n_cap,
               total, scratch, st);
}

// The table of the smaller workgroups is the larger one: it serves either.
size_t radix_scratch_bytes(int64_t n_cap) {
  const int64_t blocks = (n_cap + kRadixItems - 1) / kRadixItems;
  const int64_t table = blocks * kRadix;
  return sizeof(uint32_t) * (size_t)(table + 16) + scan_scratch_bytes(table);
}

template <typename K, int NT, typename V>
int radix_sort_nt(K* key[2], V* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
                  void* scratch, hipStream_t st) {
  constexpr int64_t ITEMS = (int64_t)NT * kRadixPerThread;
  const int64_t blocks = (n_cap + ITEMS - 1) / ITEMS;
  if (blocks == 0 || bits <= 0) return 0;
  uint32_t* hist = static_cast<uint32_t*>(scratch);
  void* scan_tmp = hist + blocks * kRadix + 16;
  int cur = 0;
  for (int shift = 0; shift < bits; shift += kRadixBits) {
    const int nb = (bits - shift) < kRadixBits ? (bits - shift) : kRadixBits;
    const uint32_t mask = (1u << nb) - 1u;
    hipLaunchKernelGGL((k_radix_hist<K, NT>), dim3((unsigned)blocks), dim3(NT), 0, st, key[cur],
                       n_dev, shift, mask, hist, (int)blocks);
    scan_generic(InPlain{hist}, InPlain{hist}, OutStore{hist}, nullptr, blocks * kRadix, nullptr,
                 scan_tmp, st);
    hipLaunchKernelGGL((k_radix_scatter<K, NT, V>), dim3((unsigned)blocks), dim3(NT), 0, st,
                       key[cur], val[cur], key[cur ^ 1], val[cur ^ 1], n_dev, shift, mask, hist,
                       (int)blocks);
    cur ^= 1;
  }
  return cur;
}

template <typename K, typename V>
int radix_sort_t(K* key[2], V* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
                 bool wide, void* scratch, hipStream_t st) {
  if (wide) return radix_sort_nt<K, kWideThreads, V>(key, val, n_dev, n_cap, bits, scratch, st);
  return radix_sort_nt<K, kThreads, V>(key, val, n_dev, n_cap, bits, scratch, st);
}

int radix_sort(uint32_t* key[2], uint32_t* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
               bool wide, void* scratch, hipStream_t st) {
  return radix_sort_t<uint32_t>(key, val, n_dev, n_cap, bits, wide, scratch, st);
}

int radix_sort(uint16_t* key[2], uint32_t* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
               bool wide, void* scratch, hipStream_t st) {
  return radix_sort_t<uint16_t>(key, val, n_dev, n_cap, bits, wide, scratch, st);
}

// 8-byte values move through the 256-thread workgroups (their LDS staging doubles).
int radix_sort(uint32_t* key[2], uint2* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
               void* scratch, hipStream_t st) {
  return radix_sort_t<uint32_t>(key, val, n_dev, n_cap, bits, false, scratch, st);
}

int radix_sort(uint16_t* key[2], uint2* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
               void* scratch, hipStream_t st) {
  return radix_sort_t<uint16_t>(key, val, n_dev, n_cap, bits, false, scratch, st);
}

template <typename K>
void rowgen_t(const float* rec, const uint32_t* vval, const uint32_t* roff, const uint32_t* n_vis,
              int64_t n_vis_cap, const uint32_t* n_rows, int64_t row_cap, int n_slots_per_view,
              const DView* views, DSettings S, K* rkey, uint2* rval, uint32_t* flag,
              hipStream_t st) {
  const int64_t waves = (n_vis_cap + 63) / 64;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks == 0) return;
  hipLaunchKernelGGL(k_rowgen<K>, dim3((unsigned)blocks), dim3(kThreads), 0, st, rec, vval, roff,
                     n_vis, n_rows, row_cap, n_slots_per_view, views, S, rkey, rval, flag);
}

void rowgen(const float* rec, const uint32_t* vval, const uint32_t* roff, const uint32_t* n_vis,
            int64_t n_vis_cap, const uint32_t* n_rows, int64_t row_cap, int n_slots_per_view,
            const DView* views, DSettings S, uint32_t* rkey, uint2* rval, uint32_t* flag,
            hipStream_t st) {
  rowgen_t<uint32_t>(rec, vval, roff, n_vis, n_vis_cap, n_rows, row_cap, n_slots_per_view, views,
                     S, rkey, rval, flag, st);
}

void rowgen(const float* rec, const uint32_t* vval, const uint32_t* roff, const uint32_t* n_vis,
            int64_t n_vis_cap, const uint32_t* n_rows, int64_t row_cap, int n_slots_per_view,
            const DView* views, DSettings S, uint16_t* rkey, uint2* rval, uint32_t* flag,
            hipStream_t st) {
  rowgen_t<uint16_t>(rec, vval, roff, n_vis, n_vis_cap, n_rows, row_cap, n_slots_per_view, views,
                     S, rkey, rval, flag, st);
}

void expand(const uint2* rrange, int n_rows, const DView* views, int n_views, int64_t n_tiles,
            const uint2* runs, int64_t chunk_cap,
            int64_t hist_cap, int64_t pair_cap, const uint32_t* n_pairs, uint4* rinfo,
            uint32_t* crow, uint32_t* hist, uint32_t* counts, uint32_t* pval, uint2* ranges,
            uint32_t* flag, void* scratch, hipStream_t st) {
  // counts: [0..7] chunks of each XCD, [8] table entries, [9] pairs written
  if (n_rows <= 0 || n_tiles <= 0) {
    fill_u32(counts, kXcds + 2, 0u, st);
    fill_u32(reinterpret_cast<uint32_t*>(ranges), 2 * n_tiles, 0u, st);
    return;
  }
  hipLaunchKernelGGL(k_row_table, dim3(1), dim3(1024), 0, st, rrange, n_rows, views, n_views,
                     rinfo, (uint32_t)std::min<int64_t>(hist_cap, UINT32_MAX), counts);
  hipLaunchKernelGGL(k_chunk_rows, dim3((unsigned)n_rows), dim3(256), 0, st, rinfo, chunk_cap,
                     crow);
  // per XCD enough workgroups to fill its CUs, each striding over that XCD's chunks
  const int64_t per_xcd = std::min<int64_t>((chunk_cap + 3) / 4, 1024);
  const unsigned blocks = (unsigned)(kXcds * per_xcd);
  hipLaunchKernelGGL(k_expand_count, dim3(blocks), dim3(256), 0, st, rinfo, crow, chunk_cap,
                     counts, runs, hist, hist_cap);
  scan_generic(InPlain{hist}, InPlain{hist}, OutStore{hist}, counts + kXcds, hist_cap,
               counts + kXcds + 1, scratch, st);
  hipLaunchKernelGGL(k_expand_ranges, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, st,
                     rinfo, views, n_views, hist, counts + kXcds, counts + kXcds + 1, n_pairs,
                     n_tiles, (uint32_t)std::min<int64_t>(pair_cap, 1 << 29), ranges, flag);
  // (pairs beyond 2^29, which the 32-bit buffer offsets cannot address, are not written and
  // are reported as a capacity overflow by the ranges pass)
  hipLaunchKernelGGL(k_expand_write, dim3(blocks), dim3(256), 0, st, rinfo, crow, chunk_cap,
                     counts, runs, hist, hist_cap, (uint32_t)std::min<int64_t>(pair_cap, 1 << 29),
                     pval, flag);
}

template <typename K>
void tile_ranges_t(const K* pkey, const uint32_t* n_pairs, int64_t pair_cap, int64_t n_tiles,
                   uint2* ranges, hipStream_t st) {
  fill_u32(reinterpret_cast<uint32_t*>(ranges), 2 * n_tiles, 0u, st);
  const int64_t blocks = (pair_cap + 1023) / 1024;  // four keys per thread
  if (blocks == 0) return;
  hipLaunchKernelGGL(k_ranges<K>, dim3((unsigned)blocks), dim3(256), 0, st, pkey, n_pairs,
                     pair_cap, n_tiles, ranges);
}

void tile_ranges(const uint32_t* pkey, const uint32_t* n_pairs, int64_t pair_cap, int64_t n_tiles,
                 uint2* ranges, hipStream_t st) {
  tile_ranges_t<uint32_t>(pkey, n_pairs, pair_cap, n_tiles, ranges, st);
}

void tile_ranges(const uint16_t* pkey, const uint32_t* n_pairs, int64_t pair_cap, int64_t n_tiles,
                 uint2* ranges, hipStream_t st) {
  tile_ranges_t<uint16_t>(pkey, n_pairs, pair_cap, n_tiles, ranges, st);
}

void tile_ids_of(const uint2* ranges, int64_t n_tiles, int64_t n, uint32_t* ids, hipStream_t st) {
  if (n_tiles <= 0 || n <= 0) return;
  const int64_t blocks = std::min<int64_t>(n_tiles, 1 << 20);
  hipLaunchKernelGGL(k_tile_ids, dim3((unsigned)blocks), dim3(256), 0, st, ranges, n_tiles, n,
                     ids);
}

void clamp_count(const uint32_t* n, uint32_t cap, uint32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_clamp_count, dim3(1), dim3(64), 0, st, n, cap, out);
}

void view_setup(DView* views, int n_views, float jac_margin, hipStream_t st) {
  hipLaunchKernelGGL(k_view_setup, dim3((n_views + 63) / 64), dim3(64), 0, st, views, n_views,
                     jac_margin);
}

}  // namespace g4d
