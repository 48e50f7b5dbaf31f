// Binning kernels: stream compaction of visible (view, Gaussian) slots, device-wide scans,
// key generation, an LDS-staged wavefront LSD radix sort and tile-range detection.
//
// Binning follows the tile-based rasterizer the paper adopts (Sec. 3.2): every splat is
// listed in each screen tile its reach ellipse touches, and each tile's list is ordered by
// camera depth, front to back (Sec. 3.1 composites the splats in depth order).  Here the depth order is made
// once per visible splat (a 32-bit depth sort of the compacted slots); the (tile, splat)
// pairs are then emitted in depth order and stably sorted by tile id alone, so each tile's
// list inherits the depth order (ties keep the slot order, i.e. the Gaussian index).
#include <hip/hip_runtime.h>

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

template <typename K, int NT>
__global__ __launch_bounds__(NT) void k_radix_scatter(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* n_dev, int shift, uint32_t mask,
    const uint32_t* __restrict__ hist, int nblocks) {
  constexpr int NW = NT / 64, ITEMS = NT * kRadixPerThread;
  static_assert(NT >= kRadix, "one thread per digit");
  __shared__ uint32_t wcount[NW][kRadix];
  __shared__ uint32_t bstart[kRadix];
  __shared__ uint32_t goff[kRadix];
  __shared__ K sk[ITEMS];
  __shared__ uint32_t sv[ITEMS];
  __shared__ uint32_t lds4[4];
  const int64_t n = *n_dev;
  const int64_t bbase = (int64_t)blockIdx.x * ITEMS;
  if (bbase >= n) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int d = threadIdx.x; d < NW * kRadix; d += NT) (&wcount[0][0])[d] = 0;
  __syncthreads();
  const int64_t base = bbase + w * (ITEMS / NW);
  const uint64_t lt = lanemask_lt();
  uint32_t k[kRadixPerThread], v[kRadixPerThread], rank[kRadixPerThread];
#pragma unroll
  for (int r = 0; r < kRadixPerThread; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool valid = i < n;
    k[r] = valid ? (uint32_t)kin[i] : 0u;
    v[r] = valid ? vin[i] : 0u;
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
// Key generation: each wave takes 64 consecutive visible splats (in depth order).  Their tile
// rows (rows of each splat's tile box) are numbered consecutively; in rounds of 64 rows, each
// lane finds its row's run of tile columns with tile_row_span (the same function the
// preprocess counted with), a wave scan gives each run its place, and the lane writes its run.
// So a splat that covers thousands of tiles is spread over many lanes, and the pairs come out
// in depth order, each splat's tiles in row-major order.
// ------------------------------------------------------------------------------------------

template <typename K>
__global__ __launch_bounds__(kThreads) void k_keygen(
    const float* __restrict__ rec, const uint32_t* __restrict__ vval,
    const uint32_t* __restrict__ voff, const uint32_t* n_vis_dev, const uint32_t* n_pairs_dev,
    int64_t pair_cap, int n_per_view, int n_tiles, const DView* __restrict__ views, DSettings S,
    K* __restrict__ pkey, uint32_t* __restrict__ pval, uint32_t* overflow) {
  __shared__ uint32_t s_rows[4][65];
  __shared__ float s_u[4][64], s_v[4][64], s_a[4][64], s_b[4][64], s_c[4][64];
  __shared__ float s_ex[4][64], s_ey[4][64];
  __shared__ int32_t s_x0[4][64], s_x1[4][64], s_y0[4][64], s_tx[4][64], s_tb[4][64];
  __shared__ int32_t s_w[4][64], s_h[4][64];
  __shared__ float s_lim[4][64];
  __shared__ uint32_t s_slot[4][64];
  __shared__ uint32_t s_start[4][64], s_key0[4][64], s_val[4][64];  // runs of one round
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t n_vis = *n_vis_dev;
  const int64_t first = ((int64_t)blockIdx.x * 4 + w) * 64;
  if (first >= n_vis) return;
  const int64_t r = first + lane;
  const int64_t last = (n_vis - first < 64 ? n_vis : first + 64) - 1;
  const uint32_t off0 = voff[first];
  const uint32_t off_end = (last + 1 < n_vis) ? voff[last + 1] : *n_pairs_dev;
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
    s_tx[w][lane] = V.tiles_x;
    s_tb[w][lane] = V.tile_base;
    s_w[w][lane] = V.width;
    s_h[w][lane] = V.height;
    s_slot[w][lane] = slot;
  }
  uint32_t n_rows;
  const uint32_t row0 = wave_excl_scan(rows, n_rows);
  s_rows[w][lane] = (r < n_vis) ? row0 : n_rows;
  if (lane == 0) s_rows[w][64] = n_rows;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t cursor = off0;
  for (uint32_t k0 = 0; k0 < n_rows; k0 += 64) {
    const uint32_t k = k0 + lane;
    uint32_t cnt = 0;
    int i = 0, ty = 0, c0 = 0;
    if (k < n_rows) {
      int lo = 0, hi = 63;  // largest i with s_rows[i] <= k
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_rows[w][mid] <= k) lo = mid; else hi = mid - 1;
      }
      i = lo;
      ty = s_y0[w][i] + (int)(k - s_rows[w][i]);
      const int span = tile_row_span(s_u[w][i], s_v[w][i], s_a[w][i], s_b[w][i], s_c[w][i],
                                     s_lim[w][i],
                                     s_ex[w][i], s_ey[w][i], ty, S.tile_shift, s_w[w][i],
                                     s_h[w][i], s_x0[w][i], s_x1[w][i]);
      if (span >= 0) {
        c0 = span >> 16;
        cnt = (uint32_t)((span & 0xFFFF) - c0 + 1);
      }
    }
    uint32_t total;
    const uint32_t start = wave_excl_scan(cnt, total);
    // Publish the runs, then write the round's pairs with consecutive lanes on consecutive
    // addresses: pair e belongs to the last run starting at or before e.
    s_start[w][lane] = start;
    s_key0[w][lane] = (uint32_t)(s_tb[w][i] + ty * s_tx[w][i] + c0);
    s_val[w][lane] = s_slot[w][i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t e = lane; e < total; e += 64) {
      int lo = 0, hi = 63;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[w][mid] <= e) lo = mid; else hi = mid - 1;
      }
      const uint32_t dst = cursor + e;
      if (dst < off_end && (int64_t)dst < pair_cap) {
        pkey[dst] = (K)(s_key0[w][lo] + (e - s_start[w][lo]));
        pval[dst] = s_val[w][lo];
      } else {
        *overflow = 1u;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    cursor += total;
  }
  // The preprocess counted exactly these pairs.  Should the two ever disagree, the shortfall
  // is filled with the dummy tile id n_tiles (listed after every real tile, never drawn) so
  // that no stale key survives, and the disagreement is reported.
  if (cursor != off_end) {
    if (lane == 0) *overflow = 2u;
    for (uint32_t dst = cursor + lane; dst < off_end; dst += 64)
      if ((int64_t)dst < pair_cap) {
        pkey[dst] = (K)n_tiles;
        pval[dst] = 0u;
      }
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

__global__ void k_widen_u16(const uint16_t* __restrict__ in, int64_t n, uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
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

void pair_offsets(const uint32_t* tiles, const uint32_t* val, const uint32_t* n_dev,
                  int64_t n_cap, uint32_t* offsets, uint32_t* total, void* scratch,
                  hipStream_t st) {
  // the reduce pass leaves the gathered counts in `offsets`; the apply pass scans them in place
  scan_generic(InGatherKeep{tiles, val, offsets}, InPlain{offsets}, OutStore{offsets}, n_dev, n_cap,
               total, scratch, st);
}

// The table of the smaller workgroups is the larger one: it serves either.
size_t radix_scratch_bytes(int64_t n_cap) {
  const int64_t blocks = (n_cap + kRadixItems - 1) / kRadixItems;
  const int64_t table = blocks * kRadix;
  return sizeof(uint32_t) * (size_t)(table + 16) + scan_scratch_bytes(table);
}

template <typename K, int NT>
int radix_sort_nt(K* key[2], uint32_t* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
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
    hipLaunchKernelGGL((k_radix_scatter<K, NT>), dim3((unsigned)blocks), dim3(NT), 0, st,
                       key[cur], val[cur], key[cur ^ 1], val[cur ^ 1], n_dev, shift, mask, hist,
                       (int)blocks);
    cur ^= 1;
  }
  return cur;
}

template <typename K>
int radix_sort_t(K* key[2], uint32_t* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
                 bool wide, void* scratch, hipStream_t st) {
  if (wide) return radix_sort_nt<K, kWideThreads>(key, val, n_dev, n_cap, bits, scratch, st);
  return radix_sort_nt<K, kThreads>(key, val, n_dev, n_cap, bits, scratch, st);
}

int radix_sort(uint32_t* key[2], uint32_t* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
               bool wide, void* scratch, hipStream_t st) {
  return radix_sort_t<uint32_t>(key, val, n_dev, n_cap, bits, wide, scratch, st);
}

int radix_sort(uint16_t* key[2], uint32_t* val[2], const uint32_t* n_dev, int64_t n_cap, int bits,
               bool wide, void* scratch, hipStream_t st) {
  return radix_sort_t<uint16_t>(key, val, n_dev, n_cap, bits, wide, scratch, st);
}

template <typename K>
void keygen_t(const float* rec, const uint32_t* vval, const uint32_t* voff, const uint32_t* n_vis,
              int64_t n_vis_cap, const uint32_t* n_pairs, int64_t pair_cap, int n_slots_per_view,
              int n_tiles, const DView* views, DSettings S, K* pkey, uint32_t* pval,
              uint32_t* overflow, hipStream_t st) {
  const int64_t waves = (n_vis_cap + 63) / 64;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks == 0) return;
  hipLaunchKernelGGL(k_keygen<K>, dim3((unsigned)blocks), dim3(kThreads), 0, st, rec, vval, voff,
                     n_vis, n_pairs, pair_cap, n_slots_per_view, n_tiles, views, S, pkey, pval,
                     overflow);
}

void keygen(const float* rec, const uint32_t* vval, const uint32_t* voff, const uint32_t* n_vis,
            int64_t n_vis_cap, const uint32_t* n_pairs, int64_t pair_cap, int n_slots_per_view,
            int n_tiles, const DView* views, DSettings S, uint32_t* pkey, uint32_t* pval,
            uint32_t* overflow, hipStream_t st) {
  keygen_t<uint32_t>(rec, vval, voff, n_vis, n_vis_cap, n_pairs, pair_cap, n_slots_per_view,
                     n_tiles, views, S, pkey, pval, overflow, st);
}

void keygen(const float* rec, const uint32_t* vval, const uint32_t* voff, const uint32_t* n_vis,
            int64_t n_vis_cap, const uint32_t* n_pairs, int64_t pair_cap, int n_slots_per_view,
            int n_tiles, const DView* views, DSettings S, uint16_t* pkey, uint32_t* pval,
            uint32_t* overflow, hipStream_t st) {
  keygen_t<uint16_t>(rec, vval, voff, n_vis, n_vis_cap, n_pairs, pair_cap, n_slots_per_view,
                     n_tiles, views, S, pkey, pval, overflow, st);
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

void widen_u16(const uint16_t* in, int64_t n, uint32_t* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_widen_u16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, n, out);
}

void clamp_count(const uint32_t* n, uint32_t cap, uint32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_clamp_count, dim3(1), dim3(64), 0, st, n, cap, out);
}

void view_setup(DView* views, int n_views, float jac_margin, hipStream_t st) {
  hipLaunchKernelGGL(k_view_setup, dim3((n_views + 63) / 64), dim3(64), 0, st, views, n_views,
                     jac_margin);
}

}  // namespace g4d
