// Binning kernels: device-wide scans, a per-view LDS-staged wavefront LSD radix sort of the
// listed (view, Gaussian) slots by depth, and the row binning.
//
// Binning follows the tile-based rasterizer the paper adopts (Sec. 3.2): every splat is
// listed in each screen tile its reach ellipse touches, and each tile's list is ordered by
// camera depth, front to back (Sec. 3.1 composites the splats in depth order).  Here the
// depth order is made once per visible splat (a 32-bit sort of each view's listed slots);
// each view's splats are then transposed, in depth order, into runs of tile columns per tile
// row, and the runs into the tile lists, each by a count pass, one scan and a write pass, so
// each tile's list inherits the depth order (ties keep the slot order, i.e. the Gaussian index).
#include <hip/hip_runtime.h>
#include <algorithm>

#include "../../include/g4d.h"
#include "g4d_internal.h"

namespace g4d {
namespace {

constexpr int kThreads = kSortThreads;          // 4 waves of 64
constexpr int kItems = kScanItems;              // 16 items per thread
constexpr int kPerThread = kItems / kThreads;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
// Items per workgroup of a radix pass (a multiple of 4 x 64).  The depth sort of the
// 300k-Gaussian, 16-view workload (1.8M slots, 32-bit keys) took 0.149 ms at 4096,
// 0.143 at 2048 and 0.201 at 8192 as one sort over all views.
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

// acc + the set bits of m below this lane (v_mbcnt_lo and v_mbcnt_hi: two instructions).
__device__ __forceinline__ uint32_t rank_below(uint64_t m, uint32_t acc) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, acc));
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
struct InPlain {
  const uint32_t* p;
  __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct OutStore {
  uint32_t* out;
  __device__ void operator()(int64_t i, uint32_t excl, uint32_t) const { out[i] = excl; }
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
// Depth sort within each view.  Slots are view-major (slot = view * N + Gaussian), so each
// view's listed slots lie together, in slot order; a stable LSD radix sort of their depth keys
// inside each view's segment (8 bits per pass) leaves them grouped by view, in depth order,
// slot order among equal keys, with no compaction and no pass over all views.  The first pass
// takes the listed slots straight from the preprocess's arrays (workgroups of kRadixItems slots
// of one view); the later passes take up to kRadixItems listed slots of one view per
// workgroup.  A pass counts digits per workgroup, turns each view's counts into scatter
// offsets with one workgroup per view (starting at the view's place in the sorted list) and
// scatters.  Each wave owns a contiguous 1024-item run of its workgroup; ranks inside a wave
// come from ballot-based digit matching, so equal digits keep their input order.
// ------------------------------------------------------------------------------------------

// The items of a radix workgroup.  The first pass reads the preprocess's arrays themselves:
// workgroup b covers kRadixItems slots of view b / nb1, its items the listed ones (key = the
// depth key, value = the slot), found from the listing masks: vmask[view * n_wc + c] has bit l
// set if slot view * N + 64 c + l is listed.  The later passes take binfo[b] = (first item,
// items, ...).
struct SegItems {
  uint32_t first, end, vbase;  // vbase: the view's first slot (first pass)
  __device__ bool load(bool first_pass, const uint4* __restrict__ binfo, uint32_t nb1,
                       uint32_t n_per_view) {
    if (first_pass) {
      const uint32_t v = blockIdx.x / nb1, j = blockIdx.x - v * nb1;
      vbase = v * n_per_view;
      first = vbase + j * (uint32_t)kRadixItems;
      end = min(first + (uint32_t)kRadixItems, vbase + n_per_view);
    } else {
      const uint4 bi = binfo[blockIdx.x];
      first = bi.x;
      end = bi.x + bi.y;
      vbase = 0;
    }
    return end > first;
  }
  // First pass: the listing mask of the 64 slots from slot0 (a multiple of 64 past vbase);
  // 0 past the workgroup's end.
  __device__ uint64_t mask(const uint64_t* __restrict__ vmask, uint64_t row,
                           uint32_t slot0) const {
    return slot0 < end ? vmask[row + ((slot0 - vbase) >> 6)] : 0ull;
  }
};

// Digit counts of one workgroup's items: table[256 b + d] for workgroup b and digit d.
// In the first pass also bcount[b] = the workgroup's listed slots.
template <bool FIRST>
__global__ __launch_bounds__(kThreads) void k_seg_hist(const uint32_t* __restrict__ key,
                                                       const uint64_t* __restrict__ vmask,
                                                       int64_t n_wc,
                                                       const uint4* __restrict__ binfo,
                                                       uint32_t nb1, uint32_t n_per_view,
                                                       int shift, uint32_t* __restrict__ table,
                                                       uint32_t* __restrict__ bcount) {
  constexpr int NW = kThreads / 64;
  static_assert(kThreads == kRadix, "one thread per digit");
  __shared__ uint32_t wh[NW][kRadix];
  __shared__ uint32_t s_tot[NW];
  SegItems it;
  if (!it.load(FIRST, binfo, nb1, n_per_view)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int d = threadIdx.x; d < NW * kRadix; d += kThreads) (&wh[0][0])[d] = 0;
  __syncthreads();
  const uint32_t end = it.end;
  const uint32_t base = it.first + (uint32_t)w * (kRadixItems / NW);
  const uint64_t row = FIRST ? (uint64_t)(blockIdx.x / nb1) * (uint64_t)n_wc : 0;
#pragma unroll 4
  for (int r = 0; r < kRadixPerThread; ++r) {
    const uint32_t i = base + (uint32_t)(r * 64 + lane);
    const bool valid = FIRST ? ((it.mask(vmask, row, base + (uint32_t)(r * 64)) >> lane) & 1ull)
                             : i < end;
    if (valid) atomicAdd(&wh[w][(key[i] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  const int d = threadIdx.x;
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) t += wh[k][d];
  table[(uint32_t)kRadix * blockIdx.x + (uint32_t)d] = t;
  if constexpr (FIRST) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) s_tot[w] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t n = 0;
#pragma unroll
      for (int k = 0; k < NW; ++k) n += s_tot[k];
      bcount[blockIdx.x] = n;
    }
  }
}

// A view's digit counts (its nb workgroups from fb, table[256 b + d]) become scatter offsets:
// each digit's total over the workgroups, an exclusive scan over the digits from `start` (the
// view's first place in the sorted list), and per workgroup the counts of the digit in the
// view's earlier ones.  A workgroup of four threads per digit, each over a quarter of the
// workgroups with eight loads in flight; every thread of the workgroup calls it.
constexpr int kScanThreads = 4 * kRadix;
__device__ void view_digit_scan(uint32_t* __restrict__ table, uint32_t fb, uint32_t nb,
                                uint32_t start) {
  __shared__ uint32_t s_part[4][kRadix], s_base[kRadix], lds4[4];
  const int d = threadIdx.x & (kRadix - 1), q = threadIdx.x / kRadix;
  const uint32_t per = (nb + 3u) / 4u;
  const uint32_t j0 = min((uint32_t)q * per, nb), j1 = min(j0 + per, nb);
  uint32_t* col = table + (uint32_t)kRadix * fb + (uint32_t)d;
  uint32_t part = 0;
  for (uint32_t j = j0; j < j1; j += 8) {
    uint32_t c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = (j + u < j1) ? col[(uint32_t)kRadix * (j + u)] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u) part += c[u];
  }
  s_part[q][d] = part;
  __syncthreads();
  uint32_t tot = 0, inc = 0;
  if (q == 0) {  // waves 0-3: the exclusive scan of the digit totals
    tot = s_part[0][d] + s_part[1][d] + s_part[2][d] + s_part[3][d];
    inc = wave_incl_scan(tot);
    if ((d & 63) == 63) lds4[d >> 6] = inc;
  }
  __syncthreads();
  if (q == 0) {
    uint32_t pre = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) pre += (k < (d >> 6)) ? lds4[k] : 0u;
    s_base[d] = start + pre + inc - tot;
  }
  __syncthreads();
  uint32_t run = s_base[d];
  for (int k = 0; k < q; ++k) run += s_part[k][d];
  for (uint32_t j = j0; j < j1; j += 8) {
    uint32_t c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = (j + u < j1) ? col[(uint32_t)kRadix * (j + u)] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j + u < j1) {
        col[(uint32_t)kRadix * (j + u)] = run;
        run += c[u];
      }
  }
}

// Later passes: one workgroup per view, its workgroups from vfirst / binfo.
__global__ __launch_bounds__(kScanThreads) void k_seg_scan(const uint2* __restrict__ vrange,
                                                           const uint4* __restrict__ binfo,
                                                           const uint32_t* __restrict__ vfirst,
                                                           uint32_t* __restrict__ table) {
  const uint32_t v = blockIdx.x;
  const uint2 r = vrange[v];
  if (r.y == r.x) return;
  const uint32_t fb = vfirst[v];
  view_digit_scan(table, fb, binfo[fb].w, r.x);
}

// First pass, one workgroup per view v: the listed slots of the views up to v from the first
// histogram's per-workgroup counts (bcount, nb1 workgroups per view) give the view's place
// [lo, lo + len) in the sorted list (lo = the listed slots of the views before it, written to
// vrange[v]) and its workgroups of the later passes (vfirst[v]; binfo[b] = (first item, items,
// the view's first workgroup, the view's workgroups)).  The last view also writes *n_vis and
// clears binfo past the last workgroup (items = 0, up to bcap); the first adds up the
// preprocess's per-wave pair and run counts (see depth_sort_by_view).  Then the view's
// first-pass counts become scatter offsets.
__global__ __launch_bounds__(kScanThreads) void k_first_scan(
    const uint32_t* __restrict__ bcount, uint32_t nb1, int n_views, uint32_t* n_vis,
    uint2* __restrict__ vrange, uint32_t* __restrict__ vfirst, uint4* __restrict__ binfo,
    int64_t bcap, const uint2* __restrict__ wsum, int64_t n_wsum, uint32_t* totals,
    uint32_t* __restrict__ table) {
  __shared__ uint32_t s_len[G4D_MAX_VIEWS], s_a[16], s_b[16];
  __shared__ uint64_t s_p[16], s_r[16];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t v = blockIdx.x;
  for (int u = w; u <= (int)v; u += 16) {  // a wave per view
    const uint32_t* c = bcount + (size_t)u * nb1;
    uint32_t t = 0;
    for (uint32_t j = (uint32_t)lane; j < nb1; j += 64) t += c[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) s_len[u] = t;
  }
  const bool sums = v == 0 && wsum;
  if (sums) {
    uint64_t p = 0, r = 0;
    for (int64_t i = threadIdx.x; i < n_wsum; i += kScanThreads) {
      const uint2 c = wsum[i];
      p += c.x;
      r += c.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      p += ((uint64_t)__shfl_xor((uint32_t)(p >> 32), o, 64) << 32) | __shfl_xor((uint32_t)p, o, 64);
      r += ((uint64_t)__shfl_xor((uint32_t)(r >> 32), o, 64) << 32) | __shfl_xor((uint32_t)r, o, 64);
    }
    if (lane == 0) {
      s_p[w] = p;
      s_r[w] = r;
    }
  }
  __syncthreads();
  // lo and the first workgroup: sums over the views before v (a thread per view)
  uint32_t a = 0, b = 0;
  if (threadIdx.x < v) {
    a = s_len[threadIdx.x];
    b = (a + (uint32_t)kRadixItems - 1u) / (uint32_t)kRadixItems;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  if (lane == 0) {
    s_a[w] = a;
    s_b[w] = b;
  }
  __syncthreads();
  uint32_t lo = 0, fb = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    lo += s_a[k];
    fb += s_b[k];
  }
  const uint32_t len = s_len[v];
  const uint32_t nb = (len + (uint32_t)kRadixItems - 1u) / (uint32_t)kRadixItems;
  if (threadIdx.x == 0) {
    vrange[v] = make_uint2(lo, lo + len);
    vfirst[v] = fb;
  }
  for (uint32_t j = threadIdx.x; j < nb; j += kScanThreads) {
    const uint32_t first = j * (uint32_t)kRadixItems;
    if ((int64_t)(fb + j) < bcap)
      binfo[fb + j] = make_uint4(lo + first, min((uint32_t)kRadixItems, len - first), fb, nb);
  }
  if (v == (uint32_t)n_views - 1u) {
    if (threadIdx.x == 0) *n_vis = lo + len;
    for (int64_t k = (int64_t)(fb + nb) + threadIdx.x; k < bcap; k += kScanThreads)
      binfo[k] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (sums && threadIdx.x == 0) {
    uint64_t p = 0, r = 0;
    for (int k = 0; k < 16; ++k) {
      p += s_p[k];
      r += s_r[k];
    }
    totals[0] = (uint32_t)min(p, (uint64_t)UINT32_MAX);
    totals[2] = (uint32_t)min(r, (uint64_t)UINT32_MAX);
    totals[4] = (p >= 0x80000000ull || r >= 0x80000000ull) ? 1u : 0u;
  }
  if (len == 0) return;
  view_digit_scan(table, v * nb1, nb1, lo);
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

template <bool FIRST>
__global__ __launch_bounds__(kThreads) void k_seg_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    const uint64_t* __restrict__ vmask, int64_t n_wc, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint4* __restrict__ binfo, uint32_t nb1,
    uint32_t n_per_view, int shift, const uint32_t* __restrict__ table) {
  constexpr int NW = kThreads / 64;
  static_assert(kThreads >= kRadix, "one thread per digit");
  __shared__ uint32_t wcount[NW][kRadix];
  __shared__ uint32_t bstart[kRadix];
  __shared__ uint32_t goff[kRadix];
  __shared__ uint32_t sk[kRadixItems];
  __shared__ uint32_t sv[kRadixItems];
  __shared__ uint32_t lds4[4];
  SegItems it;
  if (!it.load(FIRST, binfo, nb1, n_per_view)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int d = threadIdx.x; d < NW * kRadix; d += kThreads) (&wcount[0][0])[d] = 0;
  __syncthreads();
  const uint32_t end = it.end;
  const uint32_t base = it.first + (uint32_t)w * (kRadixItems / NW);
  const uint64_t lt = lanemask_lt();
  // The wave's items as dense rounds of 64: in the first pass its listed slots, packed in
  // slot order into its quarter of sk (which the ranking frees before the LDS sort uses it).
  uint32_t n_w;  // the wave's items (uniform)
  uint32_t* stage = sk + w * (kRadixItems / NW);
  if constexpr (FIRST) {
    const uint64_t row = (uint64_t)(blockIdx.x / nb1) * (uint64_t)n_wc;
    n_w = 0;
#pragma unroll 4
    for (int r = 0; r < kRadixPerThread; ++r) {
      const uint32_t slot0 = base + (uint32_t)(r * 64);
      const uint64_t m = it.mask(vmask, row, slot0);
      if ((m >> lane) & 1ull) stage[rank_below(m, n_w)] = slot0 + (uint32_t)lane;
      n_w += (uint32_t)__popcll(m);
    }
    wave_lds_sync();
  } else {
    n_w = end > base ? min(end - base, (uint32_t)(kRadixItems / NW)) : 0u;
  }
  uint32_t k[kRadixPerThread], v[kRadixPerThread], rank[kRadixPerThread];
#pragma unroll
  for (int r = 0; r < kRadixPerThread; ++r) {
    if ((uint32_t)(r * 64) >= n_w) break;  // uniform: the wave's items are done
    const uint32_t e = (uint32_t)(r * 64 + lane);
    const bool valid = e < n_w;
    const uint32_t i = FIRST ? (valid ? stage[e] : 0u) : base + e;
    k[r] = valid ? kin[i] : 0u;
    v[r] = valid ? (FIRST ? i : vin[i]) : 0u;
    const uint32_t d = (k[r] >> shift) & (kRadix - 1);
    const uint64_t peers = match_digit(d, __ballot(valid));
    const uint32_t before = wcount[w][d];
    rank[r] = rank_below(peers, before);
    __builtin_amdgcn_wave_barrier();
    if (valid && (peers & lt) == 0ull) wcount[w][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // Per-digit totals, exclusive prefix over waves (in place) and over digits (bstart): a
  // thread per digit.
  uint32_t tot = 0;
  {
    const int d = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const uint32_t c = wcount[q][d];
      wcount[q][d] = tot;
      tot += c;
    }
    goff[d] = table[(uint32_t)kRadix * blockIdx.x + (uint32_t)d];
  }
  const uint32_t inc = wave_incl_scan(tot);
  if (lane == 63) lds4[w] = inc;
  __syncthreads();
  {
    uint32_t pre = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) pre += (q < w) ? lds4[q] : 0u;
    bstart[threadIdx.x] = pre + inc - tot;
  }
  const uint32_t cnt = lds4[0] + lds4[1] + lds4[2] + lds4[3];  // the workgroup's items
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRadixPerThread; ++r) {
    if ((uint32_t)(r * 64 + lane) < n_w) {
      const uint32_t d = (k[r] >> shift) & (kRadix - 1);
      const uint32_t pos = bstart[d] + wcount[w][d] + rank[r];
      sk[pos] = k[r];
      sv[pos] = v[r];
    }
  }
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < cnt; p += kThreads) {
    const uint32_t kk = sk[p];
    const uint32_t d = (kk >> shift) & (kRadix - 1);
    const uint32_t dst = goff[d] + (p - bstart[d]);
    kout[dst] = kk;
    vout[dst] = sv[p];
  }
}

// ------------------------------------------------------------------------------------------
// Row binning.  The tiles a splat is listed in are, in each tile row of its box, one run of
// columns (tile_row_span).  Instead of one (tile, splat) pair per tile, sorted by tile, the
// depth-ordered splats of each view are transposed into per-tile-row lists of runs (splats ->
// rows) and each row's runs into the tile lists (rows -> tiles).  Each transpose is a count pass
// over chunks of 64 items (one wave each), one exclusive scan of the (row or column, chunk)
// count table, and a write pass; since every list takes its chunks in order and each chunk's
// items in order, a tile's list holds its splats in depth order, exactly as a stable sort of
// the individual pairs by tile would leave them, without sorting anything.
// ------------------------------------------------------------------------------------------

// ------------------------------------------------------------------------------------------
// Splats to tile rows.  After the depth sort each view's splats lie together in depth order.
// Each view's list is taken 64 splats at a time (a chunk, one wave): a count pass tallies how
// many of the chunk's splats have each tile row of the view in their box (an LDS difference
// array), an exclusive scan over (row, chunk) in row order gives every chunk its place in each
// row's run list, and a write pass deals the chunk's (splat, row) runs out over the lanes,
// finds each run's columns (tile_row_span) and lays it down as (slot, span), span = (first
// column << 16) | last, or ~0u for a row the ellipse misses.  Each row's runs so come in
// depth order.
// ------------------------------------------------------------------------------------------

// Minimum and maximum over the 64 lanes of a wave (all lanes active), wave-uniform.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  x = wave_scan_op(x, ~0u, [](uint32_t a, uint32_t b) { return min(a, b); });
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  x = wave_scan_op(x, 0u, [](uint32_t a, uint32_t b) { return max(a, b); });
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Per view v (one workgroup of 1024 threads, a thread per view): its splats [lo, lo + len) in
// the depth-sorted list, its chunks of 64 splats, the index of its first chunk, and the base of
// its (row, chunk) count table: vinfo[2v] = (lo, len, first chunk, table base),
// vinfo[2v + 1] = (chunks, tiles_y, row_base, 0); totals = (chunks, table entries); then
// cview[chunk] = its view for every chunk below chunk_cap (a wave per view).
__global__ __launch_bounds__(1024) void k_view_table(const uint2* __restrict__ vrange, int n_views,
                                                     const DView* __restrict__ views,
                                                     uint4* __restrict__ vinfo, uint32_t rhist_cap,
                                                     uint32_t* totals, int64_t chunk_cap,
                                                     uint16_t* __restrict__ cview) {
  __shared__ uint32_t s_c[16], s_h[16], s_first[G4D_MAX_VIEWS], s_nch[G4D_MAX_VIEWS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int v = threadIdx.x;
  uint32_t lo = 0, len = 0, nch = 0, ny = 0, rb = 0;
  if (v < n_views) {
    const uint2 g = vrange[v];
    lo = g.x;
    len = g.y - g.x;
    nch = (len + 63u) >> 6;
    ny = (uint32_t)views[v].tiles_y;
    rb = (uint32_t)views[v].row_base;
  }
  const uint32_t hs = nch * ny;
  const uint32_t ic = wave_incl_scan(nch), ih = wave_incl_scan(hs);
  if (lane == 63) {
    s_c[w] = ic;
    s_h[w] = ih;
  }
  __syncthreads();
  uint32_t pc = 0, ph = 0, tc = 0, th = 0;
  for (int k = 0; k < 16; ++k) {
    pc += (k < w) ? s_c[k] : 0u;
    ph += (k < w) ? s_h[k] : 0u;
    tc += s_c[k];
    th += s_h[k];
  }
  if (v < n_views) {
    vinfo[2 * v] = make_uint4(lo, len, pc + ic - nch, ph + ih - hs);
    vinfo[2 * v + 1] = make_uint4(nch, ny, rb, 0u);
    s_first[v] = pc + ic - nch;
    s_nch[v] = nch;
  }
  if (threadIdx.x == 0) {
    totals[0] = tc;
    // (the table capacity covers every view's chunks; the clamp only keeps a broken count
    // from taking the scan past it)
    totals[1] = min(th, rhist_cap);
  }
  __syncthreads();
  for (int u = w; u < n_views; u += 16) {
    const uint32_t first = s_first[u], n = s_nch[u];
    for (uint32_t k = (uint32_t)lane; k < n && (int64_t)(first + k) < chunk_cap; k += 64)
      cview[first + k] = (uint16_t)u;
  }
}

// A chunk of a view's splats: the view's table entries, the chunk within the view, and per
// lane its splat's box rows [y0, y0 + h] (an empty lane: y0 = ~0u, h = 0).
struct SplatChunk {
  uint4 a, b;  // vinfo of the view
  uint32_t c, y0, h;
};

// Chunk g: its view (scalar) and its splats' box rows.
__device__ __forceinline__ bool load_splat_chunk(const uint4* __restrict__ vinfo,
                                                 const uint16_t* __restrict__ cview,
                                                 const uint32_t* n_chunks_dev,
                                                 const uint32_t* __restrict__ vval,
                                                 const uint32_t* __restrict__ rowbox,
                                                 SplatChunk& ck) {
  const int lane = threadIdx.x & 63;
  const uint32_t g = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6));
  if (g >= *n_chunks_dev) return false;
  const uint32_t v = __builtin_amdgcn_readfirstlane((uint32_t)cview[g]);
  ck.a = vinfo[2 * v];
  ck.b = vinfo[2 * v + 1];
  ck.c = g - ck.a.z;
  const uint32_t e = ck.c * 64u + (uint32_t)lane;
  ck.y0 = ~0u;
  ck.h = 0u;
  if (e < ck.a.y) {
    const uint32_t rb = rowbox[vval[ck.a.x + e]];
    if (rb != ~0u) {
      ck.y0 = rb >> 16;
      ck.h = (rb & 0xFFFFu) - ck.y0;
    }
  }
  return true;
}

// Count pass: rhist[table base + row * chunks + chunk] = splats of the chunk whose box holds
// the row (row-major, so that one scan over the whole table yields run positions in row
// order), from a +1 / -1 difference array over 256 rows per window.
constexpr int kCountRows = 256;
__global__ __launch_bounds__(256) void k_rows_count(const uint4* __restrict__ vinfo,
                                                    const uint16_t* __restrict__ cview,
                                                    const uint32_t* n_chunks_dev,
                                                    const uint32_t* __restrict__ vval,
                                                    const uint32_t* __restrict__ rowbox,
                                                    uint32_t* __restrict__ rhist,
                                                    int64_t rhist_cap) {
  __shared__ int4 s_diff[4][kCountRows / 4 + 1];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int* diff = reinterpret_cast<int*>(&s_diff[w][0]);
  SplatChunk ck;
  if (!load_splat_chunk(vinfo, cview, n_chunks_dev, vval, rowbox, ck)) return;
  const uint32_t nch = ck.b.x, ny = ck.b.y;
  for (uint32_t r0 = 0; r0 < ny; r0 += kCountRows) {
    s_diff[w][lane] = make_int4(0, 0, 0, 0);
    if (lane == 0) s_diff[w][kCountRows / 4] = make_int4(0, 0, 0, 0);
    wave_lds_sync();
    if (ck.y0 != ~0u) {
      const int lo = max((int)ck.y0 - (int)r0, 0);
      const int hi = min((int)(ck.y0 + ck.h) - (int)r0, kCountRows - 1);
      if (lo <= hi) {
        atomicAdd(&diff[lo], 1);
        atomicSub(&diff[hi + 1], 1);
      }
    }
    wave_lds_sync();
    const int4 d = s_diff[w][lane];
    const int p0 = d.x, p1 = p0 + d.y, p2 = p1 + d.z, p3 = p2 + d.w;
    const int base = (int)wave_incl_scan((uint32_t)p3) - p3;
    const int val[4] = {base + p0, base + p1, base + p2, base + p3};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t row = r0 + 4u * (uint32_t)lane + (uint32_t)k;
      const int64_t at = (int64_t)ck.a.w + (int64_t)row * nch + ck.c;
      if (row < ny && at < rhist_cap) rhist[at] = (uint32_t)val[k];
    }
    wave_lds_sync();  // the next window clears the array
  }
}

// Runs of global tile row r (in view a) from the scanned (row, chunk) table: [start of (row,
// chunk 0), start of the next row), clamped to the run capacity; an empty row gets (0, 0).
__device__ __forceinline__ uint2 row_range(const RowRuns& rr, const DView* __restrict__ views,
                                           int a, int r) {
  const uint4 va = rr.vinfo[2 * a], vb = rr.vinfo[2 * a + 1];
  const uint32_t ty = (uint32_t)(r - views[a].row_base), nch = vb.x;
  uint32_t lo = 0, hi = 0;
  if (nch > 0) {
    const uint32_t n_hist = *rr.n_hist, total = *rr.total;
    const uint32_t i0 = va.w + ty * nch, i1 = i0 + nch;
    lo = i0 < n_hist ? rr.scanned[i0] : total;
    hi = i1 < n_hist ? rr.scanned[i1] : total;
    lo = min(lo, rr.row_cap);
    hi = min(hi, rr.row_cap);
  }
  return hi > lo ? make_uint2(lo, hi) : make_uint2(0u, 0u);
}

// Position of the r-th set bit of m (r < popcount(m)).
__device__ __forceinline__ int nth_set_bit(uint64_t m, uint32_t r) {
  uint32_t x = (uint32_t)m;
  int base = 0;
  uint32_t c = (uint32_t)__popc(x);
  if (r >= c) {
    r -= c;
    x = (uint32_t)(m >> 32);
    base = 32;
  }
#pragma unroll
  for (int w = 16; w >= 1; w >>= 1) {
    c = (uint32_t)__popc(x & ((1u << w) - 1u));
    if (r >= c) {
      r -= c;
      x >>= w;
      base += w;
    }
  }
  return base;
}

// Write pass.  Per window of 64 rows, lane t holds the mask of the chunk's splats whose box
// holds row t0 + t and that row's scanned place.  The chunk's runs in the window are numbered
// row by row (a wave scan of the rows' counts) and dealt out 64 per round: the lane with run k
// finds its row and its rank r in the row, the splat as the r-th set bit of the row's mask,
// computes the run's columns and stores it at the row's place + r, so that consecutive lanes
// mostly fill consecutive entries of one row's list.
__global__ __launch_bounds__(256) void k_rows_write(const uint4* __restrict__ vinfo,
                                                    const uint16_t* __restrict__ cview,
                                                    const uint32_t* n_chunks_dev,
                                                    const uint32_t* __restrict__ vval,
                                                    const float* __restrict__ rec,
                                                    const DView* __restrict__ views, DSettings S,
                                                    const uint32_t* __restrict__ scanned,
                                                    int64_t rhist_cap, int64_t row_cap,
                                                    uint2* __restrict__ runs, uint32_t* flag) {
  __shared__ float s_u[4][64], s_v[4][64], s_a[4][64], s_b[4][64], s_c[4][64];
  __shared__ float s_ex[4][64], s_ey[4][64], s_lim[4][64];
  __shared__ int32_t s_x0[4][64], s_x1[4][64];
  __shared__ uint32_t s_slot[4][64];
  __shared__ uint64_t s_mask[4][64];
  __shared__ uint32_t s_place[4][64], s_rfirst[4][64], s_mark[4][64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t g = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6));
  if (g >= *n_chunks_dev) return;
  s_mark[w][lane] = 0u;  // no round's stamp (window_owner)
  uint32_t stamp = 1u;
  const uint32_t v = __builtin_amdgcn_readfirstlane((uint32_t)cview[g]);
  const uint4 va = vinfo[2 * v], vb = vinfo[2 * v + 1];
  const uint32_t c = g - va.z, nch = vb.x, ny = vb.y;
  const DView& V = views[v];
  const uint32_t e = c * 64u + (uint32_t)lane;
  uint32_t y0 = ~0u, h = 0u, y1 = 0u, slot = 0u;
  int x0 = 0, x1 = -1;
  if (e < va.y) {
    slot = vval[va.x + e];
    const float* p = rec + (size_t)slot * kRec;
    const float u = p[R_U], pv = p[R_V], ex = p[R_EX], ey = p[R_EY];
    int ty0, ty1;
    // the box the preprocess listed the splat with (the same function on the same values)
    if (tile_rect(u, pv, ex, ey, V, S.tile_shift, x0, x1, ty0, ty1)) {
      y0 = (uint32_t)ty0;
      y1 = (uint32_t)ty1;
      h = y1 - y0;
    }
    s_u[w][lane] = u;
    s_v[w][lane] = pv;
    s_a[w][lane] = p[R_A];
    s_b[w][lane] = p[R_B];
    s_c[w][lane] = p[R_C];
    s_ex[w][lane] = ex;
    s_ey[w][lane] = ey;
    s_lim[w][lane] = coverage_limit(p[R_OPT], S);
  }
  s_x0[w][lane] = x0;
  s_x1[w][lane] = x1;
  s_slot[w][lane] = slot;
  const uint32_t ymin = __builtin_amdgcn_readfirstlane(wave_min_u32(y0));
  const uint32_t ymax = __builtin_amdgcn_readfirstlane(wave_max_u32(y1));
  const uint32_t last = min(ymax, ny - 1u);
  for (uint32_t t0 = ymin & ~63u; ymin <= last && t0 <= last; t0 += 64) {
    // masks, counts and places of the window's rows (lane t: row t0 + t)
    const uint32_t row = t0 + (uint32_t)lane;
    const int64_t at = (int64_t)va.w + (int64_t)row * nch + c;
    if (__ballot(row < ny && at >= rhist_cap)) {  // never with a table sized for the views
      if (lane == 0) *flag = 1u;
      return;
    }
    const uint32_t place = (row < ny) ? scanned[at] : 0u;
    uint64_t mine = 0ull;
    const uint32_t j0 = ymin > t0 ? ymin : t0, j1 = min(last + 1u, t0 + 64u);
    for (uint32_t y = j0; y < j1; ++y) {
      const uint64_t m = __ballot(y - y0 <= h);
      if ((uint32_t)lane == y - t0) mine = m;
    }
    uint32_t total;
    const uint32_t n_row = (uint32_t)__popcll(mine);
    const uint32_t rfirst = wave_excl_scan(n_row, total);
    s_mask[w][lane] = mine;
    s_rfirst[w][lane] = rfirst;
    s_place[w][lane] = place;
    wave_lds_sync();
    int carry = -1;
    for (uint32_t k0 = 0; k0 < total; k0 += 64) {
      const uint32_t k = k0 + (uint32_t)lane;
      // the last row whose runs start at or before k holds run k
      const int a = window_owner(rfirst, n_row, k0, &s_mark[w][0], stamp, carry);
      if (k < total) {
        const uint32_t r = k - s_rfirst[w][a];
        const int j = nth_set_bit(s_mask[w][a], r);
        const int y = (int)t0 + a;
        const int span = tile_row_span(s_u[w][j], s_v[w][j], s_a[w][j], s_b[w][j], s_c[w][j],
                                       s_lim[w][j], s_ex[w][j], s_ey[w][j], y, S.tile_shift,
                                       V.width, V.height, s_x0[w][j], s_x1[w][j]);
        const uint32_t pos = s_place[w][a] + r;
        if ((int64_t)pos < row_cap)
          runs[pos] = make_uint2(s_slot[w][j], span >= 0 ? (uint32_t)span : ~0u);
        else
          *flag = 1u;
      }
    }
    wave_lds_sync();  // the next window rewrites the arrays
  }
}

// The chunks of tile row r are expanded on XCD r % 8 (workgroup b runs on XCD b % 8): a row's
// pairs then fill whole cache lines in one L2 before they are written back, instead of
// reaching memory as partial lines from several XCDs.
constexpr int kXcds = 8;

// Per tile row r (one workgroup walks all rows): its runs [lo, lo + len) in the sorted run
// list (row_range), its chunks of 64 runs and the index of its first chunk among the chunks of
// its XCD, and the base of its (column, chunk) count table: rinfo[2r] = (lo, len, first
// chunk, table base), rinfo[2r + 1] = (chunks, tiles_x, first tile id, 0).  totals = (chunks
// of XCD 0..7, table entries).  The preprocess counted the runs the splats -> rows pass lays
// down: more than the run arrays hold sets *flag = 1 (a capacity overflow), any other
// disagreement *flag = 2 (unless set).
__global__ __launch_bounds__(1024) void k_row_table(RowRuns rr, int n_rows,
                                                    const DView* __restrict__ views, int n_views,
                                                    uint4* __restrict__ rinfo, uint32_t hist_cap,
                                                    uint32_t* totals, uint32_t* flag) {
  __shared__ uint32_t s_c[16][kXcds], s_h[16];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int x = threadIdx.x % kXcds;  // every 1024-row group starts at a multiple of 8
  if (threadIdx.x == 0) {
    const uint32_t total = *rr.total;
    if (total > rr.row_cap) *flag = 1u;
    else if (total != *rr.n_runs && *flag == 0u) *flag = 2u;
  }
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
      const uint2 g = row_range(rr, views, a, r);
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
        const uint32_t pos = rank_below(m, base);
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

__global__ void k_copy_masked_u32(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                  int64_t n, uint32_t mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] & mask;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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

void copy_masked_u32(uint32_t* dst, const uint32_t* src, int64_t n, uint32_t mask,
                     hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy_masked_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst,
                     src, n, mask);
}

size_t scan_scratch_bytes(int64_t n) {
  return sizeof(uint32_t) * (size_t)((n + kItems - 1) / kItems + 1);
}

size_t depth_sort_scratch_bytes(int64_t n_cap, int n_views) {
  const int64_t bcap = (n_cap + kRadixItems - 1) / kRadixItems + n_views;
  return sizeof(uint32_t) * (size_t)(bcap * kRadix) + sizeof(uint4) * (size_t)bcap +
         sizeof(uint32_t) * (size_t)(G4D_MAX_VIEWS + bcap);
}

int depth_sort_by_view(const uint32_t* dkey, const uint64_t* vmask, int64_t n_wc, uint32_t* key[2], uint32_t* val[2], uint32_t* n_vis,
                       int64_t n_cap, int n_views, uint32_t n_per_view, uint2* vrange,
                       const uint2* wsum, int64_t n_wsum, uint32_t* totals, void* scratch,
                       hipStream_t st) {
  if (n_views <= 0 || n_per_view == 0) return 0;
  // every view's workgroups: at most n / kRadixItems + 1 per view
  const int64_t bcap = (n_cap + kRadixItems - 1) / kRadixItems + n_views;
  uint32_t* table = static_cast<uint32_t*>(scratch);
  uint4* binfo = reinterpret_cast<uint4*>(table + bcap * kRadix);
  uint32_t* vfirst = reinterpret_cast<uint32_t*>(binfo + bcap);
  uint32_t* bcount = vfirst + G4D_MAX_VIEWS;
  // first pass: the listed slots of each view, straight from the preprocess's arrays; its scan
  // also places the views and lays out the later passes' workgroups
  const uint32_t nb1 = (n_per_view + (uint32_t)kRadixItems - 1u) / (uint32_t)kRadixItems;
  const unsigned grid1 = (unsigned)n_views * nb1;  // at most bcap
  hipLaunchKernelGGL(k_seg_hist<true>, dim3(grid1), dim3(kThreads), 0, st, dkey, vmask, n_wc,
                     binfo, nb1, n_per_view, 0, table, bcount);
  hipLaunchKernelGGL(k_first_scan, dim3((unsigned)n_views), dim3(kScanThreads), 0, st, bcount,
                     nb1, n_views, n_vis, vrange, vfirst, binfo, bcap, wsum, n_wsum, totals,
                     table);
  hipLaunchKernelGGL(k_seg_scatter<true>, dim3(grid1), dim3(kThreads), 0, st, dkey, nullptr,
                     vmask, n_wc, key[1], val[1], binfo, nb1, n_per_view, 0, table);
  int cur = 1;
  for (int shift = kRadixBits; shift < 32; shift += kRadixBits) {
    hipLaunchKernelGGL(k_seg_hist<false>, dim3((unsigned)bcap), dim3(kThreads), 0, st, key[cur],
                       nullptr, (int64_t)0, binfo, 0u, n_per_view, shift, table, nullptr);
    hipLaunchKernelGGL(k_seg_scan, dim3((unsigned)n_views), dim3(kScanThreads), 0, st, vrange,
                       binfo, vfirst, table);
    hipLaunchKernelGGL(k_seg_scatter<false>, dim3((unsigned)bcap), dim3(kThreads), 0, st,
                       key[cur], val[cur], nullptr, (int64_t)0, key[cur ^ 1], val[cur ^ 1], binfo,
                       0u, n_per_view, shift, table);
    cur ^= 1;
  }
  return cur;
}

void splats_to_rows(const uint2* vrange, int n_views, const DView* views,
                    int64_t max_tiles_y, const uint32_t* vval, const uint32_t* rowbox,
                    const float* rec, DSettings S, int64_t chunk_cap, int64_t rhist_cap,
                    int64_t row_cap, uint4* vinfo, uint16_t* cview, uint32_t* rhist,
                    uint32_t* counts, uint2* runs, uint32_t* flag, void* scratch,
                    hipStream_t st) {
  // counts: [0] chunks, [1] table entries, [2] runs laid down
  hipLaunchKernelGGL(k_view_table, dim3(1), dim3(1024), 0, st, vrange, n_views, views, vinfo,
                     (uint32_t)std::min<int64_t>(rhist_cap, UINT32_MAX), counts, chunk_cap, cview);
  const int64_t blocks = (chunk_cap + 3) / 4;
  if (blocks > 0)
    hipLaunchKernelGGL(k_rows_count, dim3((unsigned)blocks), dim3(256), 0, st, vinfo, cview,
                       counts + 0, vval, rowbox, rhist, rhist_cap);
  // the table holds at most (largest tiles_y) x chunks entries: the scan's grid covers that
  // bound rather than the buffer, which an earlier call with smaller tiles may have grown
  scan_generic(InPlain{rhist}, InPlain{rhist}, OutStore{rhist}, counts + 1,
               std::min(rhist_cap, max_tiles_y * chunk_cap), counts + 2, scratch, st);
  if (blocks > 0)
    hipLaunchKernelGGL(k_rows_write, dim3((unsigned)blocks), dim3(256), 0, st, vinfo, cview,
                       counts + 0, vval, rec, views, S, rhist, rhist_cap, row_cap, runs, flag);
}

void expand(const RowRuns& rr, int n_rows, const DView* views, int n_views, int64_t n_tiles,
            int64_t max_tiles_x, const uint2* runs, int64_t chunk_cap,
            int64_t hist_cap, int64_t pair_cap, const uint32_t* n_pairs, uint4* rinfo,
            uint32_t* crow, uint32_t* hist, uint32_t* counts, uint32_t* pval, uint2* ranges,
            uint32_t* flag, void* scratch, hipStream_t st) {
  // counts: [0..7] chunks of each XCD, [8] table entries, [9] pairs written
  if (n_rows <= 0 || n_tiles <= 0) {
    fill_u32(counts, kXcds + 2, 0u, st);
    fill_u32(reinterpret_cast<uint32_t*>(ranges), 2 * n_tiles, 0u, st);
    return;
  }
  hipLaunchKernelGGL(k_row_table, dim3(1), dim3(1024), 0, st, rr, n_rows, views, n_views,
                     rinfo, (uint32_t)std::min<int64_t>(hist_cap, UINT32_MAX), counts, flag);
  hipLaunchKernelGGL(k_chunk_rows, dim3((unsigned)n_rows), dim3(256), 0, st, rinfo, chunk_cap,
                     crow);
  // per XCD enough workgroups to fill its CUs, each striding over that XCD's chunks
  const int64_t per_xcd = std::min<int64_t>((chunk_cap + 3) / 4, 1024);
  const unsigned blocks = (unsigned)(kXcds * per_xcd);
  hipLaunchKernelGGL(k_expand_count, dim3(blocks), dim3(256), 0, st, rinfo, crow, chunk_cap,
                     counts, runs, hist, hist_cap);
  // at most (largest tiles_x) x chunks entries (see splats_to_rows)
  scan_generic(InPlain{hist}, InPlain{hist}, OutStore{hist}, counts + kXcds,
               std::min(hist_cap, max_tiles_x * chunk_cap), counts + kXcds + 1, scratch, st);
  hipLaunchKernelGGL(k_expand_ranges, dim3((unsigned)((n_tiles + 255) / 256)), dim3(256), 0, st,
                     rinfo, views, n_views, hist, counts + kXcds, counts + kXcds + 1, n_pairs,
                     n_tiles, (uint32_t)std::min<int64_t>(pair_cap, 1 << 29), ranges, flag);
  // (pairs beyond 2^29, which the 32-bit buffer offsets cannot address, are not written and
  // are reported as a capacity overflow by the ranges pass)
  hipLaunchKernelGGL(k_expand_write, dim3(blocks), dim3(256), 0, st, rinfo, crow, chunk_cap,
                     counts, runs, hist, hist_cap, (uint32_t)std::min<int64_t>(pair_cap, 1 << 29),
                     pval, flag);
}

void tile_ids_of(const uint2* ranges, int64_t n_tiles, int64_t n, uint32_t* ids, hipStream_t st) {
  if (n_tiles <= 0 || n <= 0) return;
  const int64_t blocks = std::min<int64_t>(n_tiles, 1 << 20);
  hipLaunchKernelGGL(k_tile_ids, dim3((unsigned)blocks), dim3(256), 0, st, ranges, n_tiles, n,
                     ids);
}


void view_setup(DView* views, int n_views, float jac_margin, hipStream_t st) {
  hipLaunchKernelGGL(k_view_setup, dim3((n_views + 63) / 64), dim3(64), 0, st, views, n_views,
                     jac_margin);
}

}  // namespace g4d
