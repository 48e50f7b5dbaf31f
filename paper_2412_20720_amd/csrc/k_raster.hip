// Forward and backward rasterization of sorted splats (Sec. 3.2, eq:4dblending).
//
// Work decomposition for gfx950: every 64-lane wave owns an 8x8 pixel block of a screen tile
// and walks the tile's depth-ordered list on its own, with no workgroup barrier.  A wave
// stages up to 64 list entries at a time in its private slice of LDS: each lane fetches one
// record, the lanes whose record cannot reach the wave's 8x8 block drop out (ballot +
// mbcnt compaction), and the survivors are evaluated by all 64 pixels from LDS broadcasts.
// A wave stops as soon as all of its pixels have reached the transmittance stop.
//
// Per pixel and entry i (front to back): d2 = Mahalanobis distance of the pixel centre,
// skip if d2 > cutoff^2; alpha = min(alpha_max, opacity p_i(t) exp(-d2/2)); skip if
// alpha < alpha_min; stop (entry not composited) if T (1 - alpha) < T_min; else
// C += T alpha c_i, T *= 1 - alpha.  Output C + T background.
//
// Backward: each pixel walks its list in reverse from its last composited entry, rebuilding
// the transmittance in front of an entry as T / (1 - alpha) and the color behind it as
// R <- alpha c + (1 - alpha) R (R starts at the background).  With g = dL/dC:
//   dL/dc_i = g T_i alpha_i,  dL/dalpha_i = sum_ch g (c_i - R_i) T_i,
// and through alpha = opacity p_t exp(-d2/2) (unless clamped at alpha_max) to the screen mean,
// the conic and opacity p_t.  The nine per-Gaussian values are summed over the wave with DPP
// row reductions and four readlanes, then one vector atomic (lanes 0..8) adds them to the
// (view, Gaussian) gradient slot.
#include <hip/hip_runtime.h>

#include "g4d_internal.h"

namespace g4d {
namespace {

constexpr float kNegHalfLog2e = -0.72134752044448170f;  // -log2(e) / 2

#define G4D_WAVE_SYNC()                                     \
  do {                                                      \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                        \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

struct Staged {
  float4 a;  // u, v, conic a, 2 * conic b
  float4 b;  // conic c, opacity * p_t, r, g
  float4 c;  // b, list position (bits), slot (bits), unused
};

__device__ __forceinline__ int find_view(const int32_t* __restrict__ tile_base, int n_views,
                                         int tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_base[mid] <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ float mahalanobis(float dx, float dy, const float4& a, float c) {
  return fmaf(dx, fmaf(a.z, dx, a.w * dy), (c * dy) * dy);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Sum over the 64 lanes; the result is uniform.
__device__ __forceinline__ float wave_sum(float x) {
  x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp<0x141>(x);  // row_half_mirror
  x += dpp<0x140>(x);  // row_mirror: every lane now holds its 16-lane row sum
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
  return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
  return x;
}

struct WaveTile {
  int tile, v, px, py, lane, w;
  bool inside;
  float pxc, pyc, qx0, qx1, qy0, qy1;
  uint2 range;
};

// Workgroups are dispatched to the 8 XCDs round-robin (block b on XCD b mod 8), and each XCD
// has its own L2.  Block b is given logical block (b mod 8) * per + b / 8, so that every XCD
// works through a contiguous run of tiles whose large splats it shares in its L2.  The grid
// is padded to 8 * per blocks; logical blocks past the end do nothing.
__device__ __forceinline__ int xcd_logical_block(int per) {
  return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}

template <int TILE>
__device__ __forceinline__ bool wave_tile(const RasterArgs& a, WaveTile& t) {
  constexpr int QX = TILE / 8, QPT = QX * QX;
  t.lane = threadIdx.x & 63;
  t.w = threadIdx.x >> 6;
  const int gw = __builtin_amdgcn_readfirstlane(xcd_logical_block(a.blocks_per_xcd) * 4 + t.w);
  t.tile = gw / QPT;
  if (t.tile >= a.n_tiles) return false;
  const int q = gw - t.tile * QPT;
  t.v = find_view(a.tile_base, a.n_views, t.tile);
  const DView& V = a.views[t.v];
  const int lt = t.tile - V.tile_base;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const int bx = tx * TILE + (q % QX) * 8, by = ty * TILE + (q / QX) * 8;
  t.px = bx + (t.lane & 7);
  t.py = by + (t.lane >> 3);
  t.inside = t.px < V.width && t.py < V.height;
  t.pxc = (float)t.px + 0.5f;
  t.pyc = (float)t.py + 0.5f;
  t.qx0 = (float)bx + 0.5f;
  t.qx1 = (float)bx + 7.5f;
  t.qy0 = (float)by + 0.5f;
  t.qy1 = (float)by + 7.5f;
  t.range = a.ranges[t.tile];
  return true;
}

// Fetch list entry j (if in range) and keep it if its box reaches the wave's pixel block.
__device__ __forceinline__ bool fetch_entry(const RasterArgs& a, const WaveTile& t, uint32_t j,
                                            bool in_range, Staged& s) {
  if (!in_range) return false;
  const uint32_t slot = a.pval[j];
  const float4* r = reinterpret_cast<const float4*>(a.rec + (size_t)slot * kRec);
  const float4 r0 = r[0], r1 = r[1], r2 = r[2];
  const bool keep = (r0.x + r2.y >= t.qx0) && (r0.x - r2.y <= t.qx1) &&
                    (r0.y + r2.z >= t.qy0) && (r0.y - r2.z <= t.qy1);
  s.a = make_float4(r0.x, r0.y, r0.z, 2.f * r0.w);
  s.b = r1;
  s.c = make_float4(r2.x, __int_as_float((int)j), __uint_as_float(slot), 0.f);
  return keep;
}

// Stage up to BATCH list entries starting at `base` (fetch rounds of 64 lanes) into `st`,
// keeping only those that can reach the wave's block; returns how many were kept.
template <int BATCH>
__device__ __forceinline__ int stage_batch(const RasterArgs& a, const WaveTile& t, int base,
                                           int end, Staged* st) {
  int n = 0;
#pragma unroll
  for (int r = 0; r < (BATCH + 63) / 64; ++r) {
    const int j = base + r * 64 + t.lane;
    const bool in = (BATCH >= 64 || t.lane < BATCH) && j < end;
    Staged s;
    const bool keep = fetch_entry(a, t, (uint32_t)j, in, s);
    const uint64_t mask = __ballot(keep);
    if (keep) {
      const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
      st[n + pos] = s;
    }
    n += __popcll(mask);
  }
  return n;
}

template <int TILE, int BATCH>
__global__ __launch_bounds__(256) void k_raster_fwd(RasterArgs a) {
  __shared__ Staged stage[4][BATCH];
  WaveTile t;
  if (!wave_tile<TILE>(a, t)) return;
  const DView& V = a.views[t.v];
  const DSettings& S = a.S;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  int last = -1;
  uint32_t evals = 0, contrib = 0;
  bool done = !t.inside;
  Staged* st = stage[t.w];
  const int end = (int)t.range.y;
  for (int base = (int)t.range.x; base < end; base += BATCH) {
    if (__ballot(!done) == 0ull) break;
    const int n = stage_batch<BATCH>(a, t, base, end, st);
    G4D_WAVE_SYNC();
    for (int k = 0; k < n; ++k) {
      const float4 e0 = st[k].a, e1 = st[k].b;
      const float2 e2 = make_float2(st[k].c.x, st[k].c.y);
      if (!done) {
        const float dx = t.pxc - e0.x, dy = t.pyc - e0.y;
        const float d2 = mahalanobis(dx, dy, e0, e1.x);
        if (d2 <= S.cut2) {
          ++evals;
          const float alpha = fminf(S.alpha_max, e1.y * exp2f(d2 * kNegHalfLog2e));
          if (alpha >= S.alpha_min) {
            const float Tn = T * (1.f - alpha);
            if (Tn < S.T_min) {
              done = true;
            } else {
              const float wgt = T * alpha;
              C0 = fmaf(wgt, e1.z, C0);
              C1 = fmaf(wgt, e1.w, C1);
              C2 = fmaf(wgt, e2.x, C2);
              T = Tn;
              last = __float_as_int(e2.y);
              ++contrib;
            }
          }
        }
      }
      if (__ballot(!done) == 0ull) break;
    }
    G4D_WAVE_SYNC();
  }
  if (t.inside) {
    const int64_t hw = (int64_t)V.width * V.height;
    const int64_t pix = (int64_t)t.py * V.width + t.px;
    float* rgb = a.out_rgb + 3 * (int64_t)V.pix_base;
    rgb[pix] = fmaf(T, V.bg[0], C0);
    rgb[hw + pix] = fmaf(T, V.bg[1], C1);
    rgb[2 * hw + pix] = fmaf(T, V.bg[2], C2);
    const int64_t gp = (int64_t)V.pix_base + pix;
    if (a.out_T) a.out_T[gp] = T;
    a.px_T[gp] = T;
    a.px_last[gp] = last;
    if (a.px_evals) a.px_evals[gp] = min(evals, 65535u) | (min(contrib, 65535u) << 16);
  }
}

template <int TILE, int BATCH>
__global__ __launch_bounds__(256) void k_raster_bwd(RasterArgs a) {
  __shared__ Staged stage[4][BATCH];
  WaveTile t;
  if (!wave_tile<TILE>(a, t)) return;
  const DView& V = a.views[t.v];
  const DSettings& S = a.S;
  float T = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  int last = -1;
  if (t.inside) {
    const int64_t hw = (int64_t)V.width * V.height;
    const int64_t pix = (int64_t)t.py * V.width + t.px;
    const int64_t gp = (int64_t)V.pix_base + pix;
    T = a.px_T[gp];
    last = a.px_last[gp];
    const float* dl = a.dL + 3 * (int64_t)V.pix_base;
    g0 = dl[pix];
    g1 = dl[hw + pix];
    g2 = dl[2 * hw + pix];
  }
  const int hi_last = wave_max(last);
  if (hi_last < 0) return;
  float R0 = V.bg[0], R1 = V.bg[1], R2 = V.bg[2];
  Staged* st = stage[t.w];
  const int lo_list = (int)t.range.x;
  for (int hi = hi_last + 1; hi > lo_list; hi -= BATCH) {
    const int lo = max(lo_list, hi - BATCH);
    const int n = stage_batch<BATCH>(a, t, lo, hi, st);
    G4D_WAVE_SYNC();
    for (int k = n - 1; k >= 0; --k) {
      const float4 e0 = st[k].a, e1 = st[k].b, e2 = st[k].c;
      const int jk = __float_as_int(e2.y);
      float q[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      bool contrib = false;
      if (jk <= last) {
        const float dx = t.pxc - e0.x, dy = t.pyc - e0.y;
        const float d2 = mahalanobis(dx, dy, e0, e1.x);
        if (d2 <= S.cut2) {
          const float G = exp2f(d2 * kNegHalfLog2e);
          const float araw = e1.y * G;
          const float alpha = fminf(S.alpha_max, araw);
          if (alpha >= S.alpha_min) {
            contrib = true;
            const float Tb = __fdividef(T, 1.f - alpha);
            const float wgt = alpha * Tb;
            q[6] = g0 * wgt;
            q[7] = g1 * wgt;
            q[8] = g2 * wgt;
            const float d0 = e1.z - R0, d1 = e1.w - R1, dd2 = e2.x - R2;
            const float da = Tb * fmaf(g0, d0, fmaf(g1, d1, g2 * dd2));
            R0 = fmaf(alpha, d0, R0);
            R1 = fmaf(alpha, d1, R1);
            R2 = fmaf(alpha, dd2, R2);
            if (araw < S.alpha_max) {
              const float hb = 0.5f * e0.w;  // conic b
              q[5] = da * G;
              const float sa = da * alpha;
              q[0] = sa * fmaf(e0.z, dx, hb * dy);
              q[1] = sa * fmaf(hb, dx, e1.x * dy);
              q[2] = -0.5f * sa * dx * dx;
              q[3] = -sa * dx * dy;
              q[4] = -0.5f * sa * dy * dy;
            }
            T = Tb;
          }
        }
      }
      if (__ballot(contrib) != 0ull) {
        float sum[9];
#pragma unroll
        for (int f = 0; f < 9; ++f) sum[f] = wave_sum(q[f]);
        float val = 0.f;
#pragma unroll
        for (int f = 0; f < 9; ++f) val = (t.lane == f) ? sum[f] : val;
        if (t.lane < 9) {
          const uint32_t slot = __float_as_uint(e2.z);
          unsafeAtomicAdd(a.grad2d + (size_t)slot * kGrad2d + t.lane, val);
        }
      }
    }
    G4D_WAVE_SYNC();
  }
}

template <int TILE, int BATCH>
void launch_raster(const RasterArgs& a, hipStream_t st, bool backward) {
  constexpr int QPT = (TILE / 8) * (TILE / 8);
  const int64_t waves = (int64_t)a.n_tiles * QPT;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks == 0) return;
  RasterArgs b = a;
  b.blocks_per_xcd = (int)((blocks + 7) / 8);
  const unsigned grid = 8u * (unsigned)b.blocks_per_xcd;
  if (backward)
    hipLaunchKernelGGL((k_raster_bwd<TILE, BATCH>), dim3(grid), dim3(256), 0, st, b);
  else
    hipLaunchKernelGGL((k_raster_fwd<TILE, BATCH>), dim3(grid), dim3(256), 0, st, b);
}

template <int TILE>
void dispatch_batch(const RasterArgs& a, hipStream_t st, bool backward) {
  switch (a.S.lds_batch) {
    case 32: launch_raster<TILE, 32>(a, st, backward); break;
    case 128: launch_raster<TILE, 128>(a, st, backward); break;
    default: launch_raster<TILE, 64>(a, st, backward); break;
  }
}

void dispatch(const RasterArgs& a, hipStream_t st, bool backward) {
  switch (a.S.tile) {
    case 8: dispatch_batch<8>(a, st, backward); break;
    case 32: dispatch_batch<32>(a, st, backward); break;
    default: dispatch_batch<16>(a, st, backward); break;
  }
}

}  // namespace

void raster_forward(const RasterArgs& a, hipStream_t st) { dispatch(a, st, false); }
void raster_backward(const RasterArgs& a, hipStream_t st) { dispatch(a, st, true); }

}  // namespace g4d
