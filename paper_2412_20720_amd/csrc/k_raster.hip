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
// C += T alpha c_i, T *= 1 - alpha.  Output C + T background.  The first skip is tested
// against the entry's reach (the cutoff, or the smaller d2 beyond which alpha < alpha_min,
// slightly widened), which drops only pixels that the second skip would drop.
//
// Backward: each pixel walks its list in reverse from its last composited entry, rebuilding
// the transmittance in front of an entry as T / (1 - alpha) and the color behind it as
// R <- alpha c + (1 - alpha) R (R starts at the background).  With g = dL/dC:
//   dL/dc_i = g T_i alpha_i,  dL/dalpha_i = sum_ch g (c_i - R_i) T_i,
// and through alpha = opacity p_t exp(-d2/2) (unless clamped at alpha_max) to the screen mean,
// the conic and opacity p_t.  A lane first adds the contributions of its own pixels; the nine
// per-Gaussian values are then summed over the wave by a permlane-swap transpose-reduce and
// one vector atomic (nine lanes) adds them to the (view, Gaussian) gradient slot.
//
// Extra channels (CX > 0): each staged entry also carries CX payload values (normalized
// features, camera depth, flow; zero padding) in a second wave-private LDS array; they are
// composited with the same weights, add g_x . payload to g . c in the backward, and their
// per-entry partials are reduced like the nine above and added to the feature and depth
// gradients.  All pixels of a lane are evaluated together, so each payload value read from
// LDS serves every pixel of the lane.
#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "g4d_internal.h"

namespace g4d {
namespace {

constexpr float kNegHalfLog2e = -0.72134752044448170f;  // -log2(e) / 2
constexpr float kInvNegHalfLog2e = -1.38629436111989061f;  // 1 / kNegHalfLog2e = -2 ln 2

// alpha = min(alpha_max, opacity p_t G) with G = exp(-d2 / 2) <= 1, so an entry whose
// opacity p_t lies below alpha_max cannot be clamped at any pixel.  A staged batch made only of
// such entries runs a copy of the entry loop without the clamp; the margin 2^-12 covers the
// rounding of d2 near 0 (where the computed G may exceed 1 by an ulp or two), so both copies
// give bit-identical results.
constexpr float kNoClampScale = 1.f - 1.f / 4096.f;

// A lane's pixels are tested against an entry in groups of kSlotGroup: the group is skipped
// when none of its pixels in the whole wave is covered; otherwise all of them are evaluated
// without branches, which lets the compiler interleave their independent dependency chains.
// Measured on the 300k/16-view workload (32-pixel tiles, 4 pixels per lane), groups of 1 are
// fastest: the skipped work outweighs the extra instruction-level parallelism of larger groups.
#ifndef G4D_SLOT_GROUP
#define G4D_SLOT_GROUP 1
#endif
constexpr int kSlotGroup = G4D_SLOT_GROUP;

#define G4D_WAVE_SYNC()                                     \
  do {                                                      \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
    __builtin_amdgcn_wave_barrier();                        \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
  } while (0)

// A staged entry carries the conic pre-multiplied by kNegHalfLog2e, so that the quadratic
// form evaluated at a pixel is directly the base-2 exponent of exp(-d2 / 2).
struct Staged {
  float4 a;  // u, v, k conic a, 2 k conic b
  float4 b;  // k conic c, opacity * p_t, r, g
  float4 c;  // b, list position (bits), slot (bits), k reach2 (the lowest pw it can composite at)
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

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
  return x;
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b on XCD b mod 8), and each XCD
// has its own L2.  Block b is given logical block (b mod 8) * per + b / 8, so that every XCD
// works through a contiguous run of tiles whose large splats it shares in its L2.  The grid
// is padded to 8 * per blocks; logical blocks past the end do nothing.
__device__ __forceinline__ int xcd_logical_block(int per) {
  return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}

struct WaveTile {
  int tile, v, lane, w;
  int bx, by;                      // pixel origin of the wave's block
  float qx0, qx1, qy0, qy1;        // pixel-centre box of the block
  uint2 range;
};

// Map logical wave gw to (tile, block of BW x BH pixels).  TILE is a multiple of BW and BH.
template <int TILE, int BW, int BH>
__device__ __forceinline__ bool wave_tile_at(const RasterArgs& a, int gw, WaveTile& t) {
  constexpr int QX = TILE / BW, QPT = QX * (TILE / BH);
  t.lane = threadIdx.x & 63;
  t.w = threadIdx.x >> 6;
  t.tile = gw / QPT;
  if (t.tile >= a.n_tiles) return false;
  const int q = gw - t.tile * QPT;
  t.v = find_view(a.tile_base, a.n_views, t.tile);
  const DView& V = a.views[t.v];
  const int lt = t.tile - V.tile_base;
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  t.bx = tx * TILE + (q % QX) * BW;
  t.by = ty * TILE + (q / QX) * BH;
  t.qx0 = (float)t.bx + 0.5f;
  t.qx1 = (float)(t.bx + BW) - 0.5f;
  t.qy0 = (float)t.by + 0.5f;
  t.qy1 = (float)(t.by + BH) - 0.5f;
  t.range = a.ranges[t.tile];
  return true;
}

// The grid's own mapping: logical wave (XCD-aware logical block) * 4 + wave in the workgroup.
template <int TILE, int BW, int BH>
__device__ __forceinline__ bool wave_tile(const RasterArgs& a, WaveTile& t) {
  const int gw = __builtin_amdgcn_readfirstlane(xcd_logical_block(a.blocks_per_xcd) * 4 +
                                                (int)(threadIdx.x >> 6));
  return wave_tile_at<TILE, BW, BH>(a, gw, t);
}

// Fetch list entry j (if in range) and keep it if its box reaches the wave's pixel block.
__device__ __forceinline__ bool fetch_entry(const RasterArgs& a, const WaveTile& t, uint32_t j,
                                            bool in_range, Staged& s) {
  if (!in_range) return false;
  const uint32_t slot = a.pval[j];
  const float4* r = reinterpret_cast<const float4*>(a.rec + (size_t)slot * kRec);
  const float4 r0 = r[0], r1 = r[1], r2 = r[2];
  bool keep = (r0.x + r2.y >= t.qx0) && (r0.x - r2.y <= t.qx1) &&
              (r0.y + r2.z >= t.qy0) && (r0.y - r2.z <= t.qy1);
  const float reach = reach2(r1.y, a.S);
  if (keep) {
    // exact test: the ellipse's x-range over the block's rows must meet the block's columns
    float xl, xr;
    keep = ellipse_band_xrange(r0.z, r0.w, r1.x, reach * 1.001f, r2.y, r2.z,
                               t.qy0 - r0.y, t.qy1 - r0.y, xl, xr) &&
           r0.x + xr >= t.qx0 && r0.x + xl <= t.qx1;
  }
  s.a = make_float4(r0.x, r0.y, kNegHalfLog2e * r0.z, 2.f * kNegHalfLog2e * r0.w);
  s.b = make_float4(kNegHalfLog2e * r1.x, r1.y, r1.z, r1.w);
  s.c = make_float4(r2.x, __int_as_float((int)j), __uint_as_float(slot), kNegHalfLog2e * reach);
  return keep;
}

// Stage up to BATCH list entries starting at `base` (fetch rounds of 64 lanes) into `st`,
// keeping only those that can reach the wave's block; returns how many were kept, and in
// `clamp_free` whether none of them can reach alpha_max.
template <int BATCH>
__device__ __forceinline__ int stage_batch(const RasterArgs& a, const WaveTile& t, int base,
                                           int end, Staged* st, bool& clamp_free) {
  int n = 0;
  clamp_free = true;
  const float no_clamp = a.S.alpha_max * kNoClampScale;
#pragma unroll
  for (int r = 0; r < (BATCH + 63) / 64; ++r) {
    const int j = base + r * 64 + t.lane;
    const bool in = (BATCH >= 64 || t.lane < BATCH) && j < end;
    Staged s;
    const bool keep = fetch_entry(a, t, (uint32_t)j, in, s);
    const uint64_t mask = __ballot(keep);
    clamp_free = clamp_free && __ballot(keep && !(s.b.y < no_clamp)) == 0ull;
    if (keep) {
      const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
      st[n + pos] = s;
    }
    n += __popcll(mask);
  }
  return n;
}

// Copy the CX payload values of the n staged entries into xp[k * CX + c] (all lanes; the
// caller synchronizes the wave before and after).  Loads go out in rounds of kPayloadChunk per
// lane before any of them is stored, so their latencies overlap.
constexpr int kPayloadChunk = 12;

template <int CX>
__device__ __forceinline__ void stage_payload(const RasterArgs& a, const WaveTile& t,
                                              const Staged* st, int n, float* xp) {
  const size_t vbase = (size_t)t.v * (size_t)a.n_gauss;
  const int total = n * CX;
  for (int base = 0; base < total; base += 64 * kPayloadChunk) {
    float val[kPayloadChunk];
#pragma unroll
    for (int r = 0; r < kPayloadChunk; ++r) {
      const int idx = base + 64 * r + t.lane;
      const int k = idx / CX, c = idx - k * CX;
      val[r] = 0.f;
      if (idx < total) {
        const size_t slot = __float_as_uint(st[k].c.z);
        if (c < a.n_feat) {
          val[r] = a.fn[(slot - vbase) * (size_t)a.n_feat + c];
        } else if (c < a.n_ext) {
          const int e = c - a.n_feat;
          if (a.has_depth && e == 0)
            val[r] = a.rec[slot * kRec + 11];
          else
            val[r] = a.flow[slot * 2 + (e - a.has_depth)];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kPayloadChunk; ++r) {
      const int idx = base + 64 * r + t.lane;
      if (idx < total) xp[idx] = val[r];
    }
  }
}

// A lane owns PXX x PXY pixels of its wave's (8 PXX) x (8 PXY) block: (lane % 8 + 8 a,
// lane / 8 + 8 b), a < PXX, b < PXY.  Pixel p = b * PXX + a.
template <int PXX, int PXY>
struct LanePixels {
  static constexpr int P = PXX * PXY;
  int px[P], py[P];
  bool inside[P];
  __device__ __forceinline__ void init(const WaveTile& t, const DView& V) {
#pragma unroll
    for (int b = 0; b < PXY; ++b)
#pragma unroll
      for (int a = 0; a < PXX; ++a) {
        const int p = b * PXX + a;
        px[p] = t.bx + (t.lane & 7) + 8 * a;
        py[p] = t.by + (t.lane >> 3) + 8 * b;
        inside[p] = px[p] < V.width && py[p] < V.height;
      }
  }
};

// exp2 on the hardware instruction; its argument here is >= -6.5 log2(e) (d2 <= 9), far
// from the range where the library version adds denormal handling.
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

template <int TILE, int BATCH, int PXX, int PXY, bool COUNT, int CX>
__device__ __forceinline__ void raster_fwd_wave(const RasterArgs& a, const WaveTile& t,
                                                Staged* st, float* xp) {
  constexpr int P = PXX * PXY;
  // with extra channels a lane's pixels form one group (see the header)
  constexpr int kGroup = CX > 0 ? P : (kSlotGroup < P ? kSlotGroup : P);
  constexpr int XC = CX > 0 ? CX : 1;
  float X[P][XC];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int c = 0; c < XC; ++c) X[p][c] = 0.f;
  const DView& V = a.views[t.v];
  const DSettings& S = a.S;
  LanePixels<PXX, PXY> L;
  L.init(t, V);
  // lo[p]: a pixel takes part in an entry when the scaled quadratic form pw = k d2 is at least
  // lo[p]; lo is k cutoff^2 while the pixel is live and +inf once it has stopped (or lies
  // outside the image), so one compare covers both tests.
  const float lo_cut = kNegHalfLog2e * S.cut2;
  float T[P], C0[P], C1[P], C2[P], pxc[P], pyc[P], lo[P];
  int last[P];
  uint32_t evals[P], contrib[P];
  bool any_live = false;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T[p] = 1.f;
    C0[p] = C1[p] = C2[p] = 0.f;
    pxc[p] = (float)L.px[p] + 0.5f;
    pyc[p] = (float)L.py[p] + 0.5f;
    last[p] = -1;
    evals[p] = contrib[p] = 0;
    lo[p] = L.inside[p] ? lo_cut : INFINITY;
    any_live |= L.inside[p];
  }
  bool done = __ballot(any_live) == 0ull;
  const int end = (int)t.range.y;
  for (int base = (int)t.range.x; base < end && !done; base += BATCH) {
    bool clamp_free;  // not used here: a second copy of the loop costs the forward occupancy
    const int n = stage_batch<BATCH>(a, t, base, end, st, clamp_free);
    G4D_WAVE_SYNC();
    if constexpr (CX > 0) {
      stage_payload<CX>(a, t, st, n, xp);
      G4D_WAVE_SYNC();
    }
    for (int k = 0; k < n; ++k) {
      const float4 e0 = st[k].a, e1 = st[k].b;
      const float4 e2 = st[k].c;
      bool any_stop = false;
      bool any_take = false;
      float wk[P];  // T alpha of this entry per pixel, 0 where it is not composited
#pragma unroll
      for (int p = 0; p < P; ++p) wk[p] = 0.f;
#pragma unroll
      for (int g = 0; g < P; g += kGroup) {
        float pwg[kGroup];
        bool ing[kGroup];
        bool gin = false;
#pragma unroll
        for (int i = 0; i < kGroup; ++i) {
          const int p = g + i;
          const float dx = pxc[p] - e0.x, dy = pyc[p] - e0.y;
          pwg[i] = mahalanobis(dx, dy, e0, e1.x);
          // Pixel still live and within the cutoff.  The counting variant also applies the
          // entry's reach, as the backward does, so that its count of evaluated pairs is the
          // backward's; the timed forward leaves that test out (one more instruction per pixel
          // costs it more than the skipped pixels save).
          ing[i] = pwg[i] >= (COUNT ? __builtin_amdgcn_fmed3f(lo[p], e2.w, INFINITY) : lo[p]);
          gin |= ing[i];
        }
        if (__ballot(gin) == 0ull) continue;
#pragma unroll
        for (int i = 0; i < kGroup; ++i) {
          const int p = g + i;
          const float pw = pwg[i];
          const bool in = ing[i];
          const float alpha = fminf(S.alpha_max, e1.y * fast_exp2(pw));
          const bool ok = in && alpha >= S.alpha_min;
          const float Tn = fmaf(-T[p], alpha, T[p]);
          // Tn >= T_min on the bit patterns: both are non-negative floats (alpha <= alpha_max
          // < 1), where the integer order is the float order, so the stop is exactly the
          // negation and follows from the take with a mask operation
          const bool take = ok && __float_as_int(Tn) >= __float_as_int(S.T_min);
          const bool stop = ok && !take;
          const float wgt = take ? T[p] * alpha : 0.f;
          C0[p] = fmaf(wgt, e1.z, C0[p]);
          C1[p] = fmaf(wgt, e1.w, C1[p]);
          C2[p] = fmaf(wgt, e2.x, C2[p]);
          wk[p] = wgt;
          any_take |= take;
          T[p] = take ? Tn : T[p];
          last[p] = take ? __float_as_int(e2.y) : last[p];
          lo[p] = stop ? INFINITY : lo[p];
          any_stop |= stop;
          if (COUNT) {
            evals[p] += in ? 1u : 0u;
            contrib[p] += take ? 1u : 0u;
          }
        }
      }
      if constexpr (CX > 0) {
        if (__ballot(any_take) != 0ull) {
          const float* xk = xp + k * CX;
#pragma unroll
          for (int c = 0; c < CX; ++c) {
            const float x = xk[c];
#pragma unroll
            for (int p = 0; p < P; ++p) X[p][c] = fmaf(wk[p], x, X[p][c]);
          }
        }
      }
      if (__ballot(any_stop) != 0ull) {
        any_live = false;
#pragma unroll
        for (int p = 0; p < P; ++p) any_live |= lo[p] != INFINITY;
        done = __ballot(any_live) == 0ull;
        if (done) break;
      }
    }
    G4D_WAVE_SYNC();
  }
  const int64_t hw = (int64_t)V.width * V.height;
  float* rgb = a.out_rgb + 3 * (int64_t)V.pix_base;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (!L.inside[p]) continue;
    const int64_t pix = (int64_t)L.py[p] * V.width + L.px[p];
    float bg0 = V.bg[0], bg1 = V.bg[1], bg2 = V.bg[2];
    if (a.bg_px) {  // per-pixel background (the sky), same layout as the image
      const float* b = a.bg_px + 3 * (int64_t)V.pix_base + pix;
      bg0 = b[0];
      bg1 = b[hw];
      bg2 = b[2 * hw];
    }
    rgb[pix] = fmaf(T[p], bg0, C0[p]);
    rgb[hw + pix] = fmaf(T[p], bg1, C1[p]);
    rgb[2 * hw + pix] = fmaf(T[p], bg2, C2[p]);
    const int64_t gp = (int64_t)V.pix_base + pix;
    if (a.out_T) a.out_T[gp] = T[p];
    a.px_T[gp] = T[p];
    a.px_last[gp] = last[p];
    if (COUNT) a.px_evals[gp] = min(evals[p], 65535u) | (min(contrib[p], 65535u) << 16);
    if constexpr (CX > 0) {
      float* o = a.out_ch + (size_t)a.n_ext * (size_t)V.pix_base + pix;
#pragma unroll
      for (int c = 0; c < CX; ++c)
        if (c < a.n_ext) o[(size_t)c * hw] = X[p][c];
    }
  }
}

// One wave per (tile, block), mapped from its workgroup (XCD-aware).  A persistent grid whose
// waves take (tile, block) items from per-XCD atomic work queues was measured on the
// 300k-Gaussian, 16-view workload and was slower (raster_fwd 0.97 -> 1.53 ms, raster_bwd 1.99 ->
// 2.18 ms): the hardware dispatcher already balances the short, uneven waves.
template <int TILE, int BATCH, int PXX, int PXY, bool COUNT, int CX>
__global__ __launch_bounds__(256) void k_raster_fwd(RasterArgs a) {
  __shared__ Staged stage[4][BATCH];
  __shared__ float xstage[4][CX > 0 ? BATCH * CX : 1];
  const int w = threadIdx.x >> 6;
  WaveTile t;
  if (!wave_tile<TILE, 8 * PXX, 8 * PXY>(a, t)) return;
  raster_fwd_wave<TILE, BATCH, PXX, PXY, COUNT, CX>(a, t, stage[w], xstage[w]);
}

// Transpose-reduce of nine per-lane values over the wave.  v_permlane32_swap exchanges the
// upper 32 lanes of one register with the lower 32 lanes of another, so one swap and one add
// fold two values at once (value a over lanes 0-31, value b over lanes 32-63); a
// v_permlane16_swap folds two such registers into four values, one per 16-lane row; four DPP
// adds then sum each row.  Afterwards lane 16 r + i holds, for i = 0, 1 (and i = 2 in row 0),
// the total of value field(i, r) = 4 i + [0, 2, 1, 3][r].
__device__ __forceinline__ float fold32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float fold16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float row_sum(float x) {
  x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp<0x141>(x);  // row_half_mirror
  x += dpp<0x140>(x);  // row_mirror
  return x;
}

// Returns the lane's reduced value and sets `field` (0..8) for the lanes that hold one.
__device__ __forceinline__ float wave_reduce9(const float* q, int lane, int& field) {
  const float A = fold32(q[0], q[1]), B = fold32(q[2], q[3]);
  const float C = fold32(q[4], q[5]), D = fold32(q[6], q[7]);
  const float E = fold32(q[8], 0.f);
  const float F = row_sum(fold16(A, B));   // rows: q0, q2, q1, q3
  const float G = row_sum(fold16(C, D));   // rows: q4, q6, q5, q7
  const float H = row_sum(fold16(E, 0.f)); // row 0: q8
  const int r = lane >> 4, i = lane & 15;
  field = (i < 2 || (i == 2 && r == 0)) ? 4 * i + (((r & 1) << 1) | (r >> 1)) : -1;
  return i == 0 ? F : (i == 1 ? G : H);
}

// Transpose-reduce of N (a multiple of 4) per-lane values: r[j] then holds, in every lane of
// row `row` (lane / 16), the wave total of value 4 j + [0, 2, 1, 3][row].
template <int N>
__device__ __forceinline__ void wave_reduce_rows(const float* q, float* r) {
#pragma unroll
  for (int j = 0; j < N / 4; ++j)
    r[j] = row_sum(fold16(fold32(q[4 * j], q[4 * j + 1]), fold32(q[4 * j + 2], q[4 * j + 3])));
}

// Backward.  Per pixel the walk keeps T (transmittance in front of the entry, rebuilt by
// division) and gR = g . R (the upstream gradient dotted with the color behind the entry):
//   dL/dalpha = T_i (g . c_i - gR),  gR <- alpha (g . c_i) + (1 - alpha) gR.
// Per Gaussian the wave accumulates q = [dL/du, dL/dv, S_xx, S_xy, S_yy, dL/d(opacity p_t),
// dL/drgb] with S_.. the second moments of (dx, dy) weighted by dL/dalpha alpha; after the
// reduction they become dL/da = -S_xx / 2, dL/db = -S_xy, dL/dc = -S_yy / 2.
// Occupancy floors, measured on the 300k/16-view workload: the RGB backward is built for at
// least 4 waves per SIMD (at most 128 VGPRs; at 8 pixels per lane a few rarely used registers
// spill and it still wins, 2.16 -> 2.05 ms against 3 waves unbounded; 5 waves spill heavily,
// 5.3 ms), the extra-channel backward for 3 (its 35-channel variant drops from 197 to 168
// VGPRs with a few spills, 15.05 -> 13.64 ms; 3 blocks of its 48 KB of LDS fit a CU anyway).
template <int TILE, int BATCH, int PXX, int PXY, int CX>
__device__ __forceinline__ void raster_bwd_wave(const RasterArgs& a, const WaveTile& t,
                                                Staged* st, float* xp) {
  constexpr int P = PXX * PXY;
  static_assert(CX % 4 == 0, "extra channels come in groups of four");
  constexpr int kGroup = CX > 0 ? P : (kSlotGroup < P ? kSlotGroup : P);
  constexpr int XC = CX > 0 ? CX : 1;
  float gx[P][XC];  // upstream gradient of the extra channels per pixel (0: flow, padding)
  const DView& V = a.views[t.v];
  const DSettings& S = a.S;
  LanePixels<PXX, PXY> L;
  L.init(t, V);
  float T[P], g0[P], g1[P], g2[P], gR[P], pxc[P], pyc[P];
  // pixel centre relative to the block centre (ox, oy), and its products: the moment sums
  // below are taken in these coordinates and re-centred on the splat once per entry
  float rx[P], ry[P], rxx[P], rxy[P], ryy[P];
  const float ox = (float)t.bx + 4.f * PXX, oy = (float)t.by + 4.f * PXY;
  int last[P];
  int lane_last = -1, lane_first = INT_MAX;
  const int64_t hw = (int64_t)V.width * V.height;
  const float* dl = a.dL + 3 * (int64_t)V.pix_base;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T[p] = 1.f;
    g0[p] = g1[p] = g2[p] = 0.f;
    last[p] = -1;
    pxc[p] = (float)L.px[p] + 0.5f;
    pyc[p] = (float)L.py[p] + 0.5f;
    rx[p] = pxc[p] - ox;
    ry[p] = pyc[p] - oy;
    rxx[p] = rx[p] * rx[p];
    rxy[p] = rx[p] * ry[p];
    ryy[p] = ry[p] * ry[p];
    if (L.inside[p]) {
      const int64_t pix = (int64_t)L.py[p] * V.width + L.px[p];
      const int64_t gp = (int64_t)V.pix_base + pix;
      T[p] = a.px_T[gp];
      last[p] = a.px_last[gp];
      g0[p] = dl[pix];
      g1[p] = dl[hw + pix];
      g2[p] = dl[2 * hw + pix];
    }
    if constexpr (CX > 0) {
      const int n_grad = a.n_feat + a.has_depth;
      const float* dxp = a.dL_ch ? a.dL_ch + (size_t)a.n_ext * (size_t)V.pix_base +
                                       (size_t)L.py[p] * V.width + L.px[p]
                                 : nullptr;
#pragma unroll
      for (int c = 0; c < CX; ++c)
        gx[p][c] = (dxp && L.inside[p] && c < n_grad) ? dxp[(size_t)c * hw] : 0.f;
    }
    float bg0 = V.bg[0], bg1 = V.bg[1], bg2 = V.bg[2];
    if (a.bg_px && L.inside[p]) {
      const float* b = a.bg_px + 3 * (int64_t)V.pix_base + (int64_t)L.py[p] * V.width + L.px[p];
      bg0 = b[0];
      bg1 = b[hw];
      bg2 = b[2 * hw];
    }
    gR[p] = fmaf(g0[p], bg0, fmaf(g1[p], bg1, g2[p] * bg2));
    lane_last = max(lane_last, last[p]);
    lane_first = min(lane_first, last[p]);
  }
  const int hi_last = wave_max(lane_last);
  if (hi_last < 0) return;
  // entries at or before every pixel's last composited one need no per-pixel position test
  const int lo_last = __builtin_amdgcn_readfirstlane(wave_min(lane_first));
  const int lo_list = (int)t.range.x;
  for (int hi = hi_last + 1; hi > lo_list; hi -= BATCH) {
    const int lo = max(lo_list, hi - BATCH);
    bool clamp_free;
    const int n = stage_batch<BATCH>(a, t, lo, hi, st, clamp_free);
    G4D_WAVE_SYNC();
    if constexpr (CX > 0) {
      stage_payload<CX>(a, t, st, n, xp);
      G4D_WAVE_SYNC();
    }
    auto entries = [&](auto clamp_tag, auto check_tag) {
      constexpr bool kClamp = decltype(clamp_tag)::value;
      constexpr bool kCheckLast = decltype(check_tag)::value;
    for (int k = n - 1; k >= 0; --k) {
      const float4 e0 = st[k].a, e1 = st[k].b, e2 = st[k].c;
      const int jk = __float_as_int(e2.y);
      float qx[XC];
#pragma unroll
      for (int c = 0; c < XC; ++c) qx[c] = 0.f;
      // Per pixel the lane adds sa = alpha dL/dalpha (unclamped branch only) into the moments
      // q[0..5] = sum sa [rx, ry, rx^2, rx ry, ry^2, 1] of the block-centred pixel position
      // and the color partials into q[6..8]; once per entry they are turned into the
      // splat-centred moments and the partials (see below).
      float q[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      bool any = false;
#pragma unroll
      for (int g = 0; g < P; g += kGroup) {
        float pwg[kGroup];
        bool ing[kGroup];
        bool gin = false;
#pragma unroll
        for (int i = 0; i < kGroup; ++i) {
          const int p = g + i;
          const float dx = pxc[p] - e0.x, dy = pyc[p] - e0.y;
          pwg[i] = mahalanobis(dx, dy, e0, e1.x);
          ing[i] = (!kCheckLast || jk <= last[p]) && pwg[i] >= e2.w;
          gin |= ing[i];
        }
        if (__ballot(gin) == 0ull) continue;
        // g_x . payload per pixel, each payload value read once for the group
        float gcx[kGroup];
#pragma unroll
        for (int i = 0; i < kGroup; ++i) gcx[i] = 0.f;
        if constexpr (CX > 0) {
          const float* xk = xp + k * CX;
#pragma unroll
          for (int c = 0; c < CX; ++c) {
            const float x = xk[c];
#pragma unroll
            for (int i = 0; i < kGroup; ++i) gcx[i] = fmaf(gx[g + i][c], x, gcx[i]);
          }
        }
#pragma unroll
        for (int i = 0; i < kGroup; ++i) {
          const int p = g + i;
          const float pw = pwg[i];
          const bool in = ing[i];
          const float G = fast_exp2(pw);
          const float araw = e1.y * G;
          const float ac = kClamp ? fminf(S.alpha_max, araw) : araw;
          const bool take = in && ac >= S.alpha_min;
          // alpha = 0 for an entry the pixel did not composite: then T, gR, q[5..8] and the
          // moments below are left exactly as they were, without selects
          const float alpha = take ? ac : 0.f;
          // transmittance in front of the entry, T / (1 - alpha) = T + T alpha / (1 - alpha),
          // with v_rcp_f32 (about 1 ulp) instead of a correctly rounded division
          const float Tb = fmaf(T[p], alpha * __builtin_amdgcn_rcpf(1.f - alpha), T[p]);
          const float wgt = alpha * Tb;
          q[6] = fmaf(g0[p], wgt, q[6]);
          q[7] = fmaf(g1[p], wgt, q[7]);
          q[8] = fmaf(g2[p], wgt, q[8]);
          float gc = fmaf(g0[p], e1.z, fmaf(g1[p], e1.w, g2[p] * e2.x));
          if constexpr (CX > 0) {
#pragma unroll
            for (int c = 0; c < CX; ++c) qx[c] = fmaf(gx[p][c], wgt, qx[c]);
            gc += gcx[i];
          }
          const float diff = gc - gR[p];
          gR[p] = fmaf(alpha, diff, gR[p]);
          // dL/dalpha = Tb diff, so sa = alpha dL/dalpha = wgt diff
          const float sa = (!kClamp || araw < S.alpha_max) ? wgt * diff : 0.f;
          T[p] = Tb;
          q[0] = fmaf(sa, rx[p], q[0]);
          q[1] = fmaf(sa, ry[p], q[1]);
          q[2] = fmaf(sa, rxx[p], q[2]);
          q[3] = fmaf(sa, rxy[p], q[3]);
          q[4] = fmaf(sa, ryy[p], q[4]);
          q[5] += sa;
          any |= take;
        }
      }
      if (__ballot(any) != 0ull) {
        // Re-centre on the splat: with (cu, cv) its centre in block coordinates, dx = rx - cu,
        // so S_x = sum sa dx = q0 - cu q5, S_xx = q2 - cu q0 - cu S_x, S_xy = q3 - cu q1 -
        // cv S_x, S_yy = q4 - cv q1 - cv S_y.
        const float cu = e0.x - ox, cv = e0.y - oy;
        const float sx = fmaf(-cu, q[5], q[0]), sy = fmaf(-cv, q[5], q[1]);
        q[2] = fmaf(-cu, sx, fmaf(-cu, q[0], q[2]));
        q[3] = fmaf(-cv, sx, fmaf(-cu, q[1], q[3]));
        q[4] = fmaf(-cv, sy, fmaf(-cv, q[1], q[4]));
        // screen-mean partials (times k, the conic scale): dL/du ~ a S_x + b S_y, etc.
        const float hb = 0.5f * e0.w;  // k conic b
        q[0] = fmaf(e0.z, sx, hb * sy);
        q[1] = fmaf(hb, sx, e1.x * sy);
        // alpha = opacity p_t G on the unclamped branch, so sum G dL/dalpha = (sum sa) /
        // (opacity p_t); a composited entry has opacity p_t >= alpha_min > 0
        q[5] *= __builtin_amdgcn_rcpf(e1.y);
        int field;
        float val = wave_reduce9(q, t.lane, field);
        if (field >= 0) {
          val *= (field <= 1) ? kInvNegHalfLog2e
                              : ((field == 3) ? -1.f : ((field == 2 || field == 4) ? -0.5f : 1.f));
          const uint32_t slot = __float_as_uint(e2.z);
          unsafeAtomicAdd(a.grad2d + (size_t)slot * kGrad2d + field, val);
        }
        if constexpr (CX > 0) {
          float r[CX / 4];
          wave_reduce_rows<CX>(qx, r);
          const int row = t.lane >> 4, i = t.lane & 15;
          float v = r[0];
#pragma unroll
          for (int j = 1; j < CX / 4; ++j) v = (i == j) ? r[j] : v;
          const int c = 4 * i + (((row & 1) << 1) | (row >> 1));
          const size_t slot = __float_as_uint(e2.z);
          if (i < CX / 4 && c < a.n_feat) {
            const size_t gi = slot - (size_t)t.v * (size_t)a.n_gauss;
            unsafeAtomicAdd(a.dfn + gi * (size_t)a.n_feat + c, v);
          } else if (i < CX / 4 && a.has_depth && c == a.n_feat) {
            unsafeAtomicAdd(a.grad2d + slot * kGrad2d + G_DEPTH, v);
          }
        }
      }
    }
    };
    // the walk reaches list positions hi - 1 down to lo; past lo_last some pixel of the wave
    // has not begun its walk yet
    const bool check = hi - 1 > lo_last;
    if (clamp_free) {
      if (check) entries(std::false_type{}, std::true_type{});
      else entries(std::false_type{}, std::false_type{});
    } else {
      if (a.clamp_batches && t.lane == 0) atomicAdd(a.clamp_batches, 1u);
      if (check) entries(std::true_type{}, std::true_type{});
      else entries(std::true_type{}, std::false_type{});
    }
    G4D_WAVE_SYNC();
  }
}

template <int TILE, int BATCH, int PXX, int PXY, int CX>
__global__ __launch_bounds__(256, CX == 0 ? 4 : 3) void k_raster_bwd(RasterArgs a) {
  __shared__ Staged stage[4][BATCH];
  __shared__ float xstage[4][CX > 0 ? BATCH * CX : 1];
  const int w = threadIdx.x >> 6;
  WaveTile t;
  if (!wave_tile<TILE, 8 * PXX, 8 * PXY>(a, t)) return;
  raster_bwd_wave<TILE, BATCH, PXX, PXY, CX>(a, t, stage[w], xstage[w]);
}

// Grid of 4-wave workgroups, one wave per (8 PXX) x (8 PXY) block of every tile, padded to a
// multiple of the 8 XCDs (see xcd_logical_block); returns 0 when there is nothing to draw.
template <int TILE, int PXX, int PXY>
unsigned raster_grid(RasterArgs& b) {
  static_assert(TILE % (8 * PXX) == 0 && TILE % (8 * PXY) == 0, "block must tile the tile");
  constexpr int QPT = (TILE / (8 * PXX)) * (TILE / (8 * PXY));
  const int64_t waves = (int64_t)b.n_tiles * QPT;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks == 0) return 0u;
  b.blocks_per_xcd = (int)((blocks + 7) / 8);
  return 8u * (unsigned)b.blocks_per_xcd;
}

template <int TILE, int BATCH, int PXX, int PXY, int CX = 0>
void launch_backward(const RasterArgs& a, hipStream_t st) {
  RasterArgs b = a;
  const unsigned grid = raster_grid<TILE, PXX, PXY>(b);
  if (grid == 0u) return;
  hipLaunchKernelGGL((k_raster_bwd<TILE, BATCH, PXX, PXY, CX>), dim3(grid), dim3(256), 0, st, b);
}

template <int TILE, int BATCH, int PXX, int PXY, int CX = 0>
void launch_raster(const RasterArgs& a, hipStream_t st, bool backward) {
  if (backward) {
    launch_backward<TILE, BATCH, PXX, PXY, CX>(a, st);
    return;
  }
  RasterArgs b = a;
  const unsigned grid = raster_grid<TILE, PXX, PXY>(b);
  if (grid == 0u) return;
  if (CX == 0 && b.px_evals)
    hipLaunchKernelGGL((k_raster_fwd<TILE, BATCH, PXX, PXY, true, 0>), dim3(grid), dim3(256), 0, st,
                       b);
  else
    hipLaunchKernelGGL((k_raster_fwd<TILE, BATCH, PXX, PXY, false, CX>), dim3(grid), dim3(256), 0,
                       st, b);
}

// Extra channels: 64-entry batches, CX the smallest supported payload width that holds the E
// channels (the rest is zero padding).
template <int TILE, int PXX, int PXY>
void dispatch_ext_width(const RasterArgs& a, hipStream_t st, bool backward) {
  if (a.n_ext <= 4) launch_raster<TILE, 64, PXX, PXY, 4>(a, st, backward);
  else if (a.n_ext <= 8) launch_raster<TILE, 64, PXX, PXY, 8>(a, st, backward);
  else if (a.n_ext <= 16) launch_raster<TILE, 64, PXX, PXY, 16>(a, st, backward);
  else launch_raster<TILE, 64, PXX, PXY, 36>(a, st, backward);
}

// One or two pixels per lane (the runtime caps the extra-channel raster at two).
template <int TILE>
void dispatch_ext(const RasterArgs& a, hipStream_t st, bool backward) {
  if constexpr (TILE >= 16) {
    if (a.S.px_per_lane == 2) {
      dispatch_ext_width<TILE, 2, 1>(a, st, backward);
      return;
    }
  }
  dispatch_ext_width<TILE, 1, 1>(a, st, backward);
}

template <int TILE, int PXX, int PXY>
void dispatch_batch(const RasterArgs& a, hipStream_t st, bool backward) {
  switch (a.S.lds_batch) {
    case 32: launch_raster<TILE, 32, PXX, PXY>(a, st, backward); break;
    case 128: launch_raster<TILE, 128, PXX, PXY>(a, st, backward); break;
    default: launch_raster<TILE, 64, PXX, PXY>(a, st, backward); break;
  }
}

// 32x16 blocks (8 pixels per lane: 4 columns x 2 rows, so that the per-row terms of the
// quadratic form serve four pixels; 16x32 took 1% longer), backward only and at 32-pixel tiles.
template <int TILE>
void dispatch_backward8(const RasterArgs& a, hipStream_t st) {
  if constexpr (TILE == 32) {
    switch (a.S.lds_batch) {
      case 32: launch_backward<TILE, 32, 4, 2>(a, st); break;
      case 128: launch_backward<TILE, 128, 4, 2>(a, st); break;
      default: launch_backward<TILE, 64, 4, 2>(a, st); break;
    }
  }
}

template <int TILE>
void dispatch_px(const RasterArgs& a, hipStream_t st, bool backward) {
  switch (backward ? a.S.bwd_px_per_lane : a.S.px_per_lane) {
    case 2: dispatch_batch<TILE, 2, 1>(a, st, backward); break;
    case 4: dispatch_batch<TILE, 2, 2>(a, st, backward); break;
    case 8: dispatch_backward8<TILE>(a, st); break;
    default: dispatch_batch<TILE, 1, 1>(a, st, backward); break;
  }
}

void dispatch(const RasterArgs& a, hipStream_t st, bool backward) {
  if (a.n_ext > 0) {
    switch (a.S.tile) {
      case 8: dispatch_ext<8>(a, st, backward); break;
      case 32: dispatch_ext<32>(a, st, backward); break;
      default: dispatch_ext<16>(a, st, backward); break;
    }
    return;
  }
  switch (a.S.tile) {
    case 8: dispatch_batch<8, 1, 1>(a, st, backward); break;
    case 32: dispatch_px<32>(a, st, backward); break;
    default: dispatch_px<16>(a, st, backward); break;
  }
}

}  // namespace

void raster_forward(const RasterArgs& a, hipStream_t st) { dispatch(a, st, false); }
void raster_backward(const RasterArgs& a, hipStream_t st) { dispatch(a, st, true); }

}  // namespace g4d
