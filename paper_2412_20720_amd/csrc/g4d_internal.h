// Internal launchers shared by the runtime and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "g4d_device.h"

namespace g4d {

// Flags in the high bits of a listed slot's tile count: the color channel was held at
// color_min (its gradient is zero).
constexpr uint32_t kClampR = 1u << 29, kClampG = 1u << 30, kClampB = 1u << 31;
constexpr uint32_t kTileCountMask = (1u << 29) - 1u;

constexpr int kScanItems = 4096;  // items per workgroup in scans and radix-sort passes
constexpr int kSortThreads = 256;

// p[0..n) = v (a kernel, not a memset node, so that captured graphs replay it correctly).
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
// dst[0..n) = src[0..n) & mask.
void copy_masked_u32(uint32_t* dst, const uint32_t* src, int64_t n, uint32_t mask,
                     hipStream_t st);

// Scratch needed by scan_* for up to `n` items (bytes).
size_t scan_scratch_bytes(int64_t n);

// Sorts each view's listed slots by depth into (key, val) buffer 0 (the result's index,
// returned): (depth key, slot) grouped by view (slot / n_per_view, n_cap slots
// in all), each view's slots in ascending key order and slot order among equal keys, its range
// in vrange[v] = [first, end) and the count of all of them in *n_vis.  A stable LSD radix
// sort inside each view's segment, 8 bits per pass, four passes in workgroups of up to 4,096
// items of one view; each pass counts digits, scans each view's counts (a workgroup per view)
// and scatters.  The first pass reads dkey directly (workgroups of 4,096 slots of one view),
// taking the listed slots from the preprocess's masks per view and wave of 64 Gaussians
// (vmask[v * n_wc + wave] bit l: slot v * n_per_view + 64 wave + l is listed), so no
// compaction precedes it; the views' places come from the masks' counts.  Its first kernel (one workgroup)
// also adds up the preprocess's n_wsum per-wave pair and run counts wsum into totals[0]
// (pairs) and totals[2] (runs), each held at 2^32 - 1, and sets totals[4] = 1 if either
// reaches 2^31 (0 otherwise).  scratch: depth_sort_scratch_bytes(n_cap, n_views) bytes.
size_t depth_sort_scratch_bytes(int64_t n_cap, int n_views);
int depth_sort_by_view(const uint32_t* dkey, const uint64_t* vmask, int64_t n_wc, uint32_t* key[2], uint32_t* val[2], uint32_t* n_vis,
                       int64_t n_cap, int n_views, uint32_t n_per_view, uint2* vrange,
                       const uint2* wsum, int64_t n_wsum, uint32_t* totals, void* scratch,
                       hipStream_t st);

// The runs of every view's splats (vval grouped by view, depth order within a view), grouped
// by global tile row with each row's runs in depth order: runs = (slot, span) with span =
// (first column << 16) | last column, or ~0u for a row the ellipse misses; each row's range
// follows from the scanned count table (RowRuns).  chunk_cap >= visible / 64 + n_views and rhist_cap >=
// max_tiles_y * chunk_cap bound the chunk grid and the count table (max_tiles_y: the largest
// view's tile rows; the table's scan covers max_tiles_y * chunk_cap entries); rowbox = each slot's tile
// rows (first << 16 | last, ~0u: none); vinfo holds 2 n_views entries, cview chunk_cap; counts
// (3 words) receive the chunks, the table entries and the runs laid down.  Runs past row_cap
// are not written and set *flag = 1.
void splats_to_rows(const uint2* vrange, int n_views, const DView* views,
                    int64_t max_tiles_y, const uint32_t* vval, const uint32_t* rowbox,
                    const float* rec, DSettings S, int64_t chunk_cap, int64_t rhist_cap,
                    int64_t row_cap, uint4* vinfo, uint16_t* cview, uint32_t* rhist,
                    uint32_t* counts, uint2* runs, uint32_t* flag, void* scratch,
                    hipStream_t st);

// Where the runs of each tile row lie after splats_to_rows: its view table, the scanned count
// table, the device counts of table entries and runs laid down (its counts[1], counts[2]), the
// runs the preprocess counted, and the run capacity.
struct RowRuns {
  const uint4* vinfo;
  const uint32_t* scanned;
  const uint32_t* n_hist;
  const uint32_t* total;
  const uint32_t* n_runs;
  uint32_t row_cap;
};

// Expansion of the row-grouped runs into the tile lists: rr = where each tile row's runs lie
// (runs = their (slot, span); a run total past the run capacity sets *flag = 1, one other
// than the preprocess's count *flag = 2), pval = every tile's slots in depth order,
// ranges = [first, end) per tile ((0, 0) if empty).  chunk_cap >= runs / 64 + n_rows and
// hist_cap >= max_tiles_x * ceil(runs / 64) + n_tiles bound the chunk grid and the count
// table (max_tiles_x: the largest view's tile columns; the table's scan covers at most
// max_tiles_x * chunk_cap entries); rinfo holds 2 n_rows entries, crow 8 chunk_cap (a chunk list per XCD); counts (10
// words) receive the chunks of each XCD, the table entries and the pairs written.  A pair count
// other than *n_pairs sets *flag = 2 (unless set).
void expand(const RowRuns& rr, int n_rows, const DView* views, int n_views, int64_t n_tiles,
            int64_t max_tiles_x, const uint2* runs, int64_t chunk_cap, int64_t hist_cap,
            int64_t pair_cap,
            const uint32_t* n_pairs, uint4* rinfo,
            uint32_t* crow, uint32_t* hist, uint32_t* counts, uint32_t* pval, uint2* ranges,
            uint32_t* flag, void* scratch, hipStream_t st);

// ids[i] = the tile whose range holds pair i, for i < n.
void tile_ids_of(const uint2* ranges, int64_t n_tiles, int64_t n, uint32_t* ids, hipStream_t st);

// Derive camera centres and Jacobian clamps of the views on the device.
void view_setup(DView* views, int n_views, float jac_margin, hipStream_t st);

struct GaussPtrs {
  int n, sh_degree, t_degree;
  const float *mean4, *scale4, *rot_l, *rot_r, *opacity, *sh;
  const float* mask;      // optional volume mask (kept when mask > mask_thr)
  float mask_thr;
  const CompactPtrs* compact = nullptr;  // set: decode a compact model in the preprocess
};
struct GradPtrs {
  float *mean4, *scale4, *rot_l, *rot_r, *opacity, *sh;
  float *mask, *densify;  // optional: straight-through dL/dM; [N][3] densification statistics
};

// tiles[slot] = the slot's tile count (below 2^29: a tile has at least 64 pixels) with, for a
// listed slot, kClampR / G / B set where that color channel was held at color_min.
// Per wave of 64 Gaussians (n_wc = ceil(n / 256) * 4 of them), optional: wsum[wave] = the
// (Gaussian, tile) pairs and (Gaussian, tile row) runs it listed, each held at 2^31, and
// vmask[v * n_wc + wave] = the mask of its lanes whose Gaussian is listed in view v.
void preprocess_forward(const GaussPtrs& g, const DView* views, int n_views, DSettings S,
                        float* rec, uint32_t* tiles, uint32_t* rowbox, uint32_t* dkey,
                        uint2* wsum, uint64_t* vmask, hipStream_t st);
void decode_compact_params(int n, int sh_degree, int t_degree, const CompactPtrs& cp,
                           float* mean4, float* scale4, float* rot_l, float* rot_r,
                           float* opacity, float* sh, hipStream_t st);
// Adjoint of the preprocess: reads the forward's per-slot tile words (a nonzero word: the slot
// is listed; kClamp*: that color channel was held at color_min, its gradient is zero) and the
// screen-space gradient slots, writes every parameter gradient once and leaves the slots zero.
// A Gaussian listed in no view writes zero gradients.
void preprocess_backward(const GaussPtrs& g, const DView* views, int n_views, DSettings S,
                         const uint32_t* tiles, float* grad2d, const GradPtrs& out,
                         hipStream_t st);

struct RasterArgs {
  const float* rec;
  const uint32_t* pval;
  const uint2* ranges;
  const DView* views;
  const int32_t* tile_base;  // n_views + 1 prefix of tiles per view
  int n_views;
  int n_tiles;
  int blocks_per_xcd;        // set by the launcher
  DSettings S;
  float* out_rgb;
  float* out_T;
  float* px_T;
  int32_t* px_last;
  uint32_t* px_evals;        // optional per-pixel evaluation counter
  const float* dL;           // backward
  float* grad2d;             // backward
  // Extra channels (0 when none): E = n_feat + has_depth + 2 has_flow values per pixel, in
  // that order.  Features are read per Gaussian (fn, [n_gauss][n_feat], normalized), depth
  // from the record, flow from `flow` ([slots][2]).
  int n_ext, n_feat, has_depth, has_flow, n_gauss;
  const float* fn;
  const float* flow;
  float* out_ch;             // forward: per view [E][H][W]
  const float* dL_ch;        // backward: same layout (flow channels ignored)
  float* dfn;                // backward: dL/d(normalized features) [n_gauss][n_feat], atomics
  const float* bg_px;        // optional per-pixel background, the image's layout (the sky)
  uint32_t* clamp_batches;   // backward, optional: += 1 per staged batch that ran the entry
                             // loop with the alpha_max clamp (some entry's opacity p_t reaches it)
};

// Sky (k_sky.hip): per-pixel background from a cube map [6][R][R][3] queried by each pixel's
// ray, and the adjoint d_cube += bilinear transpose of T_final * dL/dI.
void sky_forward(const DView* views, int n_views, int max_pixels, const float* cube, int R,
                 float* bg, hipStream_t st);
void sky_backward(const DView* views, int n_views, int max_width, int max_height, int R,
                  const float* px_T, const float* dL, float* d_cube, hipStream_t st);

// Extra-channel helpers (k_channels.hip).
void feature_normalize(int n, int d, const float* f, const float* gate, float* fn, float* fnorm,
                       hipStream_t st);
void flow_forward(const GaussPtrs& g, const DView* views, int n_views, const uint32_t* tiles,
                  float dt, float* flow, hipStream_t st);
void feature_backward(int n, int d, const float* f, const float* gate, const float* fn,
                      const float* fnorm, const float* dfn, float* d_features, float* d_gate,
                      hipStream_t st);

void raster_forward(const RasterArgs& a, hipStream_t st);
void raster_backward(const RasterArgs& a, hipStream_t st);

}  // namespace g4d
