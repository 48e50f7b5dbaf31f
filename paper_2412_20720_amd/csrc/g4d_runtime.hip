// Host runtime behind the C ABI of include/g4d.h: argument checks, per-batch planning (tile
// grids and pixel offsets of every view), device scratch management and the launch sequence
//   view setup -> preprocess -> depth sort per view -> splats to tile-row runs -> runs to
//   tile lists and ranges -> raster                  (forward)
//   raster backward -> preprocess backward           (backward)
// All arithmetic of the render happens in the kernels; the host only does integer planning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/g4d.h"
#include "g4d_checks.h"
#include "g4d_internal.h"

using namespace g4d;

// Device scratch of g4d_render_step_noalloc: one fixed array on every GPU the library runs on,
// reserved when the code object is loaded and held until the process ends.  Host code never
// uses the name itself (on the host it is a stand-in, not a device address): g4d_create looks
// up each device's address once with hipGetSymbolAddress and the entry point passes slices of
// that address to the kernels.
static __device__ __align__(256) unsigned char scratch[G4D_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_looked_up[kMaxScratchDevices] = {};
void* g_scratch_ptr[kMaxScratchDevices] = {};  // device address of `scratch` per GPU
hipError_t g_scratch_err[kMaxScratchDevices] = {};

// Once per device, with that device current.
void lookup_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_looked_up[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) (void)hipGetLastError();
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
  g_scratch_looked_up[device] = true;
}

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct SavedKey {
  int32_t n = -1, sh_degree = 0, t_degree = 0, n_views = 0;
  const void* ptrs[6] = {};
  const float* mask = nullptr;
  float mask_thr = 0.f;
  std::vector<g4d_view> views;
  g4d_settings s{};
  g4d_channels ch{};  // n_features = depth = flow = 0 for a plain forward
  const float* sky_cube = nullptr;
  int32_t sky_res = 0;
};

}  // namespace

struct g4d_ctx {
  int device = 0;
  std::string err;
  DevBuf views, tile_base, rec, tiles, rowbox, dkey, wsum, vmask, vk[2], vv[2], vrange, vinfo, cview,
      rhist, runs, rinfo, crow, hist, pval, scan_tmp, sort_tmp, ranges, px_T, px_last,
      px_evals, grad2d, counters;
  DevBuf fn, fnorm, flow, dfn;     // extra channels
  DevBuf skybg;                    // per-pixel sky background
  uint32_t* h_counters = nullptr;  // pinned: visible, pairs, flag, runs, -, 2^31 reached
  DView* h_views = nullptr;        // pinned staging
  int32_t* h_tile_base = nullptr;  // pinned staging
  hipEvent_t staging_done = nullptr;
  hipEvent_t counts_ready = nullptr;  // the forward's visible and pair counts reached the host
  bool staging_pending = false;
  // the view table now on the device (skips the upload when a call repeats it)
  std::vector<DView> uploaded_views;
  void* uploaded_to = nullptr;
  // capacities of the pair list, the run list and the two expansions' count tables
  int64_t pair_cap = 0, row_cap = 0, hist_cap = 0, rhist_cap = 0;
  // the whole grad2d allocation holds zeros: the last backward ran to its preprocess adjoint,
  // which zeroes every slot the raster adjoint accumulated into (false after a reallocation or
  // an interrupted backward; the next backward then clears the whole allocation)
  bool grad2d_zero = false;
  // state left by the last forward
  bool saved = false;
  SavedKey key;
  int vis_buf = 0;
  int64_t n_tiles = 0, n_pixels = 0;
  int64_t n_rows = 0, max_tiles_x = 0, max_tiles_y = 0;  // tile rows of the batch, largest view
  int64_t last_runs = 0;                 // row runs of the last eager forward
  g4d_stats stats{};
  bool count_evals = false;
  bool count_cutoff = false;   // counting forwards bin by the plain cutoff (g4d_eval_counters 2)
  bool fwd_cutoff_bins = false;  // the last forward binned by the plain cutoff
  bool counted_bwd = false;  // the last backward counted its clamped batches (counters[4])
  // stage profiling (stages whose bit is set in stage_mask)
  bool profiling = false;
  uint32_t stage_mask = 0xFFFFFFFFu;
  std::vector<hipEvent_t> ev_free;
  struct Interval { int stage; hipEvent_t a, b; };
  std::vector<Interval> pending;
  double stage_ms[G4D_NUM_STAGES] = {};
  int64_t stage_n[G4D_NUM_STAGES] = {};
  // autotuner cache: problem shape -> (tile, lds batch, pixels per lane, ms)
  struct Tuned { int tile, batch, px, bwd_px; double ms; };
  std::map<std::string, Tuned> tuned;
  // graph mode: while `capturing`, no host synchronization, allocation or upload happens and
  // grids are sized from the capacities found by an earlier eager pass
  bool capturing = false;
  g4d_ctx* graph_ctx = nullptr;    // private context whose buffers the captured graph uses
  // g4d_render_step_noalloc: `na` is a private context whose buffers are slices of the fixed
  // per-device scratch array (`arena`: its buffers are never allocated, grown or freed)
  g4d_ctx* na = nullptr;
  bool arena = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<unsigned char> graph_key;
};

namespace {

g4d_status fail(g4d_ctx* c, g4d_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define G4D_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, G4D_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

g4d_status ensure(g4d_ctx* ctx, DevBuf& b, size_t bytes, double grow = 1.0) {
  if (bytes == 0) bytes = 256;
  if (bytes <= b.cap) return G4D_OK;
  if (ctx->capturing) return fail(ctx, G4D_ECAPACITY, "buffer too small during graph capture");
  if (ctx->arena)
    return fail(ctx, G4D_ECAPACITY, "%zu bytes needed where the fixed scratch left %zu", bytes,
                b.cap);
  const size_t want = std::max(bytes, (size_t)((double)bytes * grow));
  if (b.p) {
    G4D_HIP(hipDeviceSynchronize());
    G4D_HIP(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(ctx, G4D_ENOMEM, "hipMalloc of %zu bytes failed", want);
  }
  b.cap = want;
  return G4D_OK;
}

const char* const kStageNames[G4D_NUM_STAGES] = {
    "preprocess", "depth_sort", "splat_rows", "row_tiles", "raster_fwd", "clear_grad",
    "raster_bwd", "preprocess_bwd"};

hipEvent_t take_event(g4d_ctx* c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

// Records a HIP event pair around one kernel group on the call's stream when profiling.
struct Stage {
  g4d_ctx* c;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Stage(g4d_ctx* c_, int s_, hipStream_t st_) : c(c_), stage(s_), st(st_) {
    if (c->profiling && !c->capturing && ((c->stage_mask >> s_) & 1u) && (a = take_event(c)))
      (void)hipEventRecord(a, st);
  }
  ~Stage() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) {
      c->ev_free.push_back(a);
      return;
    }
    (void)hipEventRecord(b, st);
    c->pending.push_back({stage, a, b});
  }
};

template <class T>
T* P(DevBuf& b) {
  return static_cast<T*>(b.p);
}

// The host-side argument checks (g4d_checks.cpp), with the message kept in the context.
g4d_status check_common(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                        int32_t n_views, const g4d_settings* s, bool params = true) {
  if (!ctx) return G4D_EINVAL;
  char msg[512];
  const g4d_status r = check_args(g, views, n_views, s, params, msg, sizeof msg);
  if (r != G4D_OK) ctx->err = msg;
  return r;
}

int max_view_pixels(const g4d_view* views, int n_views) {
  int64_t m = 0;
  for (int v = 0; v < n_views; ++v) m = std::max(m, (int64_t)views[v].width * views[v].height);
  return (int)m;
}

g4d_status check_channels(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_channels* ch) {
  char msg[512];
  const g4d_status r = check_channels_args(g, ch, msg, sizeof msg);
  if (r != G4D_OK) ctx->err = msg;
  return r;
}

bool same_channels(const g4d_channels& a, const g4d_channels& b) {
  return a.n_features == b.n_features && a.features == b.features && a.gate == b.gate &&
         a.depth == b.depth && a.flow == b.flow &&
         (!a.flow || std::memcmp(&a.flow_dt, &b.flow_dt, sizeof(float)) == 0);
}

// Settings the raster runs with.  The extra-channel raster takes 64-entry LDS batches and at
// most two pixels per lane: its per-pixel channel registers leave one wave per SIMD at four
// (measured slower on the 300k/16-view workload with 35 channels: 31.8 against 26.7 ms per
// forward + backward step at two, 33.5 at one).
g4d_settings run_settings(const g4d_settings* s, const g4d_channels* ch) {
  g4d_settings r = *s;
  if (ch) {
    r.lds_batch = 64;
    r.px_per_lane = r.tile_size == 8 ? 1 : (r.px_per_lane == 1 ? 1 : 2);
    r.bwd_px_per_lane = r.px_per_lane;
  }
  return r;
}

DSettings device_settings(const g4d_settings* s, bool cutoff_bins = false) {
  DSettings d{};
  d.cutoff_bins = cutoff_bins ? 1 : 0;
  d.near_z = s->near_z;
  d.marginal_min = s->marginal_min;
  d.cutoff = s->cutoff_sigma;
  d.cut2 = s->cutoff_sigma * s->cutoff_sigma;
  d.blur = s->blur;
  d.jac_margin = s->jacobian_margin;
  d.alpha_min = s->alpha_min;
  d.alpha_max = s->alpha_max;
  d.T_min = s->T_min;
  d.color_offset = s->color_offset;
  d.color_min = s->color_min;
  d.time_period = s->time_period;
  d.tile = s->tile_size;
  d.tile_shift = s->tile_size == 8 ? 3 : (s->tile_size == 16 ? 4 : 5);
  d.lds_batch = s->lds_batch == 0 ? 64 : s->lds_batch;
  d.px_per_lane = s->px_per_lane == 0 ? (s->tile_size == 8 ? 1 : 4) : s->px_per_lane;
  // The backward's default: 32x16 blocks where the forward takes 16x16 ones at 32-pixel
  // tiles.  It amortizes the per-entry wave reduction and atomic over twice the pixels
  // (measured on the 300k/16-view workload: raster_bwd 2.36 -> 2.16 ms; the forward, with no
  // per-entry reduction, is slower at 8: 1.04 -> 1.17 ms).
  d.bwd_px_per_lane = s->bwd_px_per_lane != 0
                          ? s->bwd_px_per_lane
                          : (s->tile_size == 32 && d.px_per_lane == 4 ? 8 : d.px_per_lane);
  return d;
}

GaussPtrs gauss_ptrs(const g4d_gaussians* g) {
  return GaussPtrs{g->n,       g->sh_degree, g->t_degree, g->mean4, g->scale4, g->rot_l,
                   g->rot_r,   g->opacity,   g->sh,       g->mask,  g->mask_threshold};
}

// The run list for `runs` row runs, the pair list for `pairs` pairs, and the tile expansion's
// chunk maps, count table and scan scratch that the run capacity implies (each capacity
// becomes what was allocated; `grow` adds headroom to what has to grow).
g4d_status size_binning(g4d_ctx* ctx, int64_t slots, int64_t runs, int64_t pairs, double grow) {
  g4d_status r;
  if (runs > ctx->row_cap) {
    if ((r = ensure(ctx, ctx->runs, sizeof(uint2) * (size_t)runs, grow)) != G4D_OK) return r;
    ctx->row_cap = std::min<int64_t>((int64_t)(ctx->runs.cap / sizeof(uint2)), INT32_MAX);
  }
  if (pairs > ctx->pair_cap) {
    if ((r = ensure(ctx, ctx->pval, sizeof(uint32_t) * (size_t)pairs, grow)) != G4D_OK) return r;
    ctx->pair_cap = std::min<int64_t>((int64_t)(ctx->pval.cap / sizeof(uint32_t)), INT32_MAX);
  }
  // a row of len runs has ceil(len / 64) chunks, each with one entry per column
  const int64_t chunk_need = (ctx->row_cap + 63) / 64 + ctx->n_rows;
  if ((r = ensure(ctx, ctx->crow, 8 * sizeof(uint32_t) * (size_t)chunk_need, grow)) != G4D_OK)
    return r;
  const int64_t hist_need = ctx->max_tiles_x * ((ctx->row_cap + 63) / 64) + ctx->n_tiles;
  if (hist_need > ctx->hist_cap) {
    if ((r = ensure(ctx, ctx->hist, sizeof(uint32_t) * (size_t)hist_need, grow)) != G4D_OK) return r;
    ctx->hist_cap = (int64_t)(ctx->hist.cap / sizeof(uint32_t));
  }
  return ensure(ctx, ctx->scan_tmp,
                scan_scratch_bytes(std::max({ctx->hist_cap, ctx->rhist_cap, slots})), grow);
}

// Plan tile grids and offsets, upload the view table and derive per-view constants.
g4d_status upload_views(g4d_ctx* ctx, const g4d_view* views, int n_views, const g4d_settings* s,
                        hipStream_t st) {
  if (ctx->staging_pending && !ctx->capturing) {
    G4D_HIP(hipEventSynchronize(ctx->staging_done));
    ctx->staging_pending = false;
  }
  const int T = s->tile_size;
  int64_t tile_base = 0, pix_base = 0, row_base = 0, max_tx = 0, max_ty = 0;
  for (int v = 0; v < n_views; ++v) {
    const g4d_view& in = views[v];
    DView& d = ctx->h_views[v];
    std::memset(&d, 0, sizeof d);
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) d.W[3 * r + c] = in.world_to_cam[4 * r + c];
      d.tau[r] = in.world_to_cam[4 * r + 3];
    }
    d.fx = in.fx;
    d.fy = in.fy;
    d.cx = in.cx;
    d.cy = in.cy;
    d.t = in.t;
    for (int c = 0; c < 3; ++c) d.bg[c] = in.background[c];
    d.width = in.width;
    d.height = in.height;
    d.tiles_x = (in.width + T - 1) / T;
    d.tiles_y = (in.height + T - 1) / T;
    d.tile_base = (int32_t)tile_base;
    d.pix_base = (int32_t)pix_base;
    d.row_base = (int32_t)row_base;
    std::memcpy(&d.pad0, &s->jacobian_margin, sizeof(float));  // part of the upload key
    ctx->h_tile_base[v] = (int32_t)tile_base;
    tile_base += (int64_t)d.tiles_x * d.tiles_y;
    row_base += d.tiles_y;
    max_tx = std::max<int64_t>(max_tx, d.tiles_x);
    max_ty = std::max<int64_t>(max_ty, d.tiles_y);
    pix_base += (int64_t)in.width * in.height;
    if (pix_base > INT32_MAX || tile_base > INT32_MAX)
      return fail(ctx, G4D_EINVAL, "total pixels of the batch exceed 2^31-1");
  }
  ctx->h_tile_base[n_views] = (int32_t)tile_base;
  ctx->n_tiles = tile_base;
  ctx->n_pixels = pix_base;
  ctx->n_rows = row_base;
  ctx->max_tiles_x = max_tx;
  ctx->max_tiles_y = max_ty;
  if (ctx->capturing) return G4D_OK;  // the view table was uploaded before the capture
  g4d_status r;
  if ((r = ensure(ctx, ctx->views, sizeof(DView) * n_views)) != G4D_OK) return r;
  if ((r = ensure(ctx, ctx->tile_base, sizeof(int32_t) * (n_views + 1))) != G4D_OK) return r;
  if (ctx->uploaded_to == ctx->views.p && (int)ctx->uploaded_views.size() == n_views &&
      std::memcmp(ctx->uploaded_views.data(), ctx->h_views, sizeof(DView) * n_views) == 0)
    return G4D_OK;  // same table (and the same jacobian margin, folded into the key below)
  ctx->uploaded_views.assign(ctx->h_views, ctx->h_views + n_views);
  ctx->uploaded_to = ctx->views.p;
  G4D_HIP(hipMemcpyAsync(ctx->views.p, ctx->h_views, sizeof(DView) * n_views,
                         hipMemcpyHostToDevice, st));
  G4D_HIP(hipMemcpyAsync(ctx->tile_base.p, ctx->h_tile_base, sizeof(int32_t) * (n_views + 1),
                         hipMemcpyHostToDevice, st));
  G4D_HIP(hipEventRecord(ctx->staging_done, st));
  ctx->staging_pending = true;
  view_setup(P<DView>(ctx->views), n_views, s->jacobian_margin, st);
  G4D_HIP(hipGetLastError());
  return G4D_OK;
}

g4d_status run_preprocess(g4d_ctx* ctx, const g4d_gaussians* g, int n_views,
                          const g4d_settings* s, hipStream_t st, bool zero_records = false,
                          const CompactPtrs* cp = nullptr, uint2* wsum = nullptr,
                          uint64_t* vmask = nullptr) {
  const int64_t slots = (int64_t)g->n * n_views;
  g4d_status r;
  if ((r = ensure(ctx, ctx->rec, sizeof(float) * kRec * slots, 1.1)) != G4D_OK) return r;
  // a fill kernel rather than a memset, so that a captured graph replays the clear correctly
  if (zero_records) fill_u32(P<uint32_t>(ctx->rec), (int64_t)kRec * slots, 0u, st);
  if ((r = ensure(ctx, ctx->tiles, sizeof(uint32_t) * slots, 1.1)) != G4D_OK) return r;
  if ((r = ensure(ctx, ctx->rowbox, sizeof(uint32_t) * slots, 1.1)) != G4D_OK) return r;
  if ((r = ensure(ctx, ctx->dkey, sizeof(uint32_t) * slots, 1.1)) != G4D_OK) return r;
  {
    Stage t(ctx, 0, st);
    GaussPtrs gp = gauss_ptrs(g);
    gp.compact = cp;
    preprocess_forward(gp, P<DView>(ctx->views), n_views,
                       device_settings(s, ctx->count_evals && ctx->count_cutoff),
                       P<float>(ctx->rec), P<uint32_t>(ctx->tiles), P<uint32_t>(ctx->rowbox),
                       P<uint32_t>(ctx->dkey), wsum, vmask, st);
  }
  G4D_HIP(hipGetLastError());
  return G4D_OK;
}

bool same_key(const SavedKey& k, const g4d_gaussians* g, const g4d_view* views, int n_views,
              const g4d_settings* s) {
  if (k.n != g->n || k.sh_degree != g->sh_degree || k.t_degree != g->t_degree ||
      k.n_views != n_views)
    return false;
  const void* p[6] = {g->mean4, g->scale4, g->rot_l, g->rot_r, g->opacity, g->sh};
  for (int i = 0; i < 6; ++i)
    if (p[i] != k.ptrs[i]) return false;
  if (g->mask != k.mask ||
      (g->mask && std::memcmp(&g->mask_threshold, &k.mask_thr, sizeof(float)) != 0))
    return false;
  if (std::memcmp(k.views.data(), views, sizeof(g4d_view) * n_views) != 0) return false;
  return std::memcmp(&k.s, s, sizeof(g4d_settings)) == 0;
}

int bits_for(int64_t n) {
  int b = 0;
  while (b < 32 && ((int64_t)1 << b) < n) ++b;
  return b;
}

}  // namespace

extern "C" {

g4d_status g4d_default_settings(g4d_settings* s) {
  if (!s) return G4D_EINVAL;
  s->near_z = 0.2f;
  s->marginal_min = 1.f / 255.f;
  s->cutoff_sigma = 3.f;
  s->blur = 0.3f;
  s->jacobian_margin = 0.15f;
  s->alpha_min = 1.f / 255.f;
  s->alpha_max = 0.99f;
  s->T_min = 1e-4f;
  s->color_offset = 0.5f;
  s->color_min = 0.f;
  s->time_period = 1.f;
  s->tile_size = 16;
  s->lds_batch = 0;
  s->px_per_lane = 0;
  s->bwd_px_per_lane = 0;
  return G4D_OK;
}

// A context with its pinned staging buffers and events; device memory comes later.
static g4d_status new_context(g4d_ctx** out, int device) {
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return G4D_EHIP;
  }
  g4d_ctx* ctx = new g4d_ctx;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void**)&ctx->h_counters, 8 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&ctx->h_views, sizeof(DView) * G4D_MAX_VIEWS, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&ctx->h_tile_base, sizeof(int32_t) * (G4D_MAX_VIEWS + 1), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->staging_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->counts_ready, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    g4d_destroy(ctx);
    return G4D_EHIP;
  }
  *out = ctx;
  return G4D_OK;
}

g4d_status g4d_create(g4d_ctx** out, int device) {
  if (!out) return G4D_EINVAL;
  *out = nullptr;
  g4d_ctx* ctx = nullptr;
  g4d_status r = new_context(&ctx, device);
  if (r != G4D_OK) return r;
  // Set-up of g4d_render_step_noalloc (new_context left `device` current): the address of the
  // device's fixed scratch array, and a private context whose buffers will be slices of it.
  lookup_scratch(device);
  g4d_ctx* na = nullptr;
  if ((r = new_context(&na, device)) != G4D_OK) {
    g4d_destroy(ctx);
    return r;
  }
  na->arena = true;
  // host-side storage the call fills, reserved here so that the call allocates nothing
  na->uploaded_views.reserve(G4D_MAX_VIEWS);
  na->key.views.reserve(G4D_MAX_VIEWS);
  na->err.reserve(512);
  ctx->err.reserve(512);
  ctx->na = na;
  *out = ctx;
  return G4D_OK;
}

g4d_status g4d_destroy(g4d_ctx* ctx) {
  if (!ctx) return G4D_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->graph_ctx) g4d_destroy(ctx->graph_ctx);
  if (ctx->na) g4d_destroy(ctx->na);
  DevBuf* bufs[] = {&ctx->views, &ctx->tile_base, &ctx->rec, &ctx->tiles, &ctx->rowbox, &ctx->dkey,
                    &ctx->wsum, &ctx->vmask,
                    &ctx->vk[0], &ctx->vk[1], &ctx->vv[0], &ctx->vv[1], &ctx->vrange,
                    &ctx->vinfo, &ctx->cview, &ctx->rhist, &ctx->runs,
                    &ctx->rinfo, &ctx->crow, &ctx->hist, &ctx->pval,
                    &ctx->scan_tmp,
                    &ctx->sort_tmp, &ctx->ranges, &ctx->px_T, &ctx->px_last, &ctx->px_evals,
                    &ctx->grad2d, &ctx->counters, &ctx->fn, &ctx->fnorm, &ctx->flow,
                    &ctx->dfn, &ctx->skybg};
  for (DevBuf* b : bufs)
    if (b->p && !ctx->arena) (void)hipFree(b->p);  // an arena's buffers are scratch slices
  if (ctx->h_counters) (void)hipHostFree(ctx->h_counters);
  if (ctx->h_views) (void)hipHostFree(ctx->h_views);
  if (ctx->h_tile_base) (void)hipHostFree(ctx->h_tile_base);
  if (ctx->staging_done) (void)hipEventDestroy(ctx->staging_done);
  if (ctx->counts_ready) (void)hipEventDestroy(ctx->counts_ready);
  for (auto& iv : ctx->pending) {
    (void)hipEventDestroy(iv.a);
    (void)hipEventDestroy(iv.b);
  }
  for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
  delete ctx;
  return G4D_OK;
}

const char* g4d_last_error(const g4d_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

g4d_status g4d_preprocess(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                          int32_t n_views, const g4d_settings* s, float* records, int32_t* tiles,
                          void* stream) {
  g4d_status r = check_common(ctx, g, views, n_views, s);
  if (r != G4D_OK) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  G4D_HIP(hipSetDevice(ctx->device));
  if ((r = upload_views(ctx, views, n_views, s, st)) != G4D_OK) return r;
  const int64_t slots = (int64_t)g->n * n_views;
  if (slots == 0) return G4D_OK;
  ctx->saved = false;  // the scratch records are overwritten
  // The kernel writes visible slots only, so clearing the scratch first leaves culled rows 0.
  if ((r = run_preprocess(ctx, g, n_views, s, st, records != nullptr)) != G4D_OK) return r;
  if (records)
    G4D_HIP(hipMemcpyAsync(records, ctx->rec.p, sizeof(float) * kRec * slots,
                           hipMemcpyDeviceToDevice, st));
  if (tiles)  // the counts without the clamp flags the backward reads
    copy_masked_u32(reinterpret_cast<uint32_t*>(tiles), P<uint32_t>(ctx->tiles), slots,
                    kTileCountMask, st);
  return G4D_OK;
}

// Forward of the whole batch; with ch, also the extra channels into out_ch.
static g4d_status forward_impl(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                               int32_t n_views, const g4d_settings* s, const g4d_channels* ch,
                               const g4d_sky* sky, float* out_rgb, float* out_T, float* out_ch,
                               void* stream, const CompactPtrs* cp = nullptr) {
  g4d_status r = check_common(ctx, g, views, n_views, s, cp == nullptr);
  if (r != G4D_OK) return r;
  if (!out_rgb) return fail(ctx, G4D_EINVAL, "null out_rgb");
  if (sky && (!sky->cube || sky->resolution < 1 || sky->resolution > G4D_MAX_SKY_RES))
    return fail(ctx, G4D_EINVAL, "sky needs a cube map and 1 <= resolution <= %d",
                G4D_MAX_SKY_RES);
  if (ch) {
    if ((r = check_channels(ctx, g, ch)) != G4D_OK) return r;
    if (!out_ch) return fail(ctx, G4D_EINVAL, "null out_ch");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  G4D_HIP(hipSetDevice(ctx->device));
  ctx->saved = false;
  if ((r = upload_views(ctx, views, n_views, s, st)) != G4D_OK) return r;
  const int64_t slots = (int64_t)g->n * n_views;
  const g4d_settings s_run = run_settings(s, ch);
  ctx->fwd_cutoff_bins = ctx->count_evals && ctx->count_cutoff;
  const DSettings DS = device_settings(&s_run, ctx->fwd_cutoff_bins);
  const int n_ext = n_ext_of(ch);
  if ((r = ensure(ctx, ctx->counters, 32 * sizeof(uint32_t))) != G4D_OK) return r;
  // [0] visible, [1] pairs the preprocess counted, [2] overflow / mismatch flag, [3] runs the
  // preprocess counted, [4] clamped batches of the last counted backward, [5] pairs or runs
  // reached 2^31, [6..15] the tile
  // expansion's chunks per XCD, table entries and pairs written, [16..18] the row expansion's
  // chunks, table entries and runs written
  uint32_t* cnt = P<uint32_t>(ctx->counters);
  ctx->counted_bwd = false;
  fill_u32(cnt, 6, 0u, st);
  if ((r = ensure(ctx, ctx->px_T, sizeof(float) * ctx->n_pixels, 1.1)) != G4D_OK) return r;
  if ((r = ensure(ctx, ctx->px_last, sizeof(int32_t) * ctx->n_pixels, 1.1)) != G4D_OK) return r;
  if ((r = ensure(ctx, ctx->ranges, sizeof(uint2) * ctx->n_tiles, 1.1)) != G4D_OK) return r;
  if ((r = ensure(ctx, ctx->rinfo, 2 * sizeof(uint4) * ctx->n_rows, 1.1)) != G4D_OK) return r;
  if (ctx->count_evals &&
      (r = ensure(ctx, ctx->px_evals, sizeof(uint32_t) * ctx->n_pixels, 1.1)) != G4D_OK)
    return r;

  int64_t n_vis = 0, n_pairs = 0, run_grid = 0;
  if (slots > 0) {
    const int64_t n_wc = ((int64_t)g->n + 255) / 256 * 4;  // waves of the preprocess
    if ((r = ensure(ctx, ctx->wsum, sizeof(uint2) * n_wc, 1.1)) != G4D_OK) return r;
    if ((r = ensure(ctx, ctx->vmask, sizeof(uint64_t) * n_wc * n_views, 1.1)) != G4D_OK) return r;
    if ((r = run_preprocess(ctx, g, n_views, &s_run, st, false, cp, P<uint2>(ctx->wsum),
                            P<uint64_t>(ctx->vmask))) != G4D_OK)
      return r;
    if (ch && ch->n_features > 0) {
      if ((r = ensure(ctx, ctx->fn, sizeof(float) * (size_t)g->n * ch->n_features, 1.1)) != G4D_OK)
        return r;
      if ((r = ensure(ctx, ctx->fnorm, sizeof(float) * (size_t)g->n, 1.1)) != G4D_OK) return r;
      feature_normalize(g->n, ch->n_features, ch->features, ch->gate, P<float>(ctx->fn),
                        P<float>(ctx->fnorm), st);
    }
    if (ch && ch->flow) {
      if ((r = ensure(ctx, ctx->flow, sizeof(float) * 2 * slots, 1.1)) != G4D_OK) return r;
      flow_forward(gauss_ptrs(g), P<DView>(ctx->views), n_views, P<uint32_t>(ctx->tiles),
                   ch->flow_dt, P<float>(ctx->flow), st);
    }
    for (int b = 0; b < 2; ++b) {
      if ((r = ensure(ctx, ctx->vk[b], sizeof(uint32_t) * slots, 1.1)) != G4D_OK) return r;
      if ((r = ensure(ctx, ctx->vv[b], sizeof(uint32_t) * slots, 1.1)) != G4D_OK) return r;
    }
    // the row expansion's count table: a row of the view per chunk of 64 visible slots
    const int64_t row_chunks = (slots + 63) / 64 + n_views;
    if ((r = ensure(ctx, ctx->rhist, sizeof(uint32_t) * (size_t)(ctx->max_tiles_y * row_chunks),
                    1.1)) != G4D_OK)
      return r;
    ctx->rhist_cap = (int64_t)(ctx->rhist.cap / sizeof(uint32_t));
    if ((r = ensure(ctx, ctx->vrange, sizeof(uint2) * n_views)) != G4D_OK) return r;
    if ((r = ensure(ctx, ctx->vinfo, 2 * sizeof(uint4) * n_views)) != G4D_OK) return r;
    if ((r = ensure(ctx, ctx->cview, sizeof(uint16_t) * row_chunks, 1.1)) != G4D_OK) return r;
    if ((r = ensure(ctx, ctx->scan_tmp, scan_scratch_bytes(std::max(slots, ctx->rhist_cap)),
                    1.1)) != G4D_OK)
      return r;
    if ((r = ensure(ctx, ctx->sort_tmp, depth_sort_scratch_bytes(slots, n_views), 1.1)) != G4D_OK)
      return r;
    uint32_t* vk[2] = {P<uint32_t>(ctx->vk[0]), P<uint32_t>(ctx->vk[1])};
    uint32_t* vv[2] = {P<uint32_t>(ctx->vv[0]), P<uint32_t>(ctx->vv[1])};
    int vb;
    {
      Stage t(ctx, 1, st);
      vb = depth_sort_by_view(P<uint32_t>(ctx->dkey), P<uint64_t>(ctx->vmask), n_wc, vk, vv,
                              cnt + 0, slots, n_views,
                              (uint32_t)g->n, P<uint2>(ctx->vrange), P<uint2>(ctx->wsum), n_wc,
                              cnt + 1, ctx->sort_tmp.p, st);
    }
    ctx->vis_buf = vb;
    G4D_HIP(hipGetLastError());
    auto run_rows = [&]() {
      Stage t(ctx, 2, st);
      splats_to_rows(P<uint2>(ctx->vrange), n_views, P<DView>(ctx->views), ctx->max_tiles_y,
                     vv[vb], P<uint32_t>(ctx->rowbox), P<float>(ctx->rec), DS, row_chunks,
                     ctx->rhist_cap, ctx->row_cap, P<uint4>(ctx->vinfo),
                     P<uint16_t>(ctx->cview), P<uint32_t>(ctx->rhist), cnt + 16,
                     P<uint2>(ctx->runs), cnt + 2, ctx->scan_tmp.p, st);
    };
    if (ctx->capturing) {
      // counts stay on the device; grids cover the capacities
      n_pairs = ctx->pair_cap;
      run_grid = ctx->row_cap;
      if (run_grid > 0) run_rows();
    } else {
      // The counts go to the host; with a run list from an earlier call the row expansion is
      // queued behind the copy at once (writes clamped to the capacity), so that the GPU does
      // not idle while the host reads the counts.  Should the runs exceed that capacity, the
      // list grows and the row expansion runs again.
      const bool early = ctx->row_cap > 0;
      G4D_HIP(hipMemcpyAsync(ctx->h_counters, cnt, 6 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      G4D_HIP(hipEventRecord(ctx->counts_ready, st));
      if (early) run_rows();
      G4D_HIP(hipEventSynchronize(ctx->counts_ready));
      n_vis = ctx->h_counters[0];
      n_pairs = ctx->h_counters[1];
      const int64_t n_runs = ctx->h_counters[3];
      // list positions are 32-bit signed in the raster kernels
      if (ctx->h_counters[5] || n_pairs > (int64_t)INT32_MAX || n_runs > (int64_t)INT32_MAX)
        return fail(ctx, G4D_ECAPACITY, "the (Gaussian, tile) pairs or row runs exceed 2^31-1");
      if (ctx->arena && (n_pairs > ctx->pair_cap || n_runs > ctx->row_cap))
        return fail(ctx, G4D_ECAPACITY,
                    "%lld (Gaussian, tile) pairs in %lld row runs exceed the %lld pairs and %lld "
                    "runs the fixed scratch leaves room for",
                    (long long)n_pairs, (long long)n_runs, (long long)ctx->pair_cap,
                    (long long)ctx->row_cap);
      const bool fits = early && n_runs <= ctx->row_cap;
      if ((r = size_binning(ctx, slots, n_runs, n_pairs, 1.2)) != G4D_OK) return r;
      if (n_runs > 0 && !fits) {
        if (early) fill_u32(cnt + 2, 1, 0u, st);  // the early pass flagged the overflow
        run_rows();
      }
      run_grid = n_runs;
      ctx->last_runs = n_runs;
    }
    if (run_grid > 0) {
      {
        Stage t(ctx, 3, st);
        const RowRuns rr{P<uint4>(ctx->vinfo), P<uint32_t>(ctx->rhist), cnt + 17, cnt + 18,
                         cnt + 3, (uint32_t)std::min<int64_t>(ctx->row_cap, UINT32_MAX)};
        expand(rr, (int)ctx->n_rows, P<DView>(ctx->views), n_views,
               ctx->n_tiles, ctx->max_tiles_x, P<uint2>(ctx->runs), (run_grid + 63) / 64 + ctx->n_rows,
               ctx->hist_cap, ctx->pair_cap, cnt + 1, P<uint4>(ctx->rinfo), P<uint32_t>(ctx->crow),
               P<uint32_t>(ctx->hist), cnt + 6, P<uint32_t>(ctx->pval), P<uint2>(ctx->ranges),
               cnt + 2, ctx->scan_tmp.p, st);
      }
      G4D_HIP(hipGetLastError());
    }
  }
  if (run_grid <= 0) {
    Stage t(ctx, 3, st);
    fill_u32(P<uint32_t>(ctx->ranges), 2 * ctx->n_tiles, 0u, st);
  }
  if (sky) {
    if ((r = ensure(ctx, ctx->skybg, sizeof(float) * 3 * ctx->n_pixels, 1.1)) != G4D_OK) return r;
    sky_forward(P<DView>(ctx->views), n_views, max_view_pixels(views, n_views), sky->cube,
                sky->resolution, P<float>(ctx->skybg), st);
  }
  RasterArgs a{};
  a.bg_px = sky ? P<float>(ctx->skybg) : nullptr;
  a.rec = P<float>(ctx->rec);
  a.pval = n_pairs > 0 ? P<uint32_t>(ctx->pval) : nullptr;
  a.ranges = P<uint2>(ctx->ranges);
  a.views = P<DView>(ctx->views);
  a.tile_base = P<int32_t>(ctx->tile_base);
  a.n_views = n_views;
  a.n_tiles = (int)ctx->n_tiles;
  a.S = DS;
  a.out_rgb = out_rgb;
  a.out_T = out_T;
  a.px_T = P<float>(ctx->px_T);
  a.px_last = P<int32_t>(ctx->px_last);
  a.px_evals = (ctx->count_evals && !ch) ? P<uint32_t>(ctx->px_evals) : nullptr;
  if (ch) {
    a.n_ext = n_ext;
    a.n_feat = ch->n_features;
    a.has_depth = ch->depth;
    a.has_flow = ch->flow;
    a.n_gauss = g->n;
    a.fn = P<float>(ctx->fn);
    a.flow = P<float>(ctx->flow);
    a.out_ch = out_ch;
  }
  {
    Stage t(ctx, 4, st);
    raster_forward(a, st);
  }
  G4D_HIP(hipGetLastError());

  if (ctx->capturing) n_vis = n_pairs = -1;  // known on the device only
  ctx->stats.n_slots = slots;
  ctx->stats.n_visible = n_vis;
  ctx->stats.n_pairs = n_pairs;
  ctx->stats.n_tiles = ctx->n_tiles;
  ctx->stats.n_pixels = ctx->n_pixels;
  ctx->stats.pair_capacity = ctx->pair_cap;
  ctx->stats.n_clamped_batches = -1;
  SavedKey& k = ctx->key;
  k.n = g->n;
  k.sh_degree = g->sh_degree;
  k.t_degree = g->t_degree;
  k.n_views = n_views;
  const void* p[6] = {g->mean4, g->scale4, g->rot_l, g->rot_r, g->opacity, g->sh};
  for (int i = 0; i < 6; ++i) k.ptrs[i] = p[i];
  k.mask = g->mask;
  k.mask_thr = g->mask_threshold;
  k.views.assign(views, views + n_views);
  k.s = *s;
  k.ch = ch ? *ch : g4d_channels{};
  k.sky_cube = sky ? sky->cube : nullptr;
  k.sky_res = sky ? sky->resolution : 0;
  ctx->saved = cp == nullptr;  // a compact forward has no parameter arrays to differentiate
  return G4D_OK;
}

// Backward of the last forward; with ch (which must match that forward's), also the extra
// channels' contributions and the feature and gate gradients.
static g4d_status backward_impl(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                                int32_t n_views, const g4d_settings* s, const g4d_channels* ch,
                                const g4d_sky* sky, const float* dL_drgb, const float* dL_dch,
                                const g4d_grads* out, float* d_features, float* d_gate,
                                float* d_cube, void* stream) {
  g4d_status r = check_common(ctx, g, views, n_views, s);
  if (r != G4D_OK) return r;
  if (!dL_drgb || !out) return fail(ctx, G4D_EINVAL, "null dL_drgb or grads");
  if (ch) {
    if ((r = check_channels(ctx, g, ch)) != G4D_OK) return r;
    if (ch->n_features > 0 && g->n > 0 && !d_features)
      return fail(ctx, G4D_EINVAL, "null d_features");
  }
  if (!ctx->saved || !same_key(ctx->key, g, views, n_views, s) ||
      (ch && !same_channels(ctx->key.ch, *ch)) ||
      (sky ? (ctx->key.sky_cube != sky->cube || ctx->key.sky_res != sky->resolution)
           : ctx->key.sky_cube != nullptr))
    return fail(ctx, G4D_ESTATE, "backward without a matching forward on this context");
  hipStream_t st = static_cast<hipStream_t>(stream);
  G4D_HIP(hipSetDevice(ctx->device));
  const int64_t slots = (int64_t)g->n * n_views;
  const int D = ch ? ch->n_features : 0;
  if (d_gate && D > 0) fill_u32(reinterpret_cast<uint32_t*>(d_gate), D, 0u, st);
  if (sky && d_cube) {
    // the sky gradient depends on the pixels only (it is there even without Gaussians)
    const int R = sky->resolution;
    fill_u32(reinterpret_cast<uint32_t*>(d_cube), (int64_t)6 * R * R * 3, 0u, st);
    int mw = 0, mh = 0;
    for (int v = 0; v < n_views; ++v) {
      mw = std::max(mw, views[v].width);
      mh = std::max(mh, views[v].height);
    }
    sky_backward(P<DView>(ctx->views), n_views, mw, mh, R, P<float>(ctx->px_T), dL_drgb, d_cube,
                 st);
  }
  if (slots == 0) return G4D_OK;
  const g4d_settings s_run = run_settings(s, ch);
  const DSettings DS = device_settings(&s_run, ctx->fwd_cutoff_bins);
  const size_t grad2d_cap = ctx->grad2d.cap;
  if ((r = ensure(ctx, ctx->grad2d, sizeof(float) * kGrad2d * slots, 1.1)) != G4D_OK) return r;
  {
    Stage t(ctx, 5, st);
    if (!ctx->grad2d_zero || ctx->grad2d.cap != grad2d_cap)
      fill_u32(P<uint32_t>(ctx->grad2d), (int64_t)(ctx->grad2d.cap / sizeof(uint32_t)), 0u, st);
  }
  ctx->grad2d_zero = false;
  if (D > 0) {
    if ((r = ensure(ctx, ctx->dfn, sizeof(float) * (size_t)g->n * D, 1.1)) != G4D_OK) return r;
    fill_u32(P<uint32_t>(ctx->dfn), (int64_t)g->n * D, 0u, st);
  }
  if (ctx->stats.n_pairs > 0 || ctx->capturing) {
    RasterArgs a{};
    a.rec = P<float>(ctx->rec);
    a.pval = P<uint32_t>(ctx->pval);
    a.ranges = P<uint2>(ctx->ranges);
    a.views = P<DView>(ctx->views);
    a.tile_base = P<int32_t>(ctx->tile_base);
    a.n_views = n_views;
    a.n_tiles = (int)ctx->n_tiles;
    a.S = DS;
    a.px_T = P<float>(ctx->px_T);
    a.px_last = P<int32_t>(ctx->px_last);
    a.dL = dL_drgb;
    a.grad2d = P<float>(ctx->grad2d);
    a.bg_px = sky ? P<float>(ctx->skybg) : nullptr;
    if (ctx->count_evals && !ctx->capturing) {
      fill_u32(P<uint32_t>(ctx->counters) + 4, 1, 0u, st);
      a.clamp_batches = P<uint32_t>(ctx->counters) + 4;
      ctx->counted_bwd = true;
    }
    if (ch) {
      a.n_ext = n_ext_of(ch);
      a.n_feat = D;
      a.has_depth = ch->depth;
      a.has_flow = ch->flow;
      a.n_gauss = g->n;
      a.fn = P<float>(ctx->fn);
      a.flow = P<float>(ctx->flow);
      a.dL_ch = dL_dch;
      a.dfn = P<float>(ctx->dfn);
    }
    Stage t(ctx, 6, st);
    raster_backward(a, st);
    G4D_HIP(hipGetLastError());
  }
  GradPtrs gp{out->mean4, out->scale4, out->rot_l,  out->rot_r,
              out->opacity, out->sh,  out->mask, out->densify};
  {
    Stage t(ctx, 7, st);
    preprocess_backward(gauss_ptrs(g), P<DView>(ctx->views), n_views, DS, P<uint32_t>(ctx->tiles),
                        P<float>(ctx->grad2d), gp, st);
    G4D_HIP(hipGetLastError());
  }
  ctx->grad2d_zero = true;
  if (D > 0)
    feature_backward(g->n, D, ch->features, ch->gate, P<float>(ctx->fn), P<float>(ctx->fnorm),
                     P<float>(ctx->dfn), d_features, d_gate, st);
  G4D_HIP(hipGetLastError());
  return G4D_OK;
}

g4d_status g4d_render_forward(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                              int32_t n_views, const g4d_settings* s, float* out_rgb,
                              float* out_T, void* stream) {
  return forward_impl(ctx, g, views, n_views, s, nullptr, nullptr, out_rgb, out_T, nullptr,
                      stream);
}

g4d_status g4d_render_backward(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                               int32_t n_views, const g4d_settings* s, const float* dL_drgb,
                               const g4d_grads* out, void* stream) {
  return backward_impl(ctx, g, views, n_views, s, nullptr, nullptr, dL_drgb, nullptr, out,
                       nullptr, nullptr, nullptr, stream);
}

g4d_status g4d_render_channels_forward(g4d_ctx* ctx, const g4d_gaussians* g,
                                       const g4d_view* views, int32_t n_views,
                                       const g4d_settings* s, const g4d_channels* ch,
                                       float* out_rgb, float* out_T, float* out_ch, void* stream) {
  if (!ctx) return G4D_EINVAL;
  if (!ch) return fail(ctx, G4D_EINVAL, "null channels");
  return forward_impl(ctx, g, views, n_views, s, ch, nullptr, out_rgb, out_T, out_ch, stream);
}

g4d_status g4d_render_channels_backward(g4d_ctx* ctx, const g4d_gaussians* g,
                                        const g4d_view* views, int32_t n_views,
                                        const g4d_settings* s, const g4d_channels* ch,
                                        const float* dL_drgb, const float* dL_dch,
                                        const g4d_grads* out, float* d_features, float* d_gate,
                                        void* stream) {
  if (!ctx) return G4D_EINVAL;
  if (!ch) return fail(ctx, G4D_EINVAL, "null channels");
  return backward_impl(ctx, g, views, n_views, s, ch, nullptr, dL_drgb, dL_dch, out, d_features,
                       d_gate, nullptr, stream);
}

static CompactPtrs compact_ptrs(const g4d_compact* c) {
  return CompactPtrs{c->mean4_h,  c->scale_idx,  c->rot_l_idx, c->rot_r_idx, c->opacity_q,
                     c->dc_idx,   c->rest_idx,   c->opacity_lo, c->opacity_hi, c->scale_cb,
                     c->rot_cb,   c->dc_cb,      c->rest_cb};
}

static g4d_status check_compact(g4d_ctx* ctx, const g4d_compact* c) {
  char msg[512];
  const g4d_status r = check_compact_args(c, msg, sizeof msg);
  if (r != G4D_OK) ctx->err = msg;
  return r;
}

g4d_status g4d_decode_compact(g4d_ctx* ctx, const g4d_compact* c, float* mean4, float* scale4,
                              float* rot_l, float* rot_r, float* opacity, float* sh,
                              void* stream) {
  if (!ctx) return G4D_EINVAL;
  g4d_status r = check_compact(ctx, c);
  if (r != G4D_OK) return r;
  if (c->n > 0 && (!mean4 || !scale4 || !rot_l || !rot_r || !opacity || !sh))
    return fail(ctx, G4D_EINVAL, "null output array");
  G4D_HIP(hipSetDevice(ctx->device));
  decode_compact_params(c->n, c->sh_degree, c->t_degree, compact_ptrs(c), mean4, scale4, rot_l,
                        rot_r, opacity, sh, static_cast<hipStream_t>(stream));
  G4D_HIP(hipGetLastError());
  return G4D_OK;
}

g4d_status g4d_render_compact_forward(g4d_ctx* ctx, const g4d_compact* c, const g4d_view* views,
                                      int32_t n_views, const g4d_settings* s, float* out_rgb,
                                      float* out_T, void* stream) {
  if (!ctx) return G4D_EINVAL;
  g4d_status r = check_compact(ctx, c);
  if (r != G4D_OK) return r;
  g4d_gaussians g{};
  g.n = c->n;
  g.sh_degree = c->sh_degree;
  g.t_degree = c->t_degree;
  const CompactPtrs cp = compact_ptrs(c);
  return forward_impl(ctx, &g, views, n_views, s, nullptr, nullptr, out_rgb, out_T, nullptr,
                      stream, &cp);
}

g4d_status g4d_render_sky_forward(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                                  int32_t n_views, const g4d_settings* s, const g4d_sky* sky,
                                  float* out_rgb, float* out_T, void* stream) {
  if (!ctx) return G4D_EINVAL;
  if (!sky) return fail(ctx, G4D_EINVAL, "null sky");
  return forward_impl(ctx, g, views, n_views, s, nullptr, sky, out_rgb, out_T, nullptr, stream);
}

g4d_status g4d_render_sky_backward(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                                   int32_t n_views, const g4d_settings* s, const g4d_sky* sky,
                                   const float* dL_drgb, const g4d_grads* out, float* d_cube,
                                   void* stream) {
  if (!ctx) return G4D_EINVAL;
  if (!sky) return fail(ctx, G4D_EINVAL, "null sky");
  return backward_impl(ctx, g, views, n_views, s, nullptr, sky, dL_drgb, nullptr, out, nullptr,
                       nullptr, d_cube, stream);
}

g4d_status g4d_render_step(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                           int32_t n_views, const g4d_settings* s, const float* dL_drgb,
                           float* out_rgb, float* out_T, const g4d_grads* grads, int32_t flags,
                           void* stream) {
  g4d_status r = check_common(ctx, g, views, n_views, s);
  if (r != G4D_OK) return r;
  if (!dL_drgb || !out_rgb || !grads) return fail(ctx, G4D_EINVAL, "null buffers");
  if (!(flags & G4D_STEP_GRAPH)) {
    if ((r = g4d_render_forward(ctx, g, views, n_views, s, out_rgb, out_T, stream)) != G4D_OK)
      return r;
    return g4d_render_backward(ctx, g, views, n_views, s, dL_drgb, grads, stream);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  G4D_HIP(hipSetDevice(ctx->device));
  // Everything the captured graph depends on: inputs, views, settings and output addresses.
  std::vector<unsigned char> key;
  auto put = [&key](const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    key.insert(key.end(), b, b + n);
  };
  put(g, sizeof *g);
  put(views, sizeof(g4d_view) * n_views);
  put(s, sizeof *s);
  put(&dL_drgb, sizeof dL_drgb);
  put(&out_rgb, sizeof out_rgb);
  put(&out_T, sizeof out_T);
  put(grads, sizeof *grads);
  if (!ctx->graph_exec || key != ctx->graph_key) {
    if (!ctx->graph_ctx) {
      if ((r = new_context(&ctx->graph_ctx, ctx->device)) != G4D_OK)
        return fail(ctx, r, "cannot create the graph context");
      G4D_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    }
    g4d_ctx* gc = ctx->graph_ctx;
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_key.clear();
    // One eager pass sizes every buffer and finds the pair and run counts; the capture then
    // gets capacities with 25% headroom (exceeding them is reported by g4d_sync_status).
    if ((r = g4d_render_forward(gc, g, views, n_views, s, out_rgb, out_T, stream)) != G4D_OK ||
        (r = g4d_render_backward(gc, g, views, n_views, s, dL_drgb, grads, stream)) != G4D_OK)
      return fail(ctx, r, "graph sizing pass: %s", gc->err.c_str());
    G4D_HIP(hipStreamSynchronize(st));
    const int64_t slots = (int64_t)g->n * n_views;
    const int64_t want_p = gc->stats.n_pairs + gc->stats.n_pairs / 4 + 4096;
    const int64_t want_r = gc->last_runs + gc->last_runs / 4 + 4096;
    if (want_p > (int64_t)INT32_MAX || want_r > (int64_t)INT32_MAX)
      return fail(ctx, G4D_ECAPACITY, "graph pair capacity %lld exceeds 2^31-1", (long long)want_p);
    if ((r = size_binning(gc, slots, want_r, want_p, 1.0)) != G4D_OK)
      return fail(ctx, r, "%s", gc->err.c_str());
    G4D_HIP(hipDeviceSynchronize());
    gc->capturing = true;
    hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      gc->capturing = false;
      return fail(ctx, G4D_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    g4d_status r1 = g4d_render_forward(gc, g, views, n_views, s, out_rgb, out_T, ctx->cap_stream);
    g4d_status r2 = r1 == G4D_OK ? g4d_render_backward(gc, g, views, n_views, s, dL_drgb, grads,
                                                       ctx->cap_stream)
                                 : r1;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(ctx->cap_stream, &graph);
    gc->capturing = false;
    if (r2 != G4D_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(ctx, r2 != G4D_OK ? r2 : G4D_EHIP, "graph capture failed: %s",
                  r2 != G4D_OK ? gc->err.c_str() : hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      ctx->graph_exec = nullptr;
      return fail(ctx, G4D_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    ctx->graph = graph;
    ctx->graph_key = key;
  }
  G4D_HIP(hipGraphLaunch(ctx->graph_exec, st));
  return G4D_OK;
}

// Points every buffer a plain forward + backward uses into the device's fixed scratch array
// (256-byte aligned slices, the counters first so that they stay at offset 0 whatever the
// sizes); the pair list, the row runs (half as many as pairs), the tile expansion's chunk maps
// and count table and the scan scratch share what remains, and the pair capacity is the
// largest that fits.
static g4d_status carve_scratch(g4d_ctx* ctx, g4d_ctx* na, unsigned char* base, int64_t slots,
                                int n_views, int64_t n_tiles, int64_t n_pixels, int64_t n_rows,
                                int64_t max_tx, int64_t max_ty) {
  const size_t cap = G4D_NOALLOC_SCRATCH_BYTES;
  auto round = [](size_t b) { return (std::max<size_t>(b, 256) + 255) & ~(size_t)255; };
  size_t off = 0;
  struct Slice { DevBuf* b; size_t off, bytes; };
  Slice plan[32];  // applied only once everything fits
  int n_plan = 0;
  auto take = [&](DevBuf& b, size_t bytes) {
    plan[n_plan++] = {&b, off, round(bytes)};
    off += round(bytes);
  };
  const int64_t rhist = max_ty * ((slots + 63) / 64 + n_views);
  take(na->counters, 32 * sizeof(uint32_t));
  take(na->views, sizeof(DView) * n_views);
  take(na->tile_base, sizeof(int32_t) * (n_views + 1));
  take(na->rec, sizeof(float) * kRec * slots);
  take(na->tiles, sizeof(uint32_t) * slots);
  take(na->rowbox, sizeof(uint32_t) * slots);
  take(na->dkey, sizeof(uint32_t) * slots);
  const int64_t n_wc = (slots / std::max(n_views, 1) + 255) / 256 * 4;
  take(na->wsum, sizeof(uint2) * n_wc);
  take(na->vmask, sizeof(uint64_t) * n_wc * n_views);
  for (int b = 0; b < 2; ++b) {
    take(na->vk[b], sizeof(uint32_t) * slots);
    take(na->vv[b], sizeof(uint32_t) * slots);
  }
  take(na->sort_tmp, depth_sort_scratch_bytes(slots, n_views));
  take(na->vrange, sizeof(uint2) * n_views);
  take(na->vinfo, 2 * sizeof(uint4) * n_views);
  take(na->cview, sizeof(uint16_t) * ((slots + 63) / 64 + n_views));
  take(na->rhist, sizeof(uint32_t) * rhist);
  take(na->ranges, sizeof(uint2) * n_tiles);
  take(na->rinfo, 2 * sizeof(uint4) * n_rows);
  take(na->px_T, sizeof(float) * n_pixels);
  take(na->px_last, sizeof(int32_t) * n_pixels);
  take(na->grad2d, sizeof(float) * kGrad2d * slots);
  const size_t fixed = off;
  // p pairs: the pair list, p / 2 runs of 8 bytes, the tile expansion's chunk maps and count
  // table, and the scan scratch of max(tables, slots) items
  auto hist_of = [&](int64_t runs) { return max_tx * ((runs + 63) / 64) + n_tiles; };
  auto chunks_of = [&](int64_t runs) { return (runs + 63) / 64 + n_rows; };
  auto need = [&](int64_t p) {
    const int64_t runs = p / 2;
    return round(sizeof(uint32_t) * (size_t)p) + round(sizeof(uint2) * (size_t)runs) +
           round(8 * sizeof(uint32_t) * (size_t)chunks_of(runs)) +
           round(sizeof(uint32_t) * (size_t)hist_of(runs)) +
           round(scan_scratch_bytes(std::max({hist_of(runs), rhist, slots})));
  };
  if (fixed > cap || need(0) > cap - fixed)
    return fail(ctx, G4D_ECAPACITY,
                "%lld slots, %lld tiles and %lld pixels need %zu bytes before any pair; the "
                "fixed scratch holds %zu (G4D_NOALLOC_SCRATCH_BYTES)",
                (long long)slots, (long long)n_tiles, (long long)n_pixels, fixed + need(0), cap);
  int64_t lo = 0, hi = (int64_t)((cap - fixed) / 4);
  while (lo < hi) {  // largest p with need(p) <= cap - fixed
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (need(mid) <= cap - fixed) lo = mid; else hi = mid - 1;
  }
  const int64_t pairs = std::min<int64_t>(lo, INT32_MAX), runs = pairs / 2;
  take(na->pval, sizeof(uint32_t) * pairs);
  take(na->runs, sizeof(uint2) * runs);
  take(na->crow, 8 * sizeof(uint32_t) * chunks_of(runs));
  take(na->hist, sizeof(uint32_t) * hist_of(runs));
  take(na->scan_tmp, scan_scratch_bytes(std::max({hist_of(runs), rhist, slots})));
  if (off > cap) return fail(ctx, G4D_EHIP, "scratch plan of %zu bytes exceeds %zu", off, cap);
  for (int k = 0; k < n_plan; ++k) {
    plan[k].b->p = base + plan[k].off;
    plan[k].b->cap = plan[k].bytes;
  }
  na->pair_cap = pairs;
  na->row_cap = runs;
  na->hist_cap = hist_of(runs);
  na->rhist_cap = rhist;
  return G4D_OK;
}

g4d_status g4d_render_step_noalloc(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                                   int32_t n_views, const g4d_settings* s, const float* dL_drgb,
                                   float* out_rgb, float* out_T, const g4d_grads* grads,
                                   void* stream) {
  g4d_status r = check_common(ctx, g, views, n_views, s);
  if (r != G4D_OK) return r;
  if (!dL_drgb || !out_rgb || !grads) return fail(ctx, G4D_EINVAL, "null buffers");
  const int dev = ctx->device;
  unsigned char* base = (dev >= 0 && dev < kMaxScratchDevices)
                            ? static_cast<unsigned char*>(g_scratch_ptr[dev])
                            : nullptr;
  if (!ctx->na || !base)
    return fail(ctx, G4D_EHIP, "no fixed scratch on device %d: %s", dev,
                dev < kMaxScratchDevices ? hipGetErrorString(g_scratch_err[dev])
                                         : "device index beyond the scratch table");
  // the sizes the forward plans (as upload_views counts them)
  int64_t n_tiles = 0, n_pixels = 0, n_rows = 0, max_tx = 0, max_ty = 0;
  for (int v = 0; v < n_views; ++v) {
    const int64_t tx = (views[v].width + s->tile_size - 1) / s->tile_size;
    const int64_t ty = (views[v].height + s->tile_size - 1) / s->tile_size;
    n_tiles += tx * ty;
    n_rows += ty;
    max_tx = std::max(max_tx, tx);
    max_ty = std::max(max_ty, ty);
    n_pixels += (int64_t)views[v].width * views[v].height;
  }
  g4d_ctx* na = ctx->na;
  if ((r = carve_scratch(ctx, na, base, (int64_t)g->n * n_views, n_views, n_tiles, n_pixels,
                         n_rows, max_tx, max_ty)) != G4D_OK)
    return r;
  // Another call may have left anything in the array: the view table is uploaded again and
  // the gradient slots, which the raster adjoint accumulates into, are cleared.
  na->uploaded_to = nullptr;
  na->uploaded_views.clear();
  na->grad2d_zero = false;
  na->count_evals = false;
  na->profiling = false;
  if ((r = g4d_render_forward(na, g, views, n_views, s, out_rgb, out_T, stream)) != G4D_OK ||
      (r = g4d_render_backward(na, g, views, n_views, s, dL_drgb, grads, stream)) != G4D_OK)
    return fail(ctx, r, "%s", na->err.c_str());
  return G4D_OK;
}

g4d_status g4d_sync_status(g4d_ctx* ctx, void* stream) {
  if (!ctx) return G4D_EINVAL;
  G4D_HIP(hipSetDevice(ctx->device));
  G4D_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  for (g4d_ctx* c : {ctx, ctx->graph_ctx, ctx->na}) {
    if (!c || !c->counters.p) continue;
    uint32_t flag = 0;
    G4D_HIP(hipMemcpy(&flag, P<uint32_t>(c->counters) + 2, sizeof flag, hipMemcpyDeviceToHost));
    if (!flag) continue;
    // reported once: the flag is cleared, and a graph that overflowed is dropped, so that the
    // next G4D_STEP_GRAPH call sizes and captures it again for the larger pair count
    const uint32_t zero = 0;
    G4D_HIP(hipMemcpy(P<uint32_t>(c->counters) + 2, &zero, sizeof zero, hipMemcpyHostToDevice));
    if (c == ctx->graph_ctx && flag == 1) {
      const long long cap = (long long)c->pair_cap;
      if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
      if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
      ctx->graph_exec = nullptr;
      ctx->graph = nullptr;
      ctx->graph_key.clear();
      return fail(ctx, G4D_ECAPACITY,
                  "graph capacity of %lld pairs or %lld row runs exceeded (the graph is dropped)",
                  cap, (long long)c->row_cap);
    }
    if (flag == 1)
      return fail(ctx, G4D_ECAPACITY, "capacity of %lld pairs or %lld row runs exceeded",
                  (long long)c->pair_cap, (long long)c->row_cap);
    return fail(ctx, G4D_EHIP, "pair count mismatch between the preprocess and the binning");
  }
  return G4D_OK;
}

g4d_status g4d_get_stats(g4d_ctx* ctx, g4d_stats* out, void* stream) {
  if (!ctx || !out) return G4D_EINVAL;
  G4D_HIP(hipSetDevice(ctx->device));
  G4D_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  *out = ctx->stats;
  if (ctx->counted_bwd) {
    uint32_t nb = 0;
    G4D_HIP(hipMemcpy(&nb, P<uint32_t>(ctx->counters) + 4, sizeof nb, hipMemcpyDeviceToHost));
    out->n_clamped_batches = nb;
  }
  return G4D_OK;
}

g4d_status g4d_get_pairs(g4d_ctx* ctx, uint32_t* tile_ids, uint32_t* slots, uint32_t* ranges,
                         void* stream) {
  if (!ctx) return G4D_EINVAL;
  if (!ctx->saved || ctx->stats.n_pairs < 0)
    return fail(ctx, G4D_ESTATE, "no eager forward whose binning is kept on this context");
  hipStream_t st = static_cast<hipStream_t>(stream);
  G4D_HIP(hipSetDevice(ctx->device));
  const int64_t np = ctx->stats.n_pairs;
  if (np > 0 && tile_ids) tile_ids_of(P<uint2>(ctx->ranges), ctx->n_tiles, np, tile_ids, st);
  if (np > 0 && slots)
    G4D_HIP(hipMemcpyAsync(slots, ctx->pval.p, sizeof(uint32_t) * np, hipMemcpyDeviceToDevice,
                           st));
  if (ranges && ctx->n_tiles > 0)
    G4D_HIP(hipMemcpyAsync(ranges, ctx->ranges.p, sizeof(uint2) * ctx->n_tiles,
                           hipMemcpyDeviceToDevice, st));
  G4D_HIP(hipGetLastError());
  return G4D_OK;
}

// Per-pixel evaluation counters (Gaussian-pixel pairs within the cutoff visited before the
// stop) of later forwards: enable = 1 turns them on, 0 off.  `out` (device, may be NULL)
// receives the counters of the last forward, pixels of all views concatenated.
g4d_status g4d_eval_counters(g4d_ctx* ctx, int enable, uint32_t* out, void* stream) {
  if (!ctx) return G4D_EINVAL;
  G4D_HIP(hipSetDevice(ctx->device));
  if (out) {
    if (!ctx->count_evals || !ctx->px_evals.p || !ctx->saved)
      return fail(ctx, G4D_ESTATE, "no counted forward on this context");
    G4D_HIP(hipMemcpyAsync(out, ctx->px_evals.p, sizeof(uint32_t) * ctx->n_pixels,
                           hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  }
  ctx->count_evals = enable != 0;
  ctx->count_cutoff = enable == 2;
  return G4D_OK;
}

g4d_status g4d_autotune(g4d_ctx* ctx, const g4d_gaussians* g, const g4d_view* views,
                        int32_t n_views, g4d_settings* s, const float* dL_drgb, float* out_rgb,
                        float* out_T, const g4d_grads* grads, int32_t reps, double* best_ms,
                        void* stream) {
  g4d_status r = check_common(ctx, g, views, n_views, s);
  if (r != G4D_OK) return r;
  if (!dL_drgb || !out_rgb || !grads) return fail(ctx, G4D_EINVAL, "null buffers");
  if (reps < 1) reps = 1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  G4D_HIP(hipSetDevice(ctx->device));
  // Problem shape: N, degrees, views and their sizes, and the settings that change the work.
  std::string key = std::to_string(g->n) + "/" + std::to_string(g->sh_degree) + "/" +
                    std::to_string(g->t_degree) + "/" + std::to_string(n_views);
  for (int v = 0; v < n_views; ++v)
    key += "/" + std::to_string(views[v].width) + "x" + std::to_string(views[v].height);
  char buf[96];
  snprintf(buf, sizeof buf, "/%g/%g/%g/%g", s->cutoff_sigma, s->marginal_min, s->alpha_min, s->T_min);
  key += buf;
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) {
    s->tile_size = it->second.tile;
    s->lds_batch = it->second.batch;
    s->px_per_lane = it->second.px;
    s->bwd_px_per_lane = it->second.bwd_px;
    if (best_ms) *best_ms = it->second.ms;
    return G4D_OK;
  }
  hipEvent_t e0, e1;
  G4D_HIP(hipEventCreate(&e0));
  G4D_HIP(hipEventCreate(&e1));
  g4d_ctx::Tuned best{16, 64, 4, 4, 1e30};
  // Candidates: tile x pixels per lane x backward pixels per lane (the forward's, or 8 at
  // 32-pixel tiles) x LDS batch.
  struct Cand { int tile, px, bwd_px; };
  std::vector<Cand> cands;
  for (int tile : {8, 16, 32})
    for (int px : {1, 2, 4}) {
      if (tile == 8 && px > 1) continue;
      cands.push_back({tile, px, px});
      if (tile == 32) cands.push_back({tile, px, 8});
    }
  for (const Cand& c : cands) {
    for (int batch : {32, 64, 128}) {
      g4d_settings trial = *s;
      trial.tile_size = c.tile;
      trial.lds_batch = batch;
      trial.px_per_lane = c.px;
      trial.bwd_px_per_lane = c.bwd_px;
      // one untimed pass sizes every buffer for this tile size
      if ((r = g4d_render_forward(ctx, g, views, n_views, &trial, out_rgb, out_T, stream)) != G4D_OK ||
          (r = g4d_render_backward(ctx, g, views, n_views, &trial, dL_drgb, grads, stream)) != G4D_OK)
        break;
      G4D_HIP(hipEventRecord(e0, st));
      for (int k = 0; k < reps && r == G4D_OK; ++k) {
        r = g4d_render_forward(ctx, g, views, n_views, &trial, out_rgb, out_T, stream);
        if (r == G4D_OK)
          r = g4d_render_backward(ctx, g, views, n_views, &trial, dL_drgb, grads, stream);
      }
      if (r != G4D_OK) break;
      G4D_HIP(hipEventRecord(e1, st));
      G4D_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      G4D_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double per = ms / reps;
      if (std::getenv("G4D_TUNE_VERBOSE"))
        fprintf(stderr, "g4d_autotune: tile %d batch %d px/lane %d (backward %d): %.3f ms\n",
                c.tile, batch, c.px, c.bwd_px, per);
      if (per < best.ms) best = {c.tile, batch, c.px, c.bwd_px, per};
    }
    if (r != G4D_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r != G4D_OK) return r;
  ctx->tuned[key] = best;
  s->tile_size = best.tile;
  s->lds_batch = best.batch;
  s->px_per_lane = best.px;
  s->bwd_px_per_lane = best.bwd_px;
  if (best_ms) *best_ms = best.ms;
  return G4D_OK;
}

g4d_status g4d_profile_mask(g4d_ctx* ctx, uint32_t stage_mask) {
  if (!ctx) return G4D_EINVAL;
  ctx->stage_mask = stage_mask;
  return G4D_OK;
}

g4d_status g4d_profile(g4d_ctx* ctx, int enable, double* ms, int64_t* launches, int reset) {
  if (!ctx) return G4D_EINVAL;
  G4D_HIP(hipSetDevice(ctx->device));
  if (ms || launches || reset) {
    G4D_HIP(hipDeviceSynchronize());
    for (auto& iv : ctx->pending) {
      float t = 0.f;
      G4D_HIP(hipEventElapsedTime(&t, iv.a, iv.b));
      ctx->stage_ms[iv.stage] += t;
      ctx->stage_n[iv.stage] += 1;
      ctx->ev_free.push_back(iv.a);
      ctx->ev_free.push_back(iv.b);
    }
    ctx->pending.clear();
    for (int k = 0; k < G4D_NUM_STAGES; ++k) {
      if (ms) ms[k] = ctx->stage_ms[k];
      if (launches) launches[k] = ctx->stage_n[k];
      if (reset) {
        ctx->stage_ms[k] = 0.0;
        ctx->stage_n[k] = 0;
      }
    }
  }
  ctx->profiling = enable != 0;
  return G4D_OK;
}

const char* g4d_stage_name(int stage) {
  return (stage >= 0 && stage < G4D_NUM_STAGES) ? kStageNames[stage] : "";
}

}  // extern "C"
