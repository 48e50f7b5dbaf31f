// Host-side argument checks of the C ABI (plain C++, no HIP): every entry point validates its
// Gaussians, views, settings, channels and compact models here before anything is enqueued.
// Kept free of the HIP runtime so that the same source also builds with the host compiler's
// address and undefined-behaviour sanitizers.
#include "g4d_checks.h"

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

namespace g4d {
namespace {

bool finite(float x) { return std::isfinite(x); }

g4d_status fail(char* err, size_t n_err, g4d_status st, const char* fmt, ...) {
  if (err && n_err > 0) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(err, n_err, fmt, ap);
    va_end(ap);
  }
  return st;
}

}  // namespace

g4d_status check_args(const g4d_gaussians* g, const g4d_view* views, int32_t n_views,
                      const g4d_settings* s, bool params, char* err, size_t n_err) {
  if (!g || !views || !s) return fail(err, n_err, G4D_EINVAL, "null gaussians, views or settings");
  if (g->n < 0) return fail(err, n_err, G4D_EINVAL, "n = %d < 0", g->n);
  if (g->sh_degree < 0 || g->sh_degree > G4D_MAX_SH_DEGREE)
    return fail(err, n_err, G4D_EINVAL, "sh_degree %d outside 0..%d", g->sh_degree, G4D_MAX_SH_DEGREE);
  if (g->t_degree < 0 || g->t_degree > G4D_MAX_T_DEGREE)
    return fail(err, n_err, G4D_EINVAL, "t_degree %d outside 0..%d", g->t_degree, G4D_MAX_T_DEGREE);
  if (params && g->n > 0 &&
      (!g->mean4 || !g->scale4 || !g->rot_l || !g->rot_r || !g->opacity || !g->sh))
    return fail(err, n_err, G4D_EINVAL, "null Gaussian parameter array");
  if (g->mask && std::isnan(g->mask_threshold)) return fail(err, n_err, G4D_EINVAL, "mask_threshold NaN");
  if (n_views < 1 || n_views > G4D_MAX_VIEWS)
    return fail(err, n_err, G4D_EINVAL, "n_views %d outside 1..%d", n_views, G4D_MAX_VIEWS);
  if ((int64_t)g->n * n_views > (int64_t)INT32_MAX)
    return fail(err, n_err, G4D_EINVAL, "n * n_views = %lld exceeds 2^31-1", (long long)g->n * n_views);
  for (int v = 0; v < n_views; ++v) {
    const g4d_view& V = views[v];
    if (V.width < 1 || V.height < 1 || V.width > G4D_MAX_SIDE || V.height > G4D_MAX_SIDE)
      return fail(err, n_err, G4D_EINVAL, "view %d: size %dx%d outside 1..%d", v, V.width, V.height,
                  G4D_MAX_SIDE);
    if (!(V.fx > 0.f) || !(V.fy > 0.f) || !finite(V.fx) || !finite(V.fy) || !finite(V.cx) ||
        !finite(V.cy) || !finite(V.t))
      return fail(err, n_err, G4D_EINVAL, "view %d: bad intrinsics or time", v);
    for (int k = 0; k < 12; ++k)
      if (!finite(V.world_to_cam[k])) return fail(err, n_err, G4D_EINVAL, "view %d: bad extrinsic", v);
  }
  // 0 < alpha_min <= alpha_max < 1: the backward rebuilds T by dividing by 1 - alpha and
  // recovers the opacity partial of an entry by dividing by its opacity p_t >= alpha_min.
  if (!(s->near_z > 0.f) || !(s->cutoff_sigma > 0.f) || !(s->alpha_min > 0.f) ||
      !(s->alpha_max >= s->alpha_min) ||
      !(s->alpha_max < 1.f) || !(s->T_min >= 0.f) || !(s->time_period > 0.f) ||
      !(s->blur >= 0.f) || !(s->jacobian_margin >= 0.f) || !finite(s->near_z) ||
      !finite(s->marginal_min) || !finite(s->color_offset) || std::isnan(s->color_min))
    return fail(err, n_err, G4D_EINVAL, "invalid settings");
  if (s->tile_size != 8 && s->tile_size != 16 && s->tile_size != 32)
    return fail(err, n_err, G4D_EINVAL, "tile_size %d not in {8, 16, 32}", s->tile_size);
  if (s->lds_batch != 0 && s->lds_batch != 32 && s->lds_batch != 64 && s->lds_batch != 128)
    return fail(err, n_err, G4D_EINVAL, "lds_batch %d not in {0, 32, 64, 128}", s->lds_batch);
  if (s->px_per_lane != 0 && s->px_per_lane != 1 && s->px_per_lane != 2 && s->px_per_lane != 4)
    return fail(err, n_err, G4D_EINVAL, "px_per_lane %d not in {0, 1, 2, 4}", s->px_per_lane);
  if (s->tile_size == 8 && s->px_per_lane > 1)
    return fail(err, n_err, G4D_EINVAL, "px_per_lane %d needs tile_size >= 16", s->px_per_lane);
  const int bp = s->bwd_px_per_lane;
  if (bp != 0 && bp != 1 && bp != 2 && bp != 4 && bp != 8)
    return fail(err, n_err, G4D_EINVAL, "bwd_px_per_lane %d not in {0, 1, 2, 4, 8}", bp);
  if ((s->tile_size == 8 && bp > 1) || (s->tile_size != 32 && bp == 8))
    return fail(err, n_err, G4D_EINVAL, "bwd_px_per_lane %d does not fit tile_size %d", bp, s->tile_size);
  return G4D_OK;
}

int n_ext_of(const g4d_channels* ch) {
  if (!ch) return 0;
  const int64_t e = (int64_t)ch->n_features + (ch->depth ? 1 : 0) + (ch->flow ? 2 : 0);
  return e > INT32_MAX ? INT32_MAX : (int)e;  // anything above G4D_MAX_CHANNELS is rejected
}

g4d_status check_channels_args(const g4d_gaussians* g, const g4d_channels* ch, char* err,
                               size_t n_err) {
  if (!ch) return fail(err, n_err, G4D_EINVAL, "null channels");
  if (ch->n_features < 0) return fail(err, n_err, G4D_EINVAL, "n_features %d < 0", ch->n_features);
  if ((ch->depth != 0 && ch->depth != 1) || (ch->flow != 0 && ch->flow != 1))
    return fail(err, n_err, G4D_EINVAL, "depth and flow must be 0 or 1");
  const int E = n_ext_of(ch);
  if (E < 1 || E > G4D_MAX_CHANNELS)
    return fail(err, n_err, G4D_EINVAL, "%d extra channels outside 1..%d", E, G4D_MAX_CHANNELS);
  if (ch->n_features > 0 && g->n > 0 && !ch->features)
    return fail(err, n_err, G4D_EINVAL, "null features");
  if (ch->flow && !finite(ch->flow_dt)) return fail(err, n_err, G4D_EINVAL, "flow_dt not finite");
  return G4D_OK;
}

g4d_status check_compact_args(const g4d_compact* c, char* err, size_t n_err) {
  if (!c) return fail(err, n_err, G4D_EINVAL, "null compact model");
  if (c->n < 0 || c->sh_degree < 0 || c->sh_degree > G4D_MAX_SH_DEGREE || c->t_degree < 0 ||
      c->t_degree > G4D_MAX_T_DEGREE)
    return fail(err, n_err, G4D_EINVAL, "compact model: bad n or degrees");
  const bool rest = (c->t_degree + 1) * (c->sh_degree + 1) * (c->sh_degree + 1) > 1;
  if (c->n > 0 && (!c->mean4_h || !c->scale_idx || !c->rot_l_idx || !c->rot_r_idx ||
                   !c->opacity_q || !c->dc_idx || !c->scale_cb || !c->rot_cb || !c->dc_cb ||
                   (rest && (!c->rest_idx || !c->rest_cb))))
    return fail(err, n_err, G4D_EINVAL, "compact model: null array");
  if (!std::isfinite(c->opacity_lo) || !std::isfinite(c->opacity_hi))
    return fail(err, n_err, G4D_EINVAL, "compact model: opacity range not finite");
  return G4D_OK;
}

}  // namespace g4d
