// Drives the host-side argument checks of the C ABI (csrc/g4d_checks.cpp) with valid and
// invalid arguments and with random bit patterns, so that a build with the address and
// undefined-behaviour sanitizers (tests/test_sanitize.py) sees every branch.  Exit status 0
// and the line "checks ok" on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>

#include "g4d_checks.h"

using namespace g4d;

namespace {

int n_cases = 0, n_failures = 0;

void expect(bool ok, int line, const char* what) {
  ++n_cases;
  if (!ok) {
    std::fprintf(stderr, "FAIL line %d: %s\n", line, what);
    ++n_failures;
  }
}
#define EXPECT(c) expect((c), __LINE__, #c)

float buf[64];

g4d_gaussians gaussians() {
  g4d_gaussians g{};
  g.n = 10;
  g.sh_degree = 3;
  g.t_degree = 1;
  g.mean4 = g.scale4 = g.rot_l = g.rot_r = g.opacity = g.sh = buf;
  return g;
}

g4d_view view() {
  g4d_view v{};
  v.width = 64;
  v.height = 48;
  v.fx = v.fy = 50.f;
  v.cx = 32.f;
  v.cy = 24.f;
  v.world_to_cam[0] = v.world_to_cam[5] = v.world_to_cam[10] = 1.f;
  v.world_to_cam[11] = 3.f;
  v.t = 0.5f;
  return v;
}

g4d_settings settings() {  // the library defaults
  g4d_settings s{};
  s.near_z = 0.2f;
  s.marginal_min = 1.f / 255.f;
  s.cutoff_sigma = 3.f;
  s.blur = 0.3f;
  s.jacobian_margin = 0.15f;
  s.alpha_min = 1.f / 255.f;
  s.alpha_max = 0.99f;
  s.T_min = 1e-4f;
  s.color_offset = 0.5f;
  s.color_min = 0.f;
  s.time_period = 1.f;
  s.tile_size = 16;
  return s;
}

g4d_status args(const g4d_gaussians& g, const g4d_view& v, const g4d_settings& s, int nv = 1) {
  static g4d_view views[G4D_MAX_VIEWS + 1];
  for (int k = 0; k < G4D_MAX_VIEWS + 1; ++k) views[k] = v;
  char msg[512];
  msg[0] = 0;
  const g4d_status r = check_args(&g, views, nv, &s, true, msg, sizeof msg);
  if (r != G4D_OK && std::strlen(msg) == 0) return G4D_OK;  // an error must say why
  return r;
}

}  // namespace

int main() {
  const float nan = std::numeric_limits<float>::quiet_NaN();
  const float inf = std::numeric_limits<float>::infinity();
  const g4d_gaussians G = gaussians();
  const g4d_view V = view();
  const g4d_settings S = settings();
  char msg[512];
  EXPECT(args(G, V, S) == G4D_OK);
  EXPECT(args(G, V, S, G4D_MAX_VIEWS) == G4D_OK);
  EXPECT(check_args(nullptr, &V, 1, &S, true, msg, sizeof msg) == G4D_EINVAL);
  EXPECT(check_args(&G, nullptr, 1, &S, true, msg, sizeof msg) == G4D_EINVAL);
  EXPECT(check_args(&G, &V, 1, nullptr, true, msg, sizeof msg) == G4D_EINVAL);
  // a short or missing message buffer is never overrun
  char tiny[4] = {'x', 'x', 'x', 'x'};
  EXPECT(check_args(nullptr, &V, 1, &S, true, tiny, sizeof tiny) == G4D_EINVAL && tiny[3] == 0);
  EXPECT(check_args(nullptr, &V, 1, &S, true, nullptr, 0) == G4D_EINVAL);
  {  // Gaussians
    g4d_gaussians g = G;
    g.n = -1;
    EXPECT(args(g, V, S) == G4D_EINVAL);
    g = G;
    g.sh_degree = 4;
    EXPECT(args(g, V, S) == G4D_EINVAL);
    g.sh_degree = -1;
    EXPECT(args(g, V, S) == G4D_EINVAL);
    g = G;
    g.t_degree = 3;
    EXPECT(args(g, V, S) == G4D_EINVAL);
    g = G;
    g.sh = nullptr;
    EXPECT(args(g, V, S) == G4D_EINVAL);
    EXPECT(check_args(&g, &V, 1, &S, false, msg, sizeof msg) == G4D_OK);  // no arrays needed
    g.n = 0;
    EXPECT(args(g, V, S) == G4D_OK);  // an empty set needs no arrays
    g = G;
    g.mask = buf;
    g.mask_threshold = nan;
    EXPECT(args(g, V, S) == G4D_EINVAL);
    g = G;
    g.n = std::numeric_limits<int32_t>::max();
    EXPECT(args(g, V, S, 1) == G4D_OK);
    EXPECT(args(g, V, S, 2) == G4D_EINVAL);  // N * views above 2^31 - 1
  }
  {  // views
    EXPECT(args(G, V, S, 0) == G4D_EINVAL);
    EXPECT(args(G, V, S, G4D_MAX_VIEWS + 1) == G4D_EINVAL);
    g4d_view v = V;
    v.width = 0;
    EXPECT(args(G, v, S) == G4D_EINVAL);
    v = V;
    v.height = G4D_MAX_SIDE + 1;
    EXPECT(args(G, v, S) == G4D_EINVAL);
    const float bad[] = {nan, inf, -inf, 0.f, -1.f};
    for (float x : bad) {
      v = V;
      v.fx = x;
      EXPECT(args(G, v, S) == G4D_EINVAL);
      v = V;
      v.fy = x;
      EXPECT(args(G, v, S) == G4D_EINVAL);
    }
    for (float x : {nan, inf}) {
      v = V;
      v.cx = x;
      EXPECT(args(G, v, S) == G4D_EINVAL);
      v = V;
      v.cy = x;
      EXPECT(args(G, v, S) == G4D_EINVAL);
      v = V;
      v.t = x;
      EXPECT(args(G, v, S) == G4D_EINVAL);
      for (int k = 0; k < 12; ++k) {
        v = V;
        v.world_to_cam[k] = x;
        EXPECT(args(G, v, S) == G4D_EINVAL);
      }
    }
  }
  {  // settings
    struct F { float g4d_settings::*f; float bad; };
    const F cases[] = {
        {&g4d_settings::near_z, 0.f},          {&g4d_settings::near_z, nan},
        {&g4d_settings::near_z, inf},          {&g4d_settings::cutoff_sigma, 0.f},
        {&g4d_settings::cutoff_sigma, nan},    {&g4d_settings::alpha_min, 0.f},
        {&g4d_settings::alpha_min, nan},       {&g4d_settings::alpha_max, 1.f},
        {&g4d_settings::alpha_max, 0.001f},    {&g4d_settings::alpha_max, nan},
        {&g4d_settings::T_min, -1e-4f},        {&g4d_settings::T_min, nan},
        {&g4d_settings::time_period, 0.f},     {&g4d_settings::time_period, nan},
        {&g4d_settings::blur, -0.1f},          {&g4d_settings::blur, nan},
        {&g4d_settings::jacobian_margin, -1.f}, {&g4d_settings::jacobian_margin, nan},
        {&g4d_settings::marginal_min, inf},    {&g4d_settings::marginal_min, nan},
        {&g4d_settings::color_offset, nan},    {&g4d_settings::color_min, nan},
    };
    for (const F& c : cases) {
      g4d_settings s = S;
      s.*(c.f) = c.bad;
      EXPECT(args(G, V, s) == G4D_EINVAL);
    }
    struct I { int32_t g4d_settings::*f; int32_t v; g4d_status want; };
    const I ints[] = {
        {&g4d_settings::tile_size, 8, G4D_OK},        {&g4d_settings::tile_size, 32, G4D_OK},
        {&g4d_settings::tile_size, 12, G4D_EINVAL},   {&g4d_settings::tile_size, 0, G4D_EINVAL},
        {&g4d_settings::lds_batch, 128, G4D_OK},      {&g4d_settings::lds_batch, 48, G4D_EINVAL},
        {&g4d_settings::px_per_lane, 4, G4D_OK},      {&g4d_settings::px_per_lane, 3, G4D_EINVAL},
        {&g4d_settings::bwd_px_per_lane, 4, G4D_OK},  {&g4d_settings::bwd_px_per_lane, 8, G4D_EINVAL},
        {&g4d_settings::bwd_px_per_lane, 5, G4D_EINVAL},
    };
    for (const I& c : ints) {
      g4d_settings s = S;
      s.*(c.f) = c.v;
      EXPECT(args(G, V, s) == c.want);
    }
    g4d_settings s = S;
    s.tile_size = 8;
    s.px_per_lane = 2;
    EXPECT(args(G, V, s) == G4D_EINVAL);
    s = S;
    s.tile_size = 32;
    s.bwd_px_per_lane = 8;
    EXPECT(args(G, V, s) == G4D_OK);
    s.color_min = -inf;  // no clamp
    EXPECT(args(G, V, s) == G4D_OK);
  }
  {  // extra channels
    g4d_channels c{};
    c.n_features = 32;
    c.features = buf;
    c.depth = 1;
    c.flow = 1;
    c.flow_dt = 0.05f;
    EXPECT(check_channels_args(&G, &c, msg, sizeof msg) == G4D_OK && n_ext_of(&c) == 35);
    EXPECT(check_channels_args(&G, nullptr, msg, sizeof msg) == G4D_EINVAL);
    g4d_channels d = c;
    d.n_features = -1;
    EXPECT(check_channels_args(&G, &d, msg, sizeof msg) == G4D_EINVAL);
    d = c;
    d.n_features = std::numeric_limits<int32_t>::max();  // no overflow in the channel count
    EXPECT(check_channels_args(&G, &d, msg, sizeof msg) == G4D_EINVAL);
    d = c;
    d.n_features = 34;
    EXPECT(check_channels_args(&G, &d, msg, sizeof msg) == G4D_EINVAL);
    d = c;
    d.depth = 2;
    EXPECT(check_channels_args(&G, &d, msg, sizeof msg) == G4D_EINVAL);
    d = c;
    d.features = nullptr;
    EXPECT(check_channels_args(&G, &d, msg, sizeof msg) == G4D_EINVAL);
    d = c;
    d.flow_dt = nan;
    EXPECT(check_channels_args(&G, &d, msg, sizeof msg) == G4D_EINVAL);
    d = g4d_channels{};
    EXPECT(check_channels_args(&G, &d, msg, sizeof msg) == G4D_EINVAL);  // no channel at all
    EXPECT(n_ext_of(nullptr) == 0);
  }
  {  // compact models
    static const uint16_t h[8] = {};
    static const uint8_t idx[16] = {};
    g4d_compact c{};
    c.n = 2;
    c.sh_degree = 3;
    c.t_degree = 1;
    c.mean4_h = h;
    c.scale_idx = c.rot_l_idx = c.rot_r_idx = c.opacity_q = c.dc_idx = c.rest_idx = idx;
    c.scale_cb = c.rot_cb = c.dc_cb = c.rest_cb = buf;
    c.opacity_lo = 0.f;
    c.opacity_hi = 1.f;
    EXPECT(check_compact_args(&c, msg, sizeof msg) == G4D_OK);
    EXPECT(check_compact_args(nullptr, msg, sizeof msg) == G4D_EINVAL);
    g4d_compact d = c;
    d.rest_idx = nullptr;
    EXPECT(check_compact_args(&d, msg, sizeof msg) == G4D_EINVAL);
    d.sh_degree = 0;
    d.t_degree = 0;  // a single coefficient: no rest codebook needed
    EXPECT(check_compact_args(&d, msg, sizeof msg) == G4D_OK);
    d = c;
    d.t_degree = 3;
    EXPECT(check_compact_args(&d, msg, sizeof msg) == G4D_EINVAL);
    d = c;
    d.opacity_hi = inf;
    EXPECT(check_compact_args(&d, msg, sizeof msg) == G4D_EINVAL);
  }
  {  // random bit patterns in every field: OK or EINVAL with a message, nothing else
    std::mt19937_64 rng(12345);
    auto rnd_float = [&rng]() {
      const uint32_t bits = (uint32_t)rng();
      float f;
      std::memcpy(&f, &bits, sizeof f);
      return f;
    };
    int ok = 0;
    for (int it = 0; it < 20000; ++it) {
      g4d_gaussians g = G;
      g4d_view v = V;
      g4d_settings s = S;
      g.n = (int32_t)(rng() % 3 == 0 ? rng() : rng() % 100000);
      g.sh_degree = (int32_t)(rng() % 6) - 1;
      g.t_degree = (int32_t)(rng() % 5) - 1;
      v.width = (int32_t)(rng() % 3 == 0 ? rng() : rng() % 9000);
      v.height = (int32_t)(rng() % 3 == 0 ? rng() : rng() % 9000);
      float* vf[] = {&v.fx, &v.fy, &v.cx, &v.cy, &v.t};
      for (float* f : vf)
        if (rng() % 4 == 0) *f = rnd_float();
      for (int k = 0; k < 12; ++k)
        if (rng() % 8 == 0) v.world_to_cam[k] = rnd_float();
      float* sf[] = {&s.near_z, &s.marginal_min, &s.cutoff_sigma, &s.blur, &s.jacobian_margin,
                     &s.alpha_min, &s.alpha_max, &s.T_min, &s.color_offset, &s.color_min,
                     &s.time_period};
      for (float* f : sf)
        if (rng() % 6 == 0) *f = rnd_float();
      int32_t* si[] = {&s.tile_size, &s.lds_batch, &s.px_per_lane, &s.bwd_px_per_lane};
      for (int32_t* x : si)
        if (rng() % 6 == 0) *x = (int32_t)rng();
      const int nv = (int)(rng() % 300) - 20;
      const g4d_status r = args(g, v, s, nv);
      EXPECT(r == G4D_OK || r == G4D_EINVAL);
      ok += r == G4D_OK;
      g4d_channels c{};
      c.n_features = (int32_t)rng();
      c.depth = (int32_t)(rng() % 3);
      c.flow = (int32_t)(rng() % 3);
      c.flow_dt = rnd_float();
      c.features = rng() % 2 ? buf : nullptr;
      const g4d_status rc = check_channels_args(&g, &c, msg, sizeof msg);
      EXPECT(rc == G4D_OK || rc == G4D_EINVAL);
    }
    EXPECT(ok > 0);
  }
  if (n_failures) {
    std::fprintf(stderr, "%d of %d checks failed\n", n_failures, n_cases);
    return 1;
  }
  std::printf("checks ok: %d cases\n", n_cases);
  return 0;
}
