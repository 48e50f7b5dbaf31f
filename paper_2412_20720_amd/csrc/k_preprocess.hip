// Per-(Gaussian, view) slice, splat and color (forward), and their adjoint (backward).
//
// One thread per Gaussian loops over all views of the batch: the rotors, the 4D covariance
// factor M = R S and the 4DSH coefficients are read and built once per batch and reused for
// every view (Sec. 3.2: the covariance and color parameters are view-independent; only the
// slice time t and the camera change).  Records are written view-major (slot = view * N + g)
// so that a wave's 64 consecutive Gaussians store 64 consecutive records.
#include <hip/hip_runtime.h>

#include "g4d_internal.h"

namespace g4d {
namespace {

// CP: the parameters come from a compact model, decoded here in registers (Sec. 4.2).
template <int DS, int DT, bool CP>
__global__ __launch_bounds__(256) void k_preprocess(
    int n, int n_views, const float4* __restrict__ mean4, const float4* __restrict__ scale4,
    const float4* __restrict__ rot_l, const float4* __restrict__ rot_r,
    const float* __restrict__ opacity, const float* __restrict__ sh,
    const DView* __restrict__ views, DSettings S, float* __restrict__ rec,
    uint32_t* __restrict__ tiles, uint32_t* __restrict__ dkey, const float* __restrict__ mask,
    float mask_thr, CompactPtrs cp) {
  constexpr int NSH = (DT + 1) * (DS + 1) * (DS + 1) * 3;
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  if (mask && !(mask[gi] > mask_thr)) {
    // volume mask (Sec. 4.3): M_hat = 0 scales S and the opacity to zero, the Gaussian is gone
    for (int v = 0; v < n_views; ++v) tiles[(size_t)v * n + gi] = 0u;
    return;
  }
  float4 mean, sc4, qlr, qrr;
  float op;
  float shc[NSH];
  if constexpr (CP) {
    decode_compact<NSH>(cp, gi, mean, sc4, qlr, qrr, op, shc);
  } else {
    mean = mean4[gi];
    sc4 = scale4[gi];
    qlr = rot_l[gi];
    qrr = rot_r[gi];
    op = opacity[gi];
    const float* shp = sh + (size_t)gi * NSH;
#pragma unroll
    for (int k = 0; k < NSH; ++k) shc[k] = shp[k];
  }
  Geom g;
  geom_forward(qlr, qrr, sc4, g);
  for (int v = 0; v < n_views; ++v) {
    const DView& V = views[v];
    const size_t slot = (size_t)v * n + gi;
    ViewFwd f;
    uint32_t cnt = 0;
    // a splat that cannot reach alpha_min at any pixel of this view is not listed
    if (view_forward(g, mean, V, S, f) && reach2(op * f.pt, S) > 0.f) {
      const float opt = op * f.pt;
      color_forward<DS, DT>(shc, S, f);
      float ex, ey;
      reach_extent(f, reach2(opt, S), ex, ey);
      int x0, x1, y0, y1;
      if (tile_rect(f.u, f.v, ex, ey, V, S.tile_shift, x0, x1, y0, y1)) {
        const float lim = coverage_limit(opt, S);
        for (int ty = y0; ty <= y1; ++ty) {
          const int span = tile_row_span(f.u, f.v, f.conic[0], f.conic[1], f.conic[2], lim, ex,
                                         ey, ty, S.tile_shift, V.width, V.height, x0, x1);
          if (span >= 0) cnt += (uint32_t)((span & 0xFFFF) - (span >> 16) + 1);
        }
      }
      if (cnt > 0) {
        float4* r = reinterpret_cast<float4*>(rec + slot * kRec);
        r[0] = make_float4(f.u, f.v, f.conic[0], f.conic[1]);
        r[1] = make_float4(f.conic[2], opt, f.color[0], f.color[1]);
        r[2] = make_float4(f.color[2], ex, ey, f.x[2]);
        dkey[slot] = __float_as_uint(f.x[2]);
      }
    }
    tiles[slot] = cnt;
  }
}

template <int DS, int DT>
__global__ __launch_bounds__(256) void k_preprocess_bwd(
    int n, int n_views, const float4* __restrict__ mean4, const float4* __restrict__ scale4,
    const float4* __restrict__ rot_l, const float4* __restrict__ rot_r,
    const float* __restrict__ opacity, const float* __restrict__ sh,
    const DView* __restrict__ views, DSettings S, const uint32_t* __restrict__ tiles,
    const float* __restrict__ grad2d, GradPtrs out) {
  constexpr int NSH = (DT + 1) * (DS + 1) * (DS + 1) * 3;
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  const float4 sc = scale4[gi];
  Geom g;
  geom_forward(rot_l[gi], rot_r[gi], sc, g);
  const float4 mean = mean4[gi];
  const float op = opacity[gi];
  float shc[NSH], gsh[NSH];
  const float* shp = sh + (size_t)gi * NSH;
#pragma unroll
  for (int k = 0; k < NSH; ++k) {
    shc[k] = shp[k];
    gsh[k] = 0.f;
  }
  float gM[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) gM[i][j] = 0.f;
  float gmean[4] = {0.f, 0.f, 0.f, 0.f};
  float gop = 0.f;
  float dens = 0.f;  // sum over listed views of |dL/d(u, v)|
  int nvis = 0;
  for (int v = 0; v < n_views; ++v) {
    const size_t slot = (size_t)v * n + gi;
    if (tiles[slot] == 0u) continue;
    const float4* gp = reinterpret_cast<const float4*>(grad2d + slot * kGrad2d);
    const float4 q0 = gp[0], q1 = gp[1], q2 = gp[2];
    dens += sqrtf(fmaf(q0.x, q0.x, q0.y * q0.y));
    ++nvis;
    const float q[10] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y};
    const DView& V = views[v];
    ViewFwd f;
    view_forward<false>(g, mean, V, S, f);
    color_forward<DS, DT>(shc, S, f);
    view_backward<DS, DT>(g, mean, op, shc, V, S, f, q, gM, gmean, gop, gsh);
  }
  float gs[4], gql[4], gqr[4];
  geom_backward(g, sc, gM, gs, gql, gqr);
  if (out.mean4) reinterpret_cast<float4*>(out.mean4)[gi] = make_float4(gmean[0], gmean[1], gmean[2], gmean[3]);
  if (out.scale4) reinterpret_cast<float4*>(out.scale4)[gi] = make_float4(gs[0], gs[1], gs[2], gs[3]);
  if (out.rot_l) reinterpret_cast<float4*>(out.rot_l)[gi] = make_float4(gql[0], gql[1], gql[2], gql[3]);
  if (out.rot_r) reinterpret_cast<float4*>(out.rot_r)[gi] = make_float4(gqr[0], gqr[1], gqr[2], gqr[3]);
  if (out.opacity) out.opacity[gi] = gop;
  // straight-through volume mask: S_hat = M_hat S, opacity_hat = M_hat opacity at M_hat = 1 (a
  // removed Gaussian has no listed view, so every term is 0)
  if (out.mask)
    out.mask[gi] = fmaf(op, gop, fmaf(sc.x, gs[0], fmaf(sc.y, gs[1], fmaf(sc.z, gs[2], sc.w * gs[3]))));
  if (out.densify) {
    out.densify[3 * (size_t)gi + 0] = dens;
    out.densify[3 * (size_t)gi + 1] = fabsf(gmean[3]);
    out.densify[3 * (size_t)gi + 2] = (float)nvis;
  }
  if (out.sh) {
    float* o = out.sh + (size_t)gi * NSH;
#pragma unroll
    for (int k = 0; k < NSH; ++k) o[k] = gsh[k];
  }
}

template <int DS, int DT>
void launch_fwd(const GaussPtrs& gp, const DView* views, int n_views, DSettings S, float* rec,
                uint32_t* tiles, uint32_t* dkey, hipStream_t st) {
  const int blocks = (gp.n + 255) / 256;
  if (gp.compact)
    hipLaunchKernelGGL((k_preprocess<DS, DT, true>), dim3(blocks), dim3(256), 0, st, gp.n, n_views,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, views, S, rec, tiles,
                       dkey, nullptr, 0.f, *gp.compact);
  else
    hipLaunchKernelGGL((k_preprocess<DS, DT, false>), dim3(blocks), dim3(256), 0, st, gp.n,
                       n_views, reinterpret_cast<const float4*>(gp.mean4),
                       reinterpret_cast<const float4*>(gp.scale4),
                       reinterpret_cast<const float4*>(gp.rot_l),
                       reinterpret_cast<const float4*>(gp.rot_r), gp.opacity, gp.sh, views, S,
                       rec, tiles, dkey, gp.mask, gp.mask_thr, CompactPtrs{});
}

template <int DS, int DT>
__global__ __launch_bounds__(256) void k_decode_compact(int n, CompactPtrs cp,
                                                        float4* __restrict__ mean4,
                                                        float4* __restrict__ scale4,
                                                        float4* __restrict__ rot_l,
                                                        float4* __restrict__ rot_r,
                                                        float* __restrict__ opacity,
                                                        float* __restrict__ sh) {
  constexpr int NSH = (DT + 1) * (DS + 1) * (DS + 1) * 3;
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  float4 m, s4, a, b;
  float op, shc[NSH];
  decode_compact<NSH>(cp, gi, m, s4, a, b, op, shc);
  mean4[gi] = m;
  scale4[gi] = s4;
  rot_l[gi] = a;
  rot_r[gi] = b;
  opacity[gi] = op;
  float* o = sh + (size_t)gi * NSH;
#pragma unroll
  for (int k = 0; k < NSH; ++k) o[k] = shc[k];
}

template <int DS, int DT>
void launch_decode(int n, const CompactPtrs& cp, float* mean4, float* scale4, float* rot_l,
                   float* rot_r, float* opacity, float* sh, hipStream_t st) {
  hipLaunchKernelGGL((k_decode_compact<DS, DT>), dim3((n + 255) / 256), dim3(256), 0, st, n, cp,
                     reinterpret_cast<float4*>(mean4), reinterpret_cast<float4*>(scale4),
                     reinterpret_cast<float4*>(rot_l), reinterpret_cast<float4*>(rot_r), opacity,
                     sh);
}

template <int DS>
void dispatch_decode_t(int n, int dt, const CompactPtrs& cp, float* mean4, float* scale4,
                       float* rot_l, float* rot_r, float* opacity, float* sh, hipStream_t st) {
  switch (dt) {
    case 0: launch_decode<DS, 0>(n, cp, mean4, scale4, rot_l, rot_r, opacity, sh, st); break;
    case 1: launch_decode<DS, 1>(n, cp, mean4, scale4, rot_l, rot_r, opacity, sh, st); break;
    default: launch_decode<DS, 2>(n, cp, mean4, scale4, rot_l, rot_r, opacity, sh, st); break;
  }
}

template <int DS, int DT>
void launch_bwd(const GaussPtrs& gp, const DView* views, int n_views, DSettings S,
                const uint32_t* tiles, const float* grad2d, const GradPtrs& out, hipStream_t st) {
  const int blocks = (gp.n + 255) / 256;
  hipLaunchKernelGGL((k_preprocess_bwd<DS, DT>), dim3(blocks), dim3(256), 0, st, gp.n, n_views,
                     reinterpret_cast<const float4*>(gp.mean4),
                     reinterpret_cast<const float4*>(gp.scale4),
                     reinterpret_cast<const float4*>(gp.rot_l),
                     reinterpret_cast<const float4*>(gp.rot_r), gp.opacity, gp.sh, views, S,
                     tiles, grad2d, out);
}

template <int DS>
void dispatch_fwd_t(const GaussPtrs& gp, const DView* views, int nv, DSettings S, float* rec,
                    uint32_t* tiles, uint32_t* dkey, hipStream_t st) {
  switch (gp.t_degree) {
    case 0: launch_fwd<DS, 0>(gp, views, nv, S, rec, tiles, dkey, st); break;
    case 1: launch_fwd<DS, 1>(gp, views, nv, S, rec, tiles, dkey, st); break;
    default: launch_fwd<DS, 2>(gp, views, nv, S, rec, tiles, dkey, st); break;
  }
}

template <int DS>
void dispatch_bwd_t(const GaussPtrs& gp, const DView* views, int nv, DSettings S,
                    const uint32_t* tiles, const float* grad2d, const GradPtrs& out,
                    hipStream_t st) {
  switch (gp.t_degree) {
    case 0: launch_bwd<DS, 0>(gp, views, nv, S, tiles, grad2d, out, st); break;
    case 1: launch_bwd<DS, 1>(gp, views, nv, S, tiles, grad2d, out, st); break;
    default: launch_bwd<DS, 2>(gp, views, nv, S, tiles, grad2d, out, st); break;
  }
}

}  // namespace

void preprocess_forward(const GaussPtrs& gp, const DView* views, int n_views, DSettings S,
                        float* rec, uint32_t* tiles, uint32_t* dkey, hipStream_t st) {
  if (gp.n == 0) return;
  switch (gp.sh_degree) {
    case 0: dispatch_fwd_t<0>(gp, views, n_views, S, rec, tiles, dkey, st); break;
    case 1: dispatch_fwd_t<1>(gp, views, n_views, S, rec, tiles, dkey, st); break;
    case 2: dispatch_fwd_t<2>(gp, views, n_views, S, rec, tiles, dkey, st); break;
    default: dispatch_fwd_t<3>(gp, views, n_views, S, rec, tiles, dkey, st); break;
  }
}

void decode_compact_params(int n, int sh_degree, int t_degree, const CompactPtrs& cp,
                           float* mean4, float* scale4, float* rot_l, float* rot_r,
                           float* opacity, float* sh, hipStream_t st) {
  if (n <= 0) return;
  switch (sh_degree) {
    case 0: dispatch_decode_t<0>(n, t_degree, cp, mean4, scale4, rot_l, rot_r, opacity, sh, st); break;
    case 1: dispatch_decode_t<1>(n, t_degree, cp, mean4, scale4, rot_l, rot_r, opacity, sh, st); break;
    case 2: dispatch_decode_t<2>(n, t_degree, cp, mean4, scale4, rot_l, rot_r, opacity, sh, st); break;
    default: dispatch_decode_t<3>(n, t_degree, cp, mean4, scale4, rot_l, rot_r, opacity, sh, st); break;
  }
}

void preprocess_backward(const GaussPtrs& gp, const DView* views, int n_views, DSettings S,
                         const uint32_t* tiles, const float* grad2d, const GradPtrs& out,
                         hipStream_t st) {
  if (gp.n == 0) return;
  switch (gp.sh_degree) {
    case 0: dispatch_bwd_t<0>(gp, views, n_views, S, tiles, grad2d, out, st); break;
    case 1: dispatch_bwd_t<1>(gp, views, n_views, S, tiles, grad2d, out, st); break;
    case 2: dispatch_bwd_t<2>(gp, views, n_views, S, tiles, grad2d, out, st); break;
    default: dispatch_bwd_t<3>(gp, views, n_views, S, tiles, grad2d, out, st); break;
  }
}

}  // namespace g4d
