// Device-side data layout and per-(Gaussian, view) math of the 4D Gaussian render for gfx950.
//
// Forward (Sec. 3.2 of arXiv 2412.20720):
//   R = L(q_l) R(q_r) from the normalized rotors (the 4D rotation as two isoclinic rotations),
//   M = R diag(s), Sigma = M M^T.
//   Conditional Gaussian at time t and marginal (Sec. 3.2 conditional mean / covariance, p(t)):
//     with m = row 4 of M, s44 = m.m = Sigma_44, sigma = M_{1:3} m^T = Sigma_{1:3,4},
//     mu_c = mu_{1:3} + sigma (t - mu_t) / s44,
//     Sigma_c = Sigma_{1:3,1:3} - sigma sigma^T / s44 = A A^T  with  A = M_{1:3} (I - m^T m / s44),
//     p(t) = exp(-(t - mu_t)^2 / (2 s44)).
//   The product form A A^T equals the printed Schur complement exactly but keeps FP32 away
//   from the cancellation of two large terms when space and time are strongly coupled.
//   EWA splat (Sec. 3.1 eq:meansplatting, eq:covsplatting): x = W mu_c + tau,
//     (u, v) = (fx x/z + cx, fy y/z + cy), Sigma_2d = (T A)(T A)^T + blur I with T = J W,
//     J the perspective Jacobian at the clamped (x/z, y/z).
//   4DSH color (Sec. 3.2): c = max(c_min, c_0 + sum_n cos(2 pi n dt / T) sum_lm k_nlm Y_lm(d)),
//     d = normalize(mu_c - camera centre), dt = t - mu_t.
// Backward: the hand-written adjoint of every step above, with the clamps' branches frozen.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace g4d {

constexpr int kRec = 12;      // floats per (view, Gaussian) record
constexpr int kGrad2d = 12;   // floats per (view, Gaussian) gradient slot (GradField, 10 used)

// Record layout (kRec floats).
enum RecField {
  R_U = 0, R_V = 1, R_A = 2, R_B = 3, R_C = 4, R_OPT = 5, R_R = 6, R_G = 7, R_BL = 8,
  R_EX = 9, R_EY = 10, R_DEPTH = 11
};
// Screen-space gradient slot layout: d/du, d/dv, d/da, d/db, d/dc, d/d(opacity p_t), d/drgb.
// G_DEPTH: dL/d(camera depth), from the depth channel of the extra-channel render (0 otherwise).
// The color adjoint replaces d/drgb by the color's dL/dmu_c (G_MUC, 3 floats) and writes its
// dL/d(t - mu_t) to G_DT, which the geometry adjoint then reads; fields 10 and 11 are zero
// between backwards.
enum GradField {
  G_U = 0, G_V = 1, G_A = 2, G_B = 3, G_C = 4, G_OPT = 5, G_R = 6, G_DEPTH = 9,
  G_MUC = 6, G_DT = 10
};

struct DView {
  float W[9];        // world-to-camera rotation, row-major
  float tau[3];
  float C[3];        // camera centre -W^T tau (filled on the device)
  float fx, fy, cx, cy, t;
  float bg[3];
  float xlo, xhi, ylo, yhi;  // Jacobian clamp of x/z and y/z (filled on the device)
  int32_t width, height, tiles_x, tiles_y;
  int32_t tile_base, pix_base;
  int32_t pad0, row_base;    // pad0: unused on the device; row_base: first global tile row
};

struct DSettings {
  float near_z, marginal_min, cutoff, cut2, blur, jac_margin;
  float alpha_min, alpha_max, T_min, color_offset, color_min, time_period;
  int32_t tile, tile_shift, lds_batch, px_per_lane, bwd_px_per_lane;
  int32_t cutoff_bins;  // bin and stage every splat within the plain cutoff (work counting)
};

// ------------------------------------------------------------------------------------------
// Real spherical harmonics without the Condon-Shortley phase, order l*l + l + m, m = -l..l,
// as polynomials of the unit direction (x, y, z).  Constants are the closed forms
// sqrt2 K_l^|m| times the polynomial factor of P_l^|m| and of cos/sin(m phi).
// ------------------------------------------------------------------------------------------
constexpr float kY0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kY1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
constexpr float kY2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float kY2b = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float kY2c = 0.54627421529603959f;  // sqrt(15 / pi) / 4
constexpr float kY3a = 0.59004358992664352f;  // sqrt(35 / (2 pi)) / 4
constexpr float kY3b = 2.8906114426405538f;   // sqrt(105 / pi) / 2
constexpr float kY3c = 0.45704579946446572f;  // sqrt(21 / (2 pi)) / 4
constexpr float kY3d = 0.37317633259011540f;  // sqrt(7 / pi) / 4
constexpr float kY3e = 1.4453057213202769f;   // sqrt(105 / pi) / 4

template <int DS>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kY0;
  if (DS >= 1) {
    Y[1] = kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = kY1 * x;
  }
  if (DS >= 2) {
    Y[4] = kY2a * x * y;
    Y[5] = kY2a * y * z;
    Y[6] = kY2b * (3.f * z * z - 1.f);
    Y[7] = kY2a * x * z;
    Y[8] = kY2c * (x * x - y * y);
  }
  if (DS >= 3) {
    Y[9] = kY3a * y * (3.f * x * x - y * y);
    Y[10] = kY3b * x * y * z;
    Y[11] = kY3c * y * (5.f * z * z - 1.f);
    Y[12] = kY3d * z * (5.f * z * z - 3.f);
    Y[13] = kY3c * x * (5.f * z * z - 1.f);
    Y[14] = kY3e * z * (x * x - y * y);
    Y[15] = kY3a * x * (x * x - 3.f * y * y);
  }
}

// Gradient of sum_k w[k] Y_k(x, y, z) with respect to (x, y, z) (as independent variables).
template <int DS>
__device__ __forceinline__ void sh_basis_vjp(float x, float y, float z, const float* w,
                                             float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.f;
  if (DS >= 1) {
    gy += kY1 * w[1];
    gz += kY1 * w[2];
    gx += kY1 * w[3];
  }
  if (DS >= 2) {
    gx += kY2a * y * w[4];
    gy += kY2a * x * w[4];
    gy += kY2a * z * w[5];
    gz += kY2a * y * w[5];
    gz += kY2b * 6.f * z * w[6];
    gx += kY2a * z * w[7];
    gz += kY2a * x * w[7];
    gx += kY2c * 2.f * x * w[8];
    gy -= kY2c * 2.f * y * w[8];
  }
  if (DS >= 3) {
    gx += kY3a * 6.f * x * y * w[9];
    gy += kY3a * (3.f * x * x - 3.f * y * y) * w[9];
    gx += kY3b * y * z * w[10];
    gy += kY3b * x * z * w[10];
    gz += kY3b * x * y * w[10];
    gy += kY3c * (5.f * z * z - 1.f) * w[11];
    gz += kY3c * 10.f * y * z * w[11];
    gz += kY3d * (15.f * z * z - 3.f) * w[12];
    gx += kY3c * (5.f * z * z - 1.f) * w[13];
    gz += kY3c * 10.f * x * z * w[13];
    gx += kY3e * 2.f * x * z * w[14];
    gy -= kY3e * 2.f * y * z * w[14];
    gz += kY3e * (x * x - y * y) * w[14];
    gx += kY3a * (3.f * x * x - 3.f * y * y) * w[15];
    gy -= kY3a * 6.f * x * y * w[15];
  }
}

// ------------------------------------------------------------------------------------------
// View-independent geometry: normalized rotors, R = L(q_l) R(q_r), M = R diag(s).
// ------------------------------------------------------------------------------------------
struct Geom {
  float ql[4], qr[4];   // normalized rotors
  float inl, inr;       // 1 / |q_l|, 1 / |q_r|
  float R[4][4];
  float M[4][4];
};

__device__ __forceinline__ void left_iso(const float* q, float L[4][4]) {
  const float a = q[0], b = q[1], c = q[2], d = q[3];
  L[0][0] = a;  L[0][1] = -b; L[0][2] = -c; L[0][3] = -d;
  L[1][0] = b;  L[1][1] = a;  L[1][2] = -d; L[1][3] = c;
  L[2][0] = c;  L[2][1] = d;  L[2][2] = a;  L[2][3] = -b;
  L[3][0] = d;  L[3][1] = -c; L[3][2] = b;  L[3][3] = a;
}

__device__ __forceinline__ void right_iso(const float* q, float P[4][4]) {
  const float p = q[0], qq = q[1], r = q[2], s = q[3];
  P[0][0] = p;  P[0][1] = -qq; P[0][2] = -r;  P[0][3] = -s;
  P[1][0] = qq; P[1][1] = p;   P[1][2] = s;   P[1][3] = -r;
  P[2][0] = r;  P[2][1] = -s;  P[2][2] = p;   P[2][3] = qq;
  P[3][0] = s;  P[3][1] = r;   P[3][2] = -qq; P[3][3] = p;
}

__device__ __forceinline__ void geom_forward(const float4 qlr, const float4 qrr, const float4 sc,
                                             Geom& g) {
  const float ql[4] = {qlr.x, qlr.y, qlr.z, qlr.w};
  const float qr[4] = {qrr.x, qrr.y, qrr.z, qrr.w};
  g.inl = rsqrtf(ql[0] * ql[0] + ql[1] * ql[1] + ql[2] * ql[2] + ql[3] * ql[3]);
  g.inr = rsqrtf(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
  for (int i = 0; i < 4; ++i) {
    g.ql[i] = ql[i] * g.inl;
    g.qr[i] = qr[i] * g.inr;
  }
  float L[4][4], P[4][4];
  left_iso(g.ql, L);
  right_iso(g.qr, P);
  const float s[4] = {sc.x, sc.y, sc.z, sc.w};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float acc = L[i][0] * P[0][j];
      acc = fmaf(L[i][1], P[1][j], acc);
      acc = fmaf(L[i][2], P[2][j], acc);
      acc = fmaf(L[i][3], P[3][j], acc);
      g.R[i][j] = acc;
      g.M[i][j] = acc * s[j];
    }
}

// ------------------------------------------------------------------------------------------
// Per-view forward state (kept for the adjoint).
// ------------------------------------------------------------------------------------------
struct ViewFwd {
  float inv_s, dt, k;        // 1 / Sigma_44, t - mu_t, dt / Sigma_44
  float sigma[3];            // Sigma_{1:3,4}
  float A[3][4];             // M_{1:3} (I - m^T m / Sigma_44)
  float muc[3], pt;
  float x[3], iz, rx, ry, txc, tyc;
  bool clx, cly;             // Jacobian argument clamped
  float Tm[2][3];            // J W
  float B[2][4];             // T A
  float cov[3];              // 2D covariance (blur included): xx, xy, yy
  float conic[3];
  float u, v;
  float dir[3], idn;         // unit view direction, 1 / |mu_c - C|
  float raw[3], color[3];
};

// Slice and splat; returns false when the Gaussian is culled in this view.  With kCull the
// function stops at the first cull; without it every field is computed (used by the adjoint,
// which must not depend on re-deciding a cull).
// View-independent slice constants: 1 / Sigma_44 and sigma = Sigma_{1:3,4} = M_{1:3} m^T.
__device__ __forceinline__ void slice_consts(const Geom& g, float& inv_s, float sigma[3]) {
  const float* m = g.M[3];
  const float s44 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2] + m[3] * m[3];
  inv_s = 1.f / s44;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float* Mi = g.M[i];
    sigma[i] = Mi[0] * m[0] + Mi[1] * m[1] + Mi[2] * m[2] + Mi[3] * m[3];
  }
}

// Conditional mean at the view's time (dt = t - mu_t, k = dt / Sigma_44) and the unit view
// direction from the camera centre (1 / |mu_c - C| in idn).  The forward, its recomputation
// in the adjoint and the color adjoint all call this, so they agree bit for bit.
__device__ __forceinline__ void slice_mean_dir(const float4 mean, float inv_s, const float* sigma,
                                               const DView& V, float& dt, float& k,
                                               float* muc, float* dir, float& idn) {
  dt = V.t - mean.w;
  k = dt * inv_s;
  const float mu[3] = {mean.x, mean.y, mean.z};
#pragma unroll
  for (int i = 0; i < 3; ++i) muc[i] = fmaf(sigma[i], k, mu[i]);
  float d[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) d[i] = muc[i] - V.C[i];
  idn = rsqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i) dir[i] = d[i] * idn;
}

template <bool kCull = true>
__device__ __forceinline__ bool view_forward(const Geom& g, const float4 mean, const DView& V,
                                             const DSettings& S, ViewFwd& f) {
  bool alive = true;
  const float* m = g.M[3];
  slice_consts(g, f.inv_s, f.sigma);
  slice_mean_dir(mean, f.inv_s, f.sigma, V, f.dt, f.k, f.muc, f.dir, f.idn);
  f.pt = __expf(-0.5f * f.dt * f.k);
  if (!(f.pt >= S.marginal_min)) {
    if (kCull) return false;
    alive = false;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float* Mi = g.M[i];
    const float c = f.sigma[i] * f.inv_s;
#pragma unroll
    for (int j = 0; j < 4; ++j) f.A[i][j] = fmaf(-c, m[j], Mi[j]);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
    f.x[i] = fmaf(V.W[3 * i + 0], f.muc[0],
                  fmaf(V.W[3 * i + 1], f.muc[1], fmaf(V.W[3 * i + 2], f.muc[2], V.tau[i])));
  if (!(f.x[2] > S.near_z)) {
    if (kCull) return false;
    alive = false;
  }
  f.iz = 1.f / f.x[2];
  f.rx = f.x[0] * f.iz;
  f.ry = f.x[1] * f.iz;
  f.u = fmaf(V.fx, f.rx, V.cx);
  f.v = fmaf(V.fy, f.ry, V.cy);
  f.clx = !(f.rx >= V.xlo && f.rx <= V.xhi);
  f.cly = !(f.ry >= V.ylo && f.ry <= V.yhi);
  f.txc = fminf(fmaxf(f.rx, V.xlo), V.xhi);
  f.tyc = fminf(fmaxf(f.ry, V.ylo), V.yhi);
  const float ax = V.fx * f.iz, ay = V.fy * f.iz;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    f.Tm[0][j] = ax * fmaf(-f.txc, V.W[6 + j], V.W[j]);
    f.Tm[1][j] = ay * fmaf(-f.tyc, V.W[6 + j], V.W[3 + j]);
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      f.B[r][j] = fmaf(f.Tm[r][0], f.A[0][j], fmaf(f.Tm[r][1], f.A[1][j], f.Tm[r][2] * f.A[2][j]));
  float cxx = 0.f, cxy = 0.f, cyy = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    cxx = fmaf(f.B[0][j], f.B[0][j], cxx);
    cxy = fmaf(f.B[0][j], f.B[1][j], cxy);
    cyy = fmaf(f.B[1][j], f.B[1][j], cyy);
  }
  f.cov[0] = cxx + S.blur;
  f.cov[1] = cxy;
  f.cov[2] = cyy + S.blur;
  const float det = f.cov[0] * f.cov[2] - f.cov[1] * f.cov[1];
  if (!(det > 0.f) || !isfinite(det) || !isfinite(f.u) || !isfinite(f.v)) {
    if (kCull) return false;
    alive = false;
  }
  const float idet = 1.f / det;
  f.conic[0] = f.cov[2] * idet;
  f.conic[1] = -f.cov[1] * idet;
  f.conic[2] = f.cov[0] * idet;
  return alive;
}

// Fourier factor cos(2 pi n dt / T) of the 4DSH time basis (1 for n = 0).
__device__ __forceinline__ float fourier_cos(int n, float dt, const DSettings& S) {
  return (n == 0) ? 1.f : __cosf(6.283185307179586f * (float)n * dt / S.time_period);
}

// 4DSH color of one view; `sh` holds the (DT+1) x (DS+1)^2 x 3 coefficients of the Gaussian.
template <int DS, int DT>
__device__ __forceinline__ void color_forward(const float* sh, const DSettings& S, ViewFwd& f) {
  constexpr int NK = (DS + 1) * (DS + 1);
  float Y[NK];
  sh_basis<DS>(f.dir[0], f.dir[1], f.dir[2], Y);
  float acc[3] = {S.color_offset, S.color_offset, S.color_offset};
#pragma unroll
  for (int n = 0; n <= DT; ++n) {
    const float fn = fourier_cos(n, f.dt, S);
    float in[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < NK; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) in[ch] = fmaf(sh[(n * NK + k) * 3 + ch], Y[k], in[ch]);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) acc[ch] = fmaf(fn, in[ch], acc[ch]);
  }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    f.raw[ch] = acc[ch];
    f.color[ch] = fmaxf(acc[ch], S.color_min);
  }
}

// Squared Mahalanobis radius within which a splat of opacity * p_t = opt can be composited:
// the cutoff^2, or less where alpha = opt exp(-d2 / 2) drops below alpha_min first, at
// d2 = 2 ln(opt / alpha_min).  That bound is widened by 1e-3 relative plus 2e-3 absolute, so
// that no pixel whose FP32 alpha passes alpha_min is ever left out; a result <= 0 means the splat
// cannot be composited anywhere.  Binning the splat with this radius instead of the cutoff
// leaves every image and gradient unchanged and drops the (tile, splat) pairs and the per-pixel
// evaluations that could only fail the alpha_min test.  The preprocess (counting) and the key
// generation (writing) evaluate it on the same stored opt with the same instructions.  With
// S.cutoff_bins (a work-counting forward) the bound is the cutoff itself, so the counting raster
// visits every candidate within the cutoff, as the plain definition of the render does.
__device__ __forceinline__ float reach2(float opt, const DSettings& S) {
  if (S.cutoff_bins) return S.cut2;
  return fminf(S.cut2, fmaf(2.002f, logf(opt / S.alpha_min), 2e-3f));
}

// Box of the ellipse d2 <= r2, widened by 5e-4 relative so that FP32 rounding never drops a
// pixel whose exact Mahalanobis distance passes the bound.
__device__ __forceinline__ void reach_extent(const ViewFwd& f, float r2, float& ex, float& ey) {
  ex = sqrtf(r2 * f.cov[0]) * 1.0005f;
  ey = sqrtf(r2 * f.cov[2]) * 1.0005f;
}

// Tiles whose pixel centres can lie inside [u - ex, u + ex] x [v - ey, v + ey]:
// (x0, x1, y0, y1), or x0 = -1 if none.  Not inlined: the preprocess (counting) and the key
// generation (writing) must see exactly the rounded u, v, ex, ey, never a product fused into
// the subtraction.
__device__ __noinline__ int4 tile_rect_of(float u, float v, float ex, float ey, int width,
                                          int height, int shift) {
  float fx0 = ceilf(u - ex - 0.5f), fx1 = floorf(u + ex - 0.5f);
  float fy0 = ceilf(v - ey - 0.5f), fy1 = floorf(v + ey - 0.5f);
  fx0 = fmaxf(fx0, 0.f);
  fy0 = fmaxf(fy0, 0.f);
  fx1 = fminf(fx1, (float)(width - 1));
  fy1 = fminf(fy1, (float)(height - 1));
  if (!(fx0 <= fx1) || !(fy0 <= fy1)) return make_int4(-1, -1, -1, -1);
  return make_int4((int)fx0 >> shift, (int)fx1 >> shift, (int)fy0 >> shift, (int)fy1 >> shift);
}

__device__ __forceinline__ bool tile_rect(float u, float v, float ex, float ey, const DView& V,
                                          int shift, int& x0, int& x1, int& y0, int& y1) {
  const int4 r = tile_rect_of(u, v, ex, ey, V.width, V.height, shift);
  x0 = r.x;
  x1 = r.y;
  y0 = r.z;
  y1 = r.w;
  return r.x >= 0;
}

// x-range [xl, xr] (relative to the splat centre) of the ellipse a dx^2 + 2 b dx dy + c dy^2
// <= lim over the band dy in [dy0, dy1]; false if the band misses it.  ex, ey are the
// ellipse's (already widened) half extents.  For fixed dy the ellipse spans
// dx = -b dy / a +- sqrt(lim a - D dy^2) / a with D = ac - b^2; over a band the leftmost
// (rightmost) x is the ellipse's own extreme -ex (+ex) if the band contains its height
// dy = b ex / c (-b ex / c), else it is reached at an end of the band.  When D is tiny next to
// ac (a thin, tilted ellipse) FP32 cannot resolve the chords and the full box is returned.
__device__ __forceinline__ bool ellipse_band_xrange(float a, float b, float c, float lim,
                                                    float ex, float ey, float dy0, float dy1,
                                                    float& xl, float& xr) {
  if (!(dy1 >= -ey) || !(dy0 <= ey)) return false;
  const float D = a * c - b * b;
  if (!(D > 1e-3f * a * c)) {
    xl = -ex;
    xr = ex;
    return true;
  }
  dy0 = fmaxf(dy0, -ey);
  dy1 = fminf(dy1, ey);
  const float ia = 1.f / a;
  const float dyl = b * ex / c;
  const float sl = -b * ia;
  const float h0 = sqrtf(fmaxf(0.f, lim * a - D * dy0 * dy0)) * ia;
  const float h1 = sqrtf(fmaxf(0.f, lim * a - D * dy1 * dy1)) * ia;
  xl = (dyl >= dy0 && dyl <= dy1) ? -ex : fminf(sl * dy0 - h0, sl * dy1 - h1);
  xr = (-dyl >= dy0 && -dyl <= dy1) ? ex : fmaxf(sl * dy0 + h0, sl * dy1 + h1);
  return true;
}

// Tile columns of tile row `ty` that hold a pixel centre the splat's cutoff ellipse (slightly
// widened) can reach, clipped to [tx0, tx1]: returns (first << 16) | last, or -1 if none.
// Not inlined, so that the preprocess (which counts the pairs) and the splats -> rows write
// (which lays the runs of columns down) run the very same instructions and always agree.
__device__ __noinline__ int tile_row_span(float u, float v, float a, float b, float c, float lim,
                                          float ex, float ey, int ty, int shift, int width,
                                          int height, int tx0, int tx1) {
  const int T = 1 << shift;
  const float y0 = (float)(ty * T) + 0.5f;
  const float y1 = fminf((float)(ty * T + T) - 0.5f, (float)height - 0.5f);
  float xl, xr;
  if (!ellipse_band_xrange(a, b, c, lim, ex, ey, y0 - v, y1 - v, xl, xr)) return -1;
  float px0 = ceilf(u + xl - 0.5f - 1e-2f), px1 = floorf(u + xr - 0.5f + 1e-2f);
  px0 = fmaxf(px0, 0.f);
  px1 = fminf(px1, (float)(width - 1));
  if (!(px0 <= px1)) return -1;
  const int c0 = max((int)px0 >> shift, tx0), c1 = min((int)px1 >> shift, tx1);
  return c0 <= c1 ? (c0 << 16) | c1 : -1;
}

// Inclusive scan under `op` (identity id) over the 64 lanes of a wave, all lanes active.  It
// stays in registers: DPP moves add the values 1, 2, 4 and 8 lanes below within each row of 16
// lanes, then the last lane of rows 0 and 2 to the rows above them (row_bcast:15, rows 1 and 3)
// and lane 31 to rows 2 and 3 (row_bcast:31).  A lane a move does not write keeps id.
template <class Op>
__device__ __forceinline__ uint32_t wave_scan_op(uint32_t x, uint32_t id, Op op) {
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x111, 0xf, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x112, 0xf, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x114, 0xf, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x118, 0xf, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x142, 0xa, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, 0x143, 0xc, 0xf, false));
  return x;
}

// Inclusive and exclusive prefix sums over the 64 lanes of a wave (all lanes active); the
// exclusive one also returns the wave total.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  return wave_scan_op(x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t& total) {
  const uint32_t inc = wave_incl_scan(x);
  total = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
  return inc - x;
}

// Owner of item k0 + lane in a window of 64 items (k0 a multiple of 64), where lane l holds the
// items [first_l, first_l + count_l), numbered in lane order with no gaps: the last lane whose
// run starts at or before the item.  Each lane whose run starts in the window marks its start
// in the wave's 64-word LDS array `mark` with the round's stamp, and a max scan carries each
// mark up to the next; `carry` passes the owner of the window's last item on to the next window
// (-1 before the first window of a numbering), `stamp` is a wave-uniform counter, 1 or more,
// that no earlier call of the wave used (the array starts at 0).  Every lane of the wave calls
// it; for every item below the total the owner is a lane with count > 0.
__device__ __forceinline__ int window_owner(uint32_t first, uint32_t count, uint32_t k0,
                                            uint32_t* mark, uint32_t& stamp, int& carry) {
  const int lane = threadIdx.x & 63;
  if (count > 0u && first - k0 < 64u) mark[first - k0] = (stamp << 6) | (uint32_t)lane;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t m = mark[lane];
  // owner + 1, so that 0 (no mark) is the identity of the max
  uint32_t o = (m >> 6) == stamp ? (m & 63u) + 1u : 0u;
  o = wave_scan_op(o, 0u, [](uint32_t a, uint32_t b) { return max(a, b); });
  int own = max((int)o - 1, carry);
  carry = __builtin_amdgcn_readlane(own, 63);
  ++stamp;
  return own < 0 ? 0 : own;
}

// Bound used for tile coverage: 1e-3 above reach2, so that FP32 rounding in the coverage test
// never drops a pixel whose exact Mahalanobis distance passes it.
__device__ __forceinline__ float coverage_limit(float opt, const DSettings& S) {
  return reach2(opt, S) * 1.001f;
}

// ------------------------------------------------------------------------------------------
// Adjoint of one view, geometry part.  Inputs: the screen-space gradient q (u, v, conic a, b,
// c, opacity p_t at G_U..G_OPT, camera depth at G_DEPTH), the color's contribution to dL/dmu_c
// (gmuc_color) and to dL/d(dt) (gdt_color) through the view direction and the Fourier factors,
// and the forward state f.  Outputs are accumulated: gM (4x4, w.r.t. M), gmean (4), gopacity.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void view_backward_geom(const Geom& g, float opacity, const DView& V,
                                                   const ViewFwd& f, const float* q,
                                                   const float* gmuc_color, float gdt_color,
                                                   float gM[4][4], float gmean[4],
                                                   float& gopacity) {
  float gmuc[3] = {gmuc_color[0], gmuc_color[1], gmuc_color[2]};
  const float gdt = gdt_color;
  // ---- opacity * p_t ----
  gopacity = fmaf(q[G_OPT], f.pt, gopacity);
  float gpt = q[G_OPT] * opacity;
  // ---- conic = inverse(cov) ----
  const float a = f.conic[0], b = f.conic[1], c = f.conic[2];
  const float ga = q[G_A], gb = 0.5f * q[G_B], gc = q[G_C];
  const float P00 = a * ga + b * gb, P01 = a * gb + b * gc;
  const float P10 = b * ga + c * gb, P11 = b * gb + c * gc;
  const float gS00 = -(P00 * a + P01 * b);
  const float gS01 = -(P00 * b + P01 * c);
  const float gS11 = -(P10 * b + P11 * c);
  // cov = B B^T + blur I  ->  gB = 2 gS B
  float gB[2][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    gB[0][j] = 2.f * (gS00 * f.B[0][j] + gS01 * f.B[1][j]);
    gB[1][j] = 2.f * (gS01 * f.B[0][j] + gS11 * f.B[1][j]);
  }
  // B = Tm A  ->  gTm = gB A^T, gA = Tm^T gB
  float gTm[2][3], gA[3][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      gTm[r][i] = gB[r][0] * f.A[i][0] + gB[r][1] * f.A[i][1] + gB[r][2] * f.A[i][2] +
                  gB[r][3] * f.A[i][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) gA[i][j] = f.Tm[0][i] * gB[0][j] + f.Tm[1][i] * gB[1][j];
  // Tm[0][j] = fx iz (W0j - txc W2j); Tm[1][j] = fy iz (W1j - tyc W2j)
  float giz = 0.f, gtxc = 0.f, gtyc = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    giz = fmaf(gTm[0][j], V.fx * fmaf(-f.txc, V.W[6 + j], V.W[j]), giz);
    giz = fmaf(gTm[1][j], V.fy * fmaf(-f.tyc, V.W[6 + j], V.W[3 + j]), giz);
    gtxc = fmaf(-gTm[0][j], V.fx * f.iz * V.W[6 + j], gtxc);
    gtyc = fmaf(-gTm[1][j], V.fy * f.iz * V.W[6 + j], gtyc);
  }
  float gx[3] = {0.f, 0.f, 0.f};
  // screen mean u = fx x iz + cx, v = fy y iz + cy; clamped Jacobian arguments are frozen
  const float grx = q[G_U] * V.fx + (f.clx ? 0.f : gtxc);
  const float gry = q[G_V] * V.fy + (f.cly ? 0.f : gtyc);
  gx[0] = grx * f.iz;
  gx[1] = gry * f.iz;
  giz = fmaf(grx, f.x[0], fmaf(gry, f.x[1], giz));
  gx[2] = fmaf(-giz * f.iz, f.iz, q[G_DEPTH]);
  // x = W mu_c + tau
#pragma unroll
  for (int j = 0; j < 3; ++j) gmuc[j] += V.W[j] * gx[0] + V.W[3 + j] * gx[1] + V.W[6 + j] * gx[2];
  // ---- slice ----
  const float* m = g.M[3];
  float gsig[3], gm[4] = {0.f, 0.f, 0.f, 0.f};
  float gk = 0.f, ginv = 0.f, gdt2 = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    gmean[i] += gmuc[i];
    gsig[i] = gmuc[i] * f.k;
    gk = fmaf(gmuc[i], f.sigma[i], gk);
  }
  gdt2 += gk * f.inv_s;
  ginv += gk * f.dt;
  // A = M1 - sigma m / s44
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float gAm = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gM[i][j] += gA[i][j];
      gAm = fmaf(gA[i][j], m[j], gAm);
      gm[j] = fmaf(-f.inv_s * f.sigma[i], gA[i][j], gm[j]);
    }
    gsig[i] = fmaf(-f.inv_s, gAm, gsig[i]);
    ginv = fmaf(-f.sigma[i], gAm, ginv);
  }
  // p_t = exp(-dt^2 inv_s / 2)
  gdt2 = fmaf(gpt * f.pt, -f.dt * f.inv_s, gdt2);
  ginv = fmaf(gpt * f.pt, -0.5f * f.dt * f.dt, ginv);
  // sigma = M1 m
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gM[i][j] = fmaf(gsig[i], m[j], gM[i][j]);
      gm[j] = fmaf(gsig[i], g.M[i][j], gm[j]);
    }
  // inv_s = 1 / (m.m)
  const float gs = -ginv * f.inv_s * f.inv_s;
#pragma unroll
  for (int j = 0; j < 4; ++j) gM[3][j] += fmaf(2.f * gs, m[j], gm[j]);
  // dt = t - mu_t (slice, marginal and Fourier basis)
  gmean[3] -= gdt2 + gdt;
}

// Compact 4DGS decode of one Gaussian (residual VQ: the sum of one codeword per codebook,
// summed in codebook order; half positions; 8-bit min-max opacity).  NSH = the 4DSH
// coefficient count K; the direct component fills sh[0..2], the rest sh[3..K-1].
struct CompactPtrs {
  const uint16_t* mean4_h;
  const uint8_t *scale_idx, *rot_l_idx, *rot_r_idx, *opacity_q, *dc_idx, *rest_idx;
  float op_lo, op_hi;
  const float *scale_cb, *rot_cb, *dc_cb, *rest_cb;
};

template <int NSH>
__device__ __forceinline__ void decode_compact(const CompactPtrs& c, int i, float4& mean,
                                               float4& scale, float4& ql, float4& qr, float& op,
                                               float* sh) {
  const uint16_t* mh = c.mean4_h + 4 * (size_t)i;
  mean = make_float4((float)__builtin_bit_cast(_Float16, mh[0]),
                     (float)__builtin_bit_cast(_Float16, mh[1]),
                     (float)__builtin_bit_cast(_Float16, mh[2]),
                     (float)__builtin_bit_cast(_Float16, mh[3]));
  float ls[4] = {0.f, 0.f, 0.f, 0.f}, l[4] = {0.f, 0.f, 0.f, 0.f}, r[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float4 a = reinterpret_cast<const float4*>(c.scale_cb)[k * 64 + c.scale_idx[6 * (size_t)i + k]];
    const float4 b = reinterpret_cast<const float4*>(c.rot_cb)[k * 64 + c.rot_l_idx[6 * (size_t)i + k]];
    const float4 d = reinterpret_cast<const float4*>(c.rot_cb)[k * 64 + c.rot_r_idx[6 * (size_t)i + k]];
    ls[0] += a.x; ls[1] += a.y; ls[2] += a.z; ls[3] += a.w;
    l[0] += b.x; l[1] += b.y; l[2] += b.z; l[3] += b.w;
    r[0] += d.x; r[1] += d.y; r[2] += d.z; r[3] += d.w;
  }
  scale = make_float4(expf(ls[0]), expf(ls[1]), expf(ls[2]), expf(ls[3]));
  ql = make_float4(l[0], l[1], l[2], l[3]);
  qr = make_float4(r[0], r[1], r[2], r[3]);
  op = fmaf(c.op_hi - c.op_lo, (float)c.opacity_q[i] * (1.f / 255.f), c.op_lo);
#pragma unroll
  for (int j = 0; j < NSH; ++j) sh[j] = 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float* w = c.dc_cb + 3 * (k * 64 + c.dc_idx[6 * (size_t)i + k]);
    sh[0] += w[0];
    sh[1] += w[1];
    sh[2] += w[2];
  }
  constexpr int KR = NSH - 3;
  if constexpr (KR > 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float* w = c.rest_cb + (size_t)KR * (k * 256 + c.rest_idx[8 * (size_t)i + k]);
#pragma unroll
      for (int j = 0; j < KR; ++j) sh[3 + j] += w[j];
    }
  }
}

// Adjoint of geom_forward: from gM (4x4) to the scale and the raw rotors.
__device__ __forceinline__ void geom_backward(const Geom& g, const float4 sc, const float gM[4][4],
                                              float gscale[4], float gql[4], float gqr[4]) {
  const float s[4] = {sc.x, sc.y, sc.z, sc.w};
  float gR[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      gR[i][j] = gM[i][j] * s[j];
      acc = fmaf(gM[i][j], g.R[i][j], acc);
    }
    gscale[j] = acc;
  }
  float L[4][4], P[4][4];
  left_iso(g.ql, L);
  right_iso(g.qr, P);
  // R = L P  ->  gL = gR P^T, gP = L^T gR
  float gL[4][4], gP[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float a = 0.f, b = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        a = fmaf(gR[i][k], P[j][k], a);
        b = fmaf(L[k][i], gR[k][j], b);
      }
      gL[i][j] = a;
      gP[i][j] = b;
    }
  float hl[4], hr[4];
  hl[0] = gL[0][0] + gL[1][1] + gL[2][2] + gL[3][3];
  hl[1] = -gL[0][1] + gL[1][0] - gL[2][3] + gL[3][2];
  hl[2] = -gL[0][2] + gL[1][3] + gL[2][0] - gL[3][1];
  hl[3] = -gL[0][3] - gL[1][2] + gL[2][1] + gL[3][0];
  hr[0] = gP[0][0] + gP[1][1] + gP[2][2] + gP[3][3];
  hr[1] = -gP[0][1] + gP[1][0] + gP[2][3] - gP[3][2];
  hr[2] = -gP[0][2] - gP[1][3] + gP[2][0] + gP[3][1];
  hr[3] = -gP[0][3] + gP[1][2] - gP[2][1] + gP[3][0];
  // q_hat = q / |q|  ->  g_q = (g_hat - q_hat (q_hat . g_hat)) / |q|
  const float dl = hl[0] * g.ql[0] + hl[1] * g.ql[1] + hl[2] * g.ql[2] + hl[3] * g.ql[3];
  const float dr = hr[0] * g.qr[0] + hr[1] * g.qr[1] + hr[2] * g.qr[2] + hr[3] * g.qr[3];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gql[i] = (hl[i] - g.ql[i] * dl) * g.inl;
    gqr[i] = (hr[i] - g.qr[i] * dr) * g.inr;
  }
}

}  // namespace g4d
