// FP64 CPU oracle of the differentiable render of native 4D Gaussians.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
// benchmark may load this library.  It shares no code, header, table or helper with the GPU
// library and never reads anything the GPU library produced.
//
// What it computes, step by step, in double precision (arXiv 2412.20720):
//   O1  rotors normalized: q_l / |q_l|, q_r / |q_r| (isoclinic rotations need unit quaternions,
//       Sec. 3.2 "Representation of 4D Gaussian").
//   O2  R = L(q_l) R(q_r) with the two 4x4 quaternion-multiplication matrices of Sec. 3.2.
//   O3  Sigma = R S S^T R^T, S = diag(s_x, s_y, s_z, s_t) (Sec. 3.2).
//   O4  conditional 3D Gaussian and temporal marginal at time t (Sec. 3.2, the conditional mean
//       and covariance equations and p(t) = N(t; mu_4, Sigma_44)), all unnormalized
//       (Sec. 3.1, eq. gaussianfunction).
//   O5  culls: p(t) below the marginal threshold (Sec. 8.1 implementation details), then the
//       near plane.
//   O6  EWA splatting: mean = Proj(mu | E, K)_{1:2} (eq. meansplatting),
//       Sigma2d = (J W Sigma W^T J^T)_{1:2,1:2} + blur I (eq. covsplatting), conic = inverse.
//   O7  color from 4D spherindrical harmonics Z = cos(2 pi n dt / T) Y_l^m(d) (Sec. 3.2,
//       "4D spherindrical harmonics"), offset and clamped below.
//   O8-O10  per pixel: candidates with Mahalanobis distance within the cutoff, sorted by
//       (camera depth, index), composited front to back (eq. eq:4dblending):
//       alpha = min(alpha_max, o p(t) p(u,v|t)); skip alpha < alpha_min; stop before the
//       Gaussian that would take transmittance below T_min; add T * background at the end.
//   O11 backward: exact derivative of O1-O10 with every discrete decision frozen.  The
//       per-pixel part is a reverse sweep over stored FP64 prefix transmittances (no division);
//       the per-Gaussian part uses forward-mode dual numbers over the 17 geometry parameters;
//       the SH part is linear in the coefficients.
//
// The only acceleration is a conservative candidate search: a Gaussian is tested against a
// pixel only if the pixel lies in the bounding box of its cutoff ellipse (widened by the
// parity margin).  The box provably contains every pixel whose Mahalanobis distance passes the
// cutoff, so candidate sets and all arithmetic are those of the definition; a test checks the
// binned search against an exhaustive all-pairs loop.
//
// Volume mask (optional, Sec. 4.3 "Insignificant Gaussian removal"): M_hat = 1{M > eps} in the
// forward with the straight-through derivative dM_hat/dM = 1; S_hat = M_hat S, alpha_hat =
// M_hat alpha.  A masked Gaussian (M_hat = 0) is dropped (its zero covariance has no slice);
// for the others dL/dM = sum_j s_j dL/ds_j + o dL/do.  Densification statistic (Sec. 3.3,
// densification in spacetime): per view, |dL/d mean2d| of every Gaussian alive in it; the
// |dL/d mu_t| indicator is the mean4 gradient's time component.
//
// Compact 4DGS decode (Sec. 4.2 parameter compression; codebook sizes of Sec. 8.3): residual
// vector quantization sums one codeword of each codebook, x = sum_k C_k[i_k]: scale (6 x 64,
// in log space, s = exp(x) -- reading: the scale is quantized before its activation), rotors
// (one 6 x 64 model shared by q_l and q_r, each with its own indices), 4DSH direct component
// (6 x 64) and the rest (8 x 256); positions stored as IEEE half; opacity by 8-bit min-max
// quantization, o = lo + (hi - lo) q / 255.
//
// Sky (optional, Sec. 5, urban scenes): I = I_gs + (1 - O_gs) M_sky(r) = C + T M_sky(r), a cube
// map queried by the world direction r of the pixel's ray (the background of that pixel).
// Readings: the OpenGL cube-map convention (faces +x, -x, +y, -y, +z, -z; the major axis of r
// picks the face, ties to x before y before z; face coordinates s = (sc / |ma| + 1) / 2,
// t = (tc / |ma| + 1) / 2 with (sc, tc) from the published face table), texel (i, j) centred
// at ((i + 1/2) / R, (j + 1/2) / R), bilinear within the face, clamped at its edges.
//
// Extra channels (optional, orc_frame_set_channels), composited with the same weights T alpha:
//   features: per Gaussian f in R^D gated by a per-call vector g (the scale gate S(s)) and
//       normalized, f_hat = (g * f) / |g * f| (0 where g * f = 0) -- the color replaced by the
//       normalized scale-gated feature (Sec. 7, segment anything in 4D);
//   depth: the camera-space z of the sliced mean (the rendered depth of the urban LiDAR loss,
//       Sec. 5, urban scenes);
//   flow: the image-plane displacement of the projected conditional mean between t and
//       t + dt (Sec. 8.1, the emerged scene dynamics), 0 where the moved mean is not in front
//       of the camera.
//   The extra channels have a zero background.  Their backward differentiates the features,
//   the gate and the depth; flow is forward only (its upstream gradient is ignored).
//
// Failure rule (a reading; the paper has none): a Gaussian with a non-finite parameter is
// dropped in every view and gets no gradient.
//
// Readings where the paper is silent (defaults chosen by the caller through orc_settings):
// unnormalized Gaussians; opacity clamp alpha_max and skip threshold alpha_min; transmittance
// stop T_min; per-pixel Mahalanobis cutoff; EWA low-pass "blur"; Jacobian clamp margin;
// pixel centres at half-integers; view direction from the camera centre to the sliced mean;
// depth = camera-space z of the sliced mean, ties by Gaussian index; temporal basis cosine-only
// with argument dt = t - mu_t and period T; real SH without the Condon-Shortley phase.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

typedef struct {
  int32_t n, sh_degree, t_degree;
  const double *mean4, *scale4, *rot_l, *rot_r, *opacity, *sh;
  const double* mask;     // [n] significance M (NULL: no mask)
  double mask_threshold;  // epsilon
} orc_gaussians;

typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
  double world_to_cam[12];  // [R | tau] row-major
  double t;
  double background[3];
} orc_view;

typedef struct {
  double near_z, marginal_min, cutoff_sigma, blur, jacobian_margin;
  double alpha_min, alpha_max, T_min, color_offset, color_min, time_period;
  // Parity margins: a decision whose deciding quantity lies within this relative distance of
  // its threshold is "marked" (FP32 and FP64 may legitimately take different sides).
  double margin_d2, margin_alpha, margin_T, margin_depth, margin_cull;
} orc_settings;

typedef struct {
  int32_t alive;     // survived every cull (decided in FP64)
  int32_t optional;  // a cull decision lies within the parity margin
  double depth;
  double mean2d[2];
  double cov2d[3];   // xx, xy, yy (blur included)
  double conic[3];   // inverse of cov2d: a, b, c
  double p_t, opt;   // temporal marginal, opacity * p_t
  double color[3];
  double mean3[3];   // conditional mean at t
  double cov3[6];    // conditional covariance xx, xy, xz, yy, yz, zz
} orc_splat;

typedef struct {
  double *mean4, *scale4, *rot_l, *rot_r, *opacity, *sh;
  double* mask;     // [n] (+=) straight-through dL/dM, or NULL
  double* densify;  // [n] (+=) |dL/d mean2d| of this view, or NULL
} orc_grads;

typedef struct {
  int32_t n_features;      // D >= 0
  const double* features;  // [n][D] (may be NULL when D = 0)
  const double* gate;      // [D], or NULL for all ones
  int32_t depth;           // 1: add a depth channel
  int32_t flow;            // 1: add two flow channels (du, dv)
  double flow_dt;          // time step of the flow
} orc_channels;

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------------------------
// Scalar types: plain double, and a forward-mode dual number over the 17 geometry parameters
// (mean4 0-3, scale4 4-7, rot_l 8-11, rot_r 12-15, opacity 16).
// ---------------------------------------------------------------------------------------------
constexpr int NG = 17;

struct Dual {
  double v;
  double d[NG];
  Dual() : v(0) { std::memset(d, 0, sizeof d); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof d); }  // NOLINT: implicit constant
  static Dual var(double x, int k) {
    Dual r(x);
    r.d[k] = 1.0;
    return r;
  }
};

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }

inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r(a.v + b.v);
  for (int k = 0; k < NG; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r(a.v - b.v);
  for (int k = 0; k < NG; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
inline Dual operator-(const Dual& a) {
  Dual r(-a.v);
  for (int k = 0; k < NG; ++k) r.d[k] = -a.d[k];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r(a.v * b.v);
  for (int k = 0; k < NG; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  const double ib2 = 1.0 / (b.v * b.v);
  for (int k = 0; k < NG; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) * ib2;
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) {
  Dual r(a.v * b);
  for (int k = 0; k < NG; ++k) r.d[k] = a.d[k] * b;
  return r;
}
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }

inline Dual chain(const Dual& a, double f, double df) {
  Dual r(f);
  for (int k = 0; k < NG; ++k) r.d[k] = df * a.d[k];
  return r;
}
inline Dual sqrt(const Dual& a) {
  const double s = std::sqrt(a.v);
  return chain(a, s, 0.5 / s);
}
inline Dual exp(const Dual& a) {
  const double e = std::exp(a.v);
  return chain(a, e, e);
}
inline Dual cos(const Dual& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
inline Dual sin(const Dual& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
inline Dual atan2(const Dual& y, const Dual& x) {
  const double r2 = x.v * x.v + y.v * y.v;
  Dual r(std::atan2(y.v, x.v));
  for (int k = 0; k < NG; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) / r2;
  return r;
}
using std::atan2;
using std::cos;
using std::exp;
using std::sin;
using std::sqrt;

// ---------------------------------------------------------------------------------------------
// O1-O3: rotors and the 4D covariance.
// ---------------------------------------------------------------------------------------------

// Left isoclinic rotation matrix of q = (a, b, c, d), as printed in Sec. 3.2.
template <class S>
void left_isoclinic(const S q[4], S L[4][4]) {
  const S &a = q[0], &b = q[1], &c = q[2], &d = q[3];
  L[0][0] = a;  L[0][1] = -b; L[0][2] = -c; L[0][3] = -d;
  L[1][0] = b;  L[1][1] = a;  L[1][2] = -d; L[1][3] = c;
  L[2][0] = c;  L[2][1] = d;  L[2][2] = a;  L[2][3] = -b;
  L[3][0] = d;  L[3][1] = -c; L[3][2] = b;  L[3][3] = a;
}

// Right isoclinic rotation matrix of q = (p, q, r, s), as printed in Sec. 3.2.
template <class S>
void right_isoclinic(const S q[4], S R[4][4]) {
  const S &p = q[0], &qq = q[1], &r = q[2], &s = q[3];
  R[0][0] = p;  R[0][1] = -qq; R[0][2] = -r; R[0][3] = -s;
  R[1][0] = qq; R[1][1] = p;   R[1][2] = s;  R[1][3] = -r;
  R[2][0] = r;  R[2][1] = -s;  R[2][2] = p;  R[2][3] = qq;
  R[3][0] = s;  R[3][1] = r;   R[3][2] = -qq; R[3][3] = p;
}

template <class S>
void normalize4(const S q[4], S out[4]) {
  const S n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) out[i] = q[i] / n;
}

// O1 + O2: R = L(q_l / |q_l|) R(q_r / |q_r|).
template <class S>
void rotation4(const S ql[4], const S qr[4], S R[4][4]) {
  S qln[4], qrn[4], L[4][4], Rr[4][4];
  normalize4(ql, qln);
  normalize4(qr, qrn);
  left_isoclinic(qln, L);
  right_isoclinic(qrn, Rr);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      S acc = L[i][0] * Rr[0][j];
      for (int k = 1; k < 4; ++k) acc = acc + L[i][k] * Rr[k][j];
      R[i][j] = acc;
    }
}

// O3: Sigma = R S S^T R^T.
template <class S>
void covariance4(const S R[4][4], const S s[4], S Sig[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      S acc = R[i][0] * s[0] * s[0] * R[j][0];
      for (int k = 1; k < 4; ++k) acc = acc + R[i][k] * s[k] * s[k] * R[j][k];
      Sig[i][j] = acc;
    }
}

// O4: conditional mean and covariance of (x, y, z) given t, and the unnormalized marginal p(t).
template <class S>
void slice(const S Sig[4][4], const S mean4[4], double t, S mu_c[3], S cov_c[3][3], S& p_t) {
  const S dt = t - mean4[3];
  for (int i = 0; i < 3; ++i) mu_c[i] = mean4[i] + Sig[i][3] / Sig[3][3] * dt;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) cov_c[i][j] = Sig[i][j] - Sig[i][3] * Sig[3][j] / Sig[3][3];
  p_t = exp(-0.5 * dt * dt / Sig[3][3]);
}

// ---------------------------------------------------------------------------------------------
// O7: real spherical harmonics without the Condon-Shortley phase, and the 4DSH color.
// ---------------------------------------------------------------------------------------------

// Associated Legendre function P_l^m(x), m >= 0, without the Condon-Shortley phase:
// P_m^m = (2m-1)!! (1-x^2)^{m/2}; P_{m+1}^m = x (2m+1) P_m^m;
// (l-m) P_l^m = x (2l-1) P_{l-1}^m - (l+m-1) P_{l-2}^m.
template <class S>
S legendre(int l, int m, const S& x, const S& sin_theta) {
  S pmm = 1.0;
  for (int i = 1; i <= m; ++i) pmm = pmm * (2.0 * i - 1.0) * sin_theta;
  if (l == m) return pmm;
  S pm1 = x * (2.0 * m + 1.0) * pmm;
  if (l == m + 1) return pm1;
  S pl = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pl = (x * (2.0 * ll - 1.0) * pm1 - (ll + m - 1.0) * pmm) / (double)(ll - m);
    pmm = pm1;
    pm1 = pl;
  }
  return pl;
}

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

// Y_l^m for all l <= deg, in the order index = l*l + l + m, m = -l..l.
// theta is measured from +z, phi from +x towards +y.
//   m < 0 : sqrt2 K_l^|m| P_l^|m|(cos theta) sin(|m| phi)
//   m = 0 : K_l^0 P_l^0(cos theta)
//   m > 0 : sqrt2 K_l^m P_l^m(cos theta) cos(m phi)
//   K_l^m = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!)
template <class S>
void sh_basis(int deg, const S dir[3], S* Y) {
  const S ct = dir[2];
  const S st = sqrt(dir[0] * dir[0] + dir[1] * dir[1]);
  const S phi = atan2(dir[1], dir[0]);
  for (int l = 0; l <= deg; ++l)
    for (int m = -l; m <= l; ++m) {
      const int am = m < 0 ? -m : m;
      const double K =
          std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
      const S P = legendre(l, am, ct, st);
      S y;
      if (m < 0)
        y = std::sqrt(2.0) * K * P * sin((double)am * phi);
      else if (m == 0)
        y = K * P;
      else
        y = std::sqrt(2.0) * K * P * cos((double)m * phi);
      Y[l * l + l + m] = y;
    }
}

// ---------------------------------------------------------------------------------------------
// O1-O7 for one Gaussian in one view.
// ---------------------------------------------------------------------------------------------
template <class S>
struct SplatT {
  bool alive = false, optional = false, in_front = false, projected = false;
  S depth{}, u{}, v{}, cov2d[3]{}, conic[3]{}, p_t{}, opt{}, color[3]{};
  S mean3[3]{}, cov3[3][3]{};
  bool color_clamped[3] = {false, false, false};
  double dir[3] = {0, 0, 0};
  double dt = 0;
};

template <class S>
S clamp_val(const S& x, double lo, double hi) {
  if (val(x) < lo) return S(lo);
  if (val(x) > hi) return S(hi);
  return x;
}

template <class S>
SplatT<S> preprocess(const S mean4[4], const S scale4[4], const S ql[4], const S qr[4],
                     const S& opacity, const double* sh, int Ds, int Dt, const orc_view& vw,
                     const orc_settings& st) {
  SplatT<S> sp;
  S R[4][4], Sig[4][4];
  rotation4(ql, qr, R);
  covariance4(R, scale4, Sig);
  slice(Sig, mean4, vw.t, sp.mean3, sp.cov3, sp.p_t);

  // Camera: x = W mu_c + tau.
  const double* E = vw.world_to_cam;
  S x[3];
  for (int i = 0; i < 3; ++i)
    x[i] = E[4 * i + 0] * sp.mean3[0] + E[4 * i + 1] * sp.mean3[1] + E[4 * i + 2] * sp.mean3[2] +
           E[4 * i + 3];
  sp.depth = x[2];

  const double pt = val(sp.p_t), z = val(x[2]);
  bool cull = false, near_threshold = false;
  // O5: the temporal marginal filter comes first, then the near plane.
  if (!(pt >= st.marginal_min)) cull = true;
  if (std::fabs(pt - st.marginal_min) <= st.margin_cull * st.marginal_min) near_threshold = true;
  if (!(z > st.near_z)) cull = true;
  if (std::fabs(z - st.near_z) <= st.margin_cull * st.near_z) near_threshold = true;
  // Projection needs a point in front of the camera; anything at or behind z = 0 is dropped
  // for good, whatever the margins say.
  if (!(z > 0.0)) return sp;
  sp.in_front = true;

  // O6: EWA mean and covariance.
  sp.u = vw.fx * x[0] / x[2] + vw.cx;
  sp.v = vw.fy * x[1] / x[2] + vw.cy;
  const double m = st.jacobian_margin;
  const double xlo = (-m * vw.width - vw.cx) / vw.fx, xhi = ((1.0 + m) * vw.width - vw.cx) / vw.fx;
  const double ylo = (-m * vw.height - vw.cy) / vw.fy,
               yhi = ((1.0 + m) * vw.height - vw.cy) / vw.fy;
  const S tx = clamp_val(S(x[0] / x[2]), xlo, xhi);
  const S ty = clamp_val(S(x[1] / x[2]), ylo, yhi);
  // J: Jacobian of the perspective map at (tx z, ty z, z); row 0 and row 1.
  S J[2][3];
  J[0][0] = vw.fx / x[2]; J[0][1] = S(0.0);        J[0][2] = -vw.fx * tx / x[2];
  J[1][0] = S(0.0);       J[1][1] = vw.fy / x[2];  J[1][2] = -vw.fy * ty / x[2];
  // T = J W, then Sigma2d = T Sigma_c T^T + blur I.
  S T[2][3];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      T[i][j] = J[i][0] * E[0 * 4 + j] + J[i][1] * E[1 * 4 + j] + J[i][2] * E[2 * 4 + j];
  S C2[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      S acc = S(0.0);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc = acc + T[i][a] * sp.cov3[a][b] * T[j][b];
      C2[i][j] = acc;
    }
  sp.cov2d[0] = C2[0][0] + st.blur;
  sp.cov2d[1] = C2[0][1];
  sp.cov2d[2] = C2[1][1] + st.blur;
  const S det = sp.cov2d[0] * sp.cov2d[2] - sp.cov2d[1] * sp.cov2d[1];
  if (!(val(det) > 0.0) || !std::isfinite(val(det))) return sp;  // degenerate: dropped
  sp.conic[0] = sp.cov2d[2] / det;
  sp.conic[1] = -sp.cov2d[1] / det;
  sp.conic[2] = sp.cov2d[0] / det;
  sp.projected = true;
  sp.opt = opacity * sp.p_t;

  // O7: color from 4DSH at d = normalize(mu_c - camera centre), dt = t - mu_t.
  double Cc[3];
  for (int j = 0; j < 3; ++j)
    Cc[j] = -(E[0 * 4 + j] * E[3] + E[1 * 4 + j] * E[7] + E[2 * 4 + j] * E[11]);
  S d[3];
  for (int j = 0; j < 3; ++j) d[j] = sp.mean3[j] - Cc[j];
  const S dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int j = 0; j < 3; ++j) {
    d[j] = d[j] / dn;
    sp.dir[j] = val(d[j]);
  }
  const int nsh = (Ds + 1) * (Ds + 1);
  std::vector<S> Y(nsh);
  sh_basis(Ds, d, Y.data());
  const S dts = vw.t - mean4[3];
  sp.dt = val(dts);
  for (int ch = 0; ch < 3; ++ch) {
    S acc = S(st.color_offset);
    for (int n = 0; n <= Dt; ++n) {
      const S fn = cos(2.0 * M_PI * (double)n * dts / st.time_period);
      S inner = S(0.0);
      for (int k = 0; k < nsh; ++k) inner = inner + sh[(n * nsh + k) * 3 + ch] * Y[k];
      acc = acc + fn * inner;
    }
    if (val(acc) < st.color_min) {
      sp.color[ch] = S(st.color_min);
      sp.color_clamped[ch] = true;
    } else {
      sp.color[ch] = acc;
    }
  }
  sp.alive = !cull;
  sp.optional = near_threshold && std::isfinite(val(sp.u)) && std::isfinite(val(sp.v));
  return sp;
}

// ---------------------------------------------------------------------------------------------
// Frame: all Gaussians preprocessed for one view, plus the candidate search.
// ---------------------------------------------------------------------------------------------
struct Splat {
  bool alive, optional;
  double depth, u, v, cxx, cyy, a, b, c, opt, col[3];
  double half_w, half_h;  // half extents of the (margin-widened) cutoff ellipse
};

struct Cand {
  double depth, d2;
  int32_t idx;
  bool optional;  // inclusion itself is a marked decision
};

enum DecType { D_INCLUDE = 0, D_SKIP = 1, D_STOP = 2, D_SWAP = 3 };

struct Decision {
  int type, pos, pos2;  // candidate positions; D_SWAP exchanges the order of pos and pos2
};

struct PixelResult {
  int px = 0, py = 0;
  double rgb[3], T;
  int n_contrib;
  int64_t n_evals;
  std::vector<Decision> marks;
  std::vector<double> ext;  // extra channels (E)
};

struct Frame {
  orc_gaussians g;
  orc_view vw;
  orc_settings st;
  std::vector<Splat> splats;
  int bin = 16, bins_x = 0, bins_y = 0;
  std::vector<std::vector<int32_t>> bins;
  bool use_bins = true;
  std::vector<double> bg_px;  // per-pixel background [H][W][3] (empty: the view's constant)
  // Extra channels: E = D + depth + 2 flow values per splat, in that order.
  int D = 0, E = 0, off_depth = -1, off_flow = -1;
  const double* features = nullptr;  // [n][D]
  std::vector<double> gate;          // [D]
  std::vector<double> fnorm;         // |g * f| per Gaussian
  std::vector<double> ext;           // [n][E]
};

void load_params(const orc_gaussians& g, int i, double m4[4], double s4[4], double ql[4],
                 double qr[4], double& o) {
  for (int k = 0; k < 4; ++k) {
    m4[k] = g.mean4[4 * i + k];
    s4[k] = g.scale4[4 * i + k];
    ql[k] = g.rot_l[4 * i + k];
    qr[k] = g.rot_r[4 * i + k];
  }
  o = g.opacity[i];
}

int sh_stride(const orc_gaussians& g) {
  return (g.t_degree + 1) * (g.sh_degree + 1) * (g.sh_degree + 1) * 3;
}

void build_frame(Frame& f) {
  const int n = f.g.n;
  f.splats.assign(n, Splat{});
  const double cut2 = f.st.cutoff_sigma * f.st.cutoff_sigma;
  const double reach = std::sqrt(cut2 * (1.0 + f.st.margin_d2)) * (1.0 + 1e-9);
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < n; ++i) {
    if (f.g.mask && !(f.g.mask[i] > f.g.mask_threshold)) {
      f.splats[i].alive = f.splats[i].optional = false;  // masked: M_hat = 0
      continue;
    }
    double m4[4], s4[4], ql[4], qr[4], o;
    load_params(f.g, i, m4, s4, ql, qr, o);
    // Failure rule (a reading): a Gaussian with a non-finite parameter is dropped in every view,
    // so it gets no gradient either.
    bool finite = std::isfinite(o);
    for (int k = 0; k < 4; ++k)
      finite = finite && std::isfinite(m4[k]) && std::isfinite(s4[k]) && std::isfinite(ql[k]) &&
               std::isfinite(qr[k]);
    for (int k = 0; k < sh_stride(f.g); ++k)
      finite = finite && std::isfinite(f.g.sh[(size_t)i * sh_stride(f.g) + k]);
    if (!finite) {
      f.splats[i].alive = f.splats[i].optional = false;
      continue;
    }
    SplatT<double> sp = preprocess<double>(m4, s4, ql, qr, o, f.g.sh + (size_t)i * sh_stride(f.g),
                                           f.g.sh_degree, f.g.t_degree, f.vw, f.st);
    Splat& s = f.splats[i];
    s.alive = sp.alive && sp.in_front && std::isfinite(sp.u) && std::isfinite(sp.v);
    s.optional = sp.optional && sp.in_front && std::isfinite(sp.u);
    const bool usable = sp.in_front && sp.projected && std::isfinite(sp.conic[0]) &&
                        std::isfinite(sp.u) && std::isfinite(sp.v);
    if (!usable) {
      s.alive = s.optional = false;
      continue;
    }
    s.depth = sp.depth;
    s.u = sp.u;
    s.v = sp.v;
    s.cxx = sp.cov2d[0];
    s.cyy = sp.cov2d[2];
    s.a = sp.conic[0];
    s.b = sp.conic[1];
    s.c = sp.conic[2];
    s.opt = sp.opt;
    for (int ch = 0; ch < 3; ++ch) s.col[ch] = sp.color[ch];
    s.half_w = reach * std::sqrt(sp.cov2d[0]);
    s.half_h = reach * std::sqrt(sp.cov2d[2]);
  }
  f.bins_x = (f.vw.width + f.bin - 1) / f.bin;
  f.bins_y = (f.vw.height + f.bin - 1) / f.bin;
  f.bins.assign((size_t)f.bins_x * f.bins_y, {});
  for (int i = 0; i < n; ++i) {
    const Splat& s = f.splats[i];
    if (!s.alive && !s.optional) continue;
    // Pixel (px, py) has centre (px + 0.5, py + 0.5); keep bins whose pixels may lie in the box.
    const double x0 = s.u - s.half_w - 0.5, x1 = s.u + s.half_w - 0.5;
    const double y0 = s.v - s.half_h - 0.5, y1 = s.v + s.half_h - 0.5;
    if (x1 < 0 || y1 < 0 || x0 > f.vw.width - 1 || y0 > f.vw.height - 1) continue;
    const int bx0 = std::max(0, (int)std::floor(x0 / f.bin));
    const int bx1 = std::min(f.bins_x - 1, (int)std::floor(x1 / f.bin));
    const int by0 = std::max(0, (int)std::floor(y0 / f.bin));
    const int by1 = std::min(f.bins_y - 1, (int)std::floor(y1 / f.bin));
    for (int by = by0; by <= by1; ++by)
      for (int bx = bx0; bx <= bx1; ++bx) f.bins[(size_t)by * f.bins_x + bx].push_back(i);
  }
}

// O8-O9: candidate list of a pixel, sorted by (depth, index).
void gather(const Frame& f, int px, int py, std::vector<Cand>& out) {
  out.clear();
  const double cx = px + 0.5, cy = py + 0.5;
  const double cut2 = f.st.cutoff_sigma * f.st.cutoff_sigma;
  const double lim = cut2 * (1.0 + f.st.margin_d2);
  auto consider = [&](int i) {
    const Splat& s = f.splats[i];
    if (!s.alive && !s.optional) return;
    const double dx = cx - s.u, dy = cy - s.v;
    const double d2 = s.a * dx * dx + 2.0 * s.b * dx * dy + s.c * dy * dy;
    if (!(d2 <= lim)) return;
    const bool near_cut = std::fabs(d2 - cut2) <= f.st.margin_d2 * cut2;
    if (!(d2 <= cut2) && !near_cut) return;
    Cand c;
    c.depth = s.depth;
    c.d2 = d2;
    c.idx = i;
    c.optional = near_cut || s.optional;
    out.push_back(c);
  };
  if (f.use_bins) {
    const int bx = px / f.bin, by = py / f.bin;
    for (int i : f.bins[(size_t)by * f.bins_x + bx]) consider(i);
  } else {
    for (int i = 0; i < f.g.n; ++i) consider(i);
  }
  std::sort(out.begin(), out.end(), [](const Cand& a, const Cand& b) {
    if (a.depth != b.depth) return a.depth < b.depth;
    return a.idx < b.idx;
  });
}

// Base FP64 outcome of candidate inclusion (before any forced flip).
inline bool base_include(const Frame& f, const Cand& c) {
  const Splat& s = f.splats[c.idx];
  return s.alive && c.d2 <= f.st.cutoff_sigma * f.st.cutoff_sigma;
}

// O10: composite one pixel.  `flip` marks which of `marks` are taken on the other side;
// when `record` is set, decisions near their thresholds are appended to `res.marks`.
// `contrib` (optional) receives (candidate position, prefix T, alpha, alpha clamped).
struct Contrib {
  int pos;
  double T, alpha, G;
  bool clamped;
};

void composite(const Frame& f, const std::vector<Cand>& cands, const std::vector<Decision>& marks,
               unsigned flip, bool record, PixelResult& res, std::vector<Contrib>* contrib) {
  const orc_settings& st = f.st;
  std::vector<int> order(cands.size());
  for (size_t k = 0; k < cands.size(); ++k) order[k] = (int)k;
  auto flipped = [&](int type, int pos) {
    for (size_t j = 0; j < marks.size(); ++j)
      if (marks[j].type == type && marks[j].pos == pos) return ((flip >> j) & 1u) != 0;
    return false;
  };
  for (size_t j = 0; j < marks.size(); ++j)
    if (marks[j].type == D_SWAP && ((flip >> j) & 1u)) std::swap(order[marks[j].pos], order[marks[j].pos2]);

  double T = 1.0, C[3] = {0, 0, 0};
  res.ext.assign(f.E, 0.0);
  int n_contrib = 0;
  int64_t n_evals = 0;
  int last_pos = -1;  // order position of the previous contributing candidate
  for (size_t k = 0; k < order.size(); ++k) {
    const Cand& cd = cands[order[k]];
    const Splat& s = f.splats[cd.idx];
    bool include = base_include(f, cd);
    if (cd.optional) {
      if (record) res.marks.push_back({D_INCLUDE, order[k], -1});
      if (flipped(D_INCLUDE, order[k])) include = !include;
    }
    if (!include) continue;
    ++n_evals;
    const double G = std::exp(-0.5 * cd.d2);
    const double raw = s.opt * G;
    const double alpha = std::min(st.alpha_max, raw);
    bool skip = alpha < st.alpha_min;
    if (std::fabs(alpha - st.alpha_min) <= st.margin_alpha * st.alpha_min) {
      if (record) res.marks.push_back({D_SKIP, order[k], -1});
      if (flipped(D_SKIP, order[k])) skip = !skip;
    }
    if (skip) continue;
    const double Tn = T * (1.0 - alpha);
    bool stop = Tn < st.T_min;
    if (std::fabs(Tn - st.T_min) <= st.margin_T * st.T_min) {
      if (record) res.marks.push_back({D_STOP, order[k], -1});
      if (flipped(D_STOP, order[k])) stop = !stop;
    }
    if (stop) break;
    // Near-tie in depth with the previous contributor: the order of the pair is a decision.
    if (record && last_pos >= 0) {
      const double z0 = cands[order[last_pos]].depth, z1 = cd.depth;
      if (std::fabs(z1 - z0) <= st.margin_depth * std::max(1.0, std::fabs(z1)))
        res.marks.push_back({D_SWAP, last_pos, (int)k});
    }
    if (contrib) contrib->push_back({order[k], T, alpha, G, raw >= st.alpha_max});
    for (int ch = 0; ch < 3; ++ch) C[ch] += T * alpha * s.col[ch];
    for (int c = 0; c < f.E; ++c) res.ext[c] += T * alpha * f.ext[(size_t)cd.idx * f.E + c];
    T = Tn;
    ++n_contrib;
    last_pos = (int)k;
  }
  const double* bg = f.vw.background;
  if (!f.bg_px.empty()) bg = f.bg_px.data() + 3 * ((size_t)res.py * f.vw.width + res.px);
  for (int ch = 0; ch < 3; ++ch) res.rgb[ch] = C[ch] + T * bg[ch];
  res.T = T;
  res.n_contrib = n_contrib;
  res.n_evals = n_evals;
}

void render_pixel(const Frame& f, int px, int py, PixelResult& res, std::vector<Cand>& cands) {
  gather(f, px, py, cands);
  res.marks.clear();
  res.px = px;
  res.py = py;
  composite(f, cands, {}, 0u, true, res, nullptr);
}

// ---------------------------------------------------------------------------------------------
// O11: backward.
// ---------------------------------------------------------------------------------------------
// Per-splat accumulated gradient of the per-view quantities:
// 0-1 mean2d (u, v), 2-4 conic (a, b, c), 5 opt, 6-8 color.
constexpr int NQ = 9;

// gx: upstream gradient of the extra channels (E values, the flow entries set to zero by the
// caller); acc_ext (n * E) receives dL/d(extra payload) per splat.  Both may be NULL.
void pixel_backward(const Frame& f, int px, int py, const double g[3], std::vector<Cand>& cands,
                    std::vector<Contrib>& contrib, double* acc /* n * NQ */,
                    const double* gx = nullptr, double* acc_ext = nullptr) {
  gather(f, px, py, cands);
  PixelResult res;
  res.px = px;
  res.py = py;
  contrib.clear();
  composite(f, cands, {}, 0u, false, res, &contrib);
  // Reverse sweep: R = color of everything behind the current contributor (incl. background).
  const double* bg = f.vw.background;
  if (!f.bg_px.empty()) bg = f.bg_px.data() + 3 * ((size_t)py * f.vw.width + px);
  double R[3] = {bg[0], bg[1], bg[2]};
  std::vector<double> Rx(gx ? f.E : 0, 0.0);  // extra channels behind (zero background)
  const double cx = px + 0.5, cy = py + 0.5;
  for (int k = (int)contrib.size() - 1; k >= 0; --k) {
    const Contrib& ct = contrib[k];
    const Cand& cd = cands[ct.pos];
    const Splat& s = f.splats[cd.idx];
    double* a = acc + (size_t)cd.idx * NQ;
    double dalpha = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
      a[6 + ch] += g[ch] * ct.T * ct.alpha;
      dalpha += g[ch] * ct.T * (s.col[ch] - R[ch]);
    }
    if (gx) {
      const double* e = f.ext.data() + (size_t)cd.idx * f.E;
      for (int c = 0; c < f.E; ++c) {
        acc_ext[(size_t)cd.idx * f.E + c] += gx[c] * ct.T * ct.alpha;
        dalpha += gx[c] * ct.T * (e[c] - Rx[c]);
        Rx[c] = ct.alpha * e[c] + (1.0 - ct.alpha) * Rx[c];
      }
    }
    if (!ct.clamped) {
      const double dx = cx - s.u, dy = cy - s.v;
      a[5] += dalpha * ct.G;
      // alpha = opt exp(-d2/2), d2 = a dx^2 + 2 b dx dy + c dy^2, dx = px - u.
      a[0] += dalpha * ct.alpha * (s.a * dx + s.b * dy);
      a[1] += dalpha * ct.alpha * (s.b * dx + s.c * dy);
      a[2] += dalpha * ct.alpha * (-0.5 * dx * dx);
      a[3] += dalpha * ct.alpha * (-dx * dy);
      a[4] += dalpha * ct.alpha * (-0.5 * dy * dy);
    }
    for (int ch = 0; ch < 3; ++ch) R[ch] = ct.alpha * s.col[ch] + (1.0 - ct.alpha) * R[ch];
  }
}

void gaussian_backward(const Frame& f, int i, const double* q /* NQ */, orc_grads& out,
                       double q_depth = 0.0) {
  double m4[4], s4[4], ql[4], qr[4], o;
  load_params(f.g, i, m4, s4, ql, qr, o);
  Dual M[4], Sc[4], QL[4], QR[4];
  for (int k = 0; k < 4; ++k) {
    M[k] = Dual::var(m4[k], k);
    Sc[k] = Dual::var(s4[k], 4 + k);
    QL[k] = Dual::var(ql[k], 8 + k);
    QR[k] = Dual::var(qr[k], 12 + k);
  }
  Dual O = Dual::var(o, 16);
  const double* sh = f.g.sh + (size_t)i * sh_stride(f.g);
  SplatT<Dual> sp = preprocess<Dual>(M, Sc, QL, QR, O, sh, f.g.sh_degree, f.g.t_degree, f.vw, f.st);
  const Dual* outs[NQ] = {&sp.u,     &sp.v,        &sp.conic[0], &sp.conic[1], &sp.conic[2],
                          &sp.opt,   &sp.color[0], &sp.color[1], &sp.color[2]};
  double grad[NG] = {0};
  for (int j = 0; j < NQ; ++j)
    for (int k = 0; k < NG; ++k) grad[k] += q[j] * outs[j]->d[k];
  for (int k = 0; k < NG; ++k) grad[k] += q_depth * sp.depth.d[k];
  for (int k = 0; k < 4; ++k) {
    out.mean4[4 * i + k] += grad[k];
    out.scale4[4 * i + k] += grad[4 + k];
    out.rot_l[4 * i + k] += grad[8 + k];
    out.rot_r[4 * i + k] += grad[12 + k];
  }
  out.opacity[i] += grad[16];
  // Straight-through mask: S_hat = M_hat S and alpha_hat = M_hat o at M_hat = 1.
  if (out.mask) {
    double gm = o * grad[16];
    for (int k = 0; k < 4; ++k) gm += s4[k] * grad[4 + k];
    out.mask[i] += gm;
  }
  if (out.densify) out.densify[i] += std::sqrt(q[0] * q[0] + q[1] * q[1]);
  // SH: color is linear in the coefficients; zero where the color was clamped.
  const int Ds = f.g.sh_degree, nsh = (Ds + 1) * (Ds + 1);
  std::vector<double> Y(nsh);
  sh_basis<double>(Ds, sp.dir, Y.data());
  double* gsh = out.sh + (size_t)i * sh_stride(f.g);
  for (int n = 0; n <= f.g.t_degree; ++n) {
    const double fn = std::cos(2.0 * M_PI * n * sp.dt / f.st.time_period);
    for (int k = 0; k < nsh; ++k)
      for (int ch = 0; ch < 3; ++ch)
        if (!sp.color_clamped[ch]) gsh[(n * nsh + k) * 3 + ch] += q[6 + ch] * fn * Y[k];
  }
}

// Cube-map face and coordinates of direction r (the OpenGL table): face 0..5 = +x, -x, +y, -y,
// +z, -z; (s, t) in [0, 1].  `alt` receives the face the next axis would pick and its
// coordinates when two axes are within `margin` (relative) of a tie, else -1.
struct CubeHit {
  int face;
  double s, t;
};

CubeHit cube_face(const double r[3], int axis) {
  const double x = r[0], y = r[1], z = r[2];
  double sc, tc, ma;
  int face;
  if (axis == 0) {
    face = x >= 0 ? 0 : 1;
    ma = std::fabs(x);
    sc = x >= 0 ? -z : z;
    tc = -y;
  } else if (axis == 1) {
    face = y >= 0 ? 2 : 3;
    ma = std::fabs(y);
    sc = x;
    tc = y >= 0 ? z : -z;
  } else {
    face = z >= 0 ? 4 : 5;
    ma = std::fabs(z);
    sc = z >= 0 ? x : -x;
    tc = -y;
  }
  return {face, 0.5 * (sc / ma + 1.0), 0.5 * (tc / ma + 1.0)};
}

int major_axis(const double r[3]) {
  const double ax = std::fabs(r[0]), ay = std::fabs(r[1]), az = std::fabs(r[2]);
  if (ax >= ay && ax >= az) return 0;
  return ay >= az ? 1 : 2;
}

// Bilinear lookup (clamped to the face) of a cube map [6][R][R][3]; with `grad`, adds w * g
// to the four texels instead.
void cube_bilinear(const CubeHit& h, int R, const double* cube, double out[3], double* grad,
                   const double g[3]) {
  const double x = h.s * R - 0.5, y = h.t * R - 0.5;
  const double fx = std::floor(x), fy = std::floor(y);
  const double ax = x - fx, ay = y - fy;
  const int x0 = (int)fx, y0 = (int)fy;
  const int xs[2] = {std::min(std::max(x0, 0), R - 1), std::min(std::max(x0 + 1, 0), R - 1)};
  const int ys[2] = {std::min(std::max(y0, 0), R - 1), std::min(std::max(y0 + 1, 0), R - 1)};
  const double wx[2] = {1.0 - ax, ax}, wy[2] = {1.0 - ay, ay};
  if (out) out[0] = out[1] = out[2] = 0.0;
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) {
      const size_t k = (((size_t)h.face * R + ys[b]) * R + xs[a]) * 3;
      const double w = wx[a] * wy[b];
      for (int c = 0; c < 3; ++c) {
        if (out) out[c] += w * cube[k + c];
        if (grad) grad[k + c] += w * g[c];
      }
    }
}

// World direction of the ray through the centre of pixel (px, py).
void pixel_ray(const orc_view& vw, int px, int py, double r[3]) {
  const double d[3] = {(px + 0.5 - vw.cx) / vw.fx, (py + 0.5 - vw.cy) / vw.fy, 1.0};
  const double* E = vw.world_to_cam;
  double n2 = 0.0;
  for (int j = 0; j < 3; ++j) {
    r[j] = E[0 * 4 + j] * d[0] + E[1 * 4 + j] * d[1] + E[2 * 4 + j] * d[2];
    n2 += r[j] * r[j];
  }
  const double inv = 1.0 / std::sqrt(n2);
  for (int j = 0; j < 3; ++j) r[j] *= inv;
}

// Image-plane displacement of the projected conditional mean of Gaussian i between the frame's
// time t and t + dt (0 where either mean is not in front of the camera).
void flow_of(const Frame& f, int i, double dt, double out[2]) {
  double m4[4], s4[4], ql[4], qr[4], o;
  load_params(f.g, i, m4, s4, ql, qr, o);
  double Rm[4][4], Sig[4][4], mu[2][3], cov[3][3], pt;
  rotation4<double>(ql, qr, Rm);
  covariance4<double>(Rm, s4, Sig);
  slice<double>(Sig, m4, f.vw.t, mu[0], cov, pt);
  slice<double>(Sig, m4, f.vw.t + dt, mu[1], cov, pt);
  const double* E = f.vw.world_to_cam;
  double uv[2][2];
  out[0] = out[1] = 0.0;
  for (int k = 0; k < 2; ++k) {
    double x[3];
    for (int r = 0; r < 3; ++r)
      x[r] = E[4 * r] * mu[k][0] + E[4 * r + 1] * mu[k][1] + E[4 * r + 2] * mu[k][2] + E[4 * r + 3];
    if (!(x[2] > 0.0)) return;
    uv[k][0] = f.vw.fx * x[0] / x[2] + f.vw.cx;
    uv[k][1] = f.vw.fy * x[1] / x[2] + f.vw.cy;
  }
  out[0] = uv[1][0] - uv[0][0];
  out[1] = uv[1][1] - uv[0][1];
}

}  // namespace

// =============================================================================================
// C ABI (ctypes).
// =============================================================================================
extern "C" {

// R = L(q_l/|q_l|) R(q_r/|q_r|), row-major 4x4.
void orc_rotation(const double* ql, const double* qr, double* R) {
  double Rm[4][4];
  rotation4<double>(ql, qr, Rm);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) R[4 * i + j] = Rm[i][j];
}

// Sigma (4x4), conditional mean (3), conditional covariance (3x3) and p(t).
void orc_slice(const double* mean4, const double* scale4, const double* ql, const double* qr,
               double t, double* cov4, double* mu_c, double* cov_c, double* p_t) {
  double Rm[4][4], Sig[4][4], mc[3], cc[3][3], pt;
  rotation4<double>(ql, qr, Rm);
  covariance4<double>(Rm, scale4, Sig);
  slice<double>(Sig, mean4, t, mc, cc, pt);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) cov4[4 * i + j] = Sig[i][j];
  for (int i = 0; i < 3; ++i) {
    mu_c[i] = mc[i];
    for (int j = 0; j < 3; ++j) cov_c[3 * i + j] = cc[i][j];
  }
  *p_t = pt;
}

double orc_legendre(int l, int m, double x) {
  return legendre<double>(l, m, x, std::sqrt(std::max(0.0, 1.0 - x * x)));
}

// Real SH basis values Y[(deg+1)^2] at unit direction dir.
void orc_sh_basis(int deg, const double* dir, double* Y) { sh_basis<double>(deg, dir, Y); }

void* orc_frame_new(const orc_gaussians* g, const orc_view* vw, const orc_settings* st,
                    int use_bins) {
  Frame* f = new Frame;
  f->g = *g;
  f->vw = *vw;
  f->st = *st;
  f->use_bins = use_bins != 0;
  build_frame(*f);
  return f;
}

void orc_frame_free(void* h) { delete static_cast<Frame*>(h); }

// Attach extra channels to the frame (features, depth, flow; see the file header).  The
// feature array must stay alive as long as the frame is used.  Returns E, the number of extra
// channels.
int orc_frame_set_channels(void* h, const orc_channels* ch) {
  Frame& f = *static_cast<Frame*>(h);
  const int n = f.g.n;
  f.D = ch->n_features;
  f.features = ch->features;
  f.off_depth = ch->depth ? f.D : -1;
  f.off_flow = ch->flow ? f.D + (ch->depth ? 1 : 0) : -1;
  f.E = f.D + (ch->depth ? 1 : 0) + (ch->flow ? 2 : 0);
  f.gate.assign(f.D, 1.0);
  if (ch->gate)
    for (int c = 0; c < f.D; ++c) f.gate[c] = ch->gate[c];
  f.fnorm.assign(n, 0.0);
  f.ext.assign((size_t)n * f.E, 0.0);
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < n; ++i) {
    double* e = f.ext.data() + (size_t)i * f.E;
    if (f.D > 0) {
      double nrm2 = 0.0;
      for (int c = 0; c < f.D; ++c) {
        const double v = f.gate[c] * f.features[(size_t)i * f.D + c];
        nrm2 += v * v;
      }
      const double nrm = std::sqrt(nrm2);
      f.fnorm[i] = nrm;
      for (int c = 0; c < f.D; ++c)
        e[c] = nrm > 0.0 ? f.gate[c] * f.features[(size_t)i * f.D + c] / nrm : 0.0;
    }
    if (f.off_depth >= 0) e[f.off_depth] = f.splats[i].depth;
    if (f.off_flow >= 0) flow_of(f, i, ch->flow_dt, e + f.off_flow);
  }
  return f.E;
}

// Full O1-O7 output per Gaussian (alive Gaussians only carry meaningful values).
int orc_frame_splats(void* h, orc_splat* out) {
  Frame& f = *static_cast<Frame*>(h);
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < f.g.n; ++i) {
    double m4[4], s4[4], ql[4], qr[4], o;
    load_params(f.g, i, m4, s4, ql, qr, o);
    SplatT<double> sp = preprocess<double>(m4, s4, ql, qr, o, f.g.sh + (size_t)i * sh_stride(f.g),
                                           f.g.sh_degree, f.g.t_degree, f.vw, f.st);
    orc_splat& s = out[i];
    std::memset(&s, 0, sizeof s);
    s.alive = f.splats[i].alive;
    s.optional = f.splats[i].optional;
    s.depth = sp.depth;
    s.mean2d[0] = sp.u;
    s.mean2d[1] = sp.v;
    for (int k = 0; k < 3; ++k) {
      s.cov2d[k] = sp.cov2d[k];
      s.conic[k] = sp.conic[k];
      s.color[k] = sp.color[k];
      s.mean3[k] = sp.mean3[k];
    }
    s.p_t = sp.p_t;
    s.opt = sp.opt;
    s.cov3[0] = sp.cov3[0][0];
    s.cov3[1] = sp.cov3[0][1];
    s.cov3[2] = sp.cov3[0][2];
    s.cov3[3] = sp.cov3[1][1];
    s.cov3[4] = sp.cov3[1][2];
    s.cov3[5] = sp.cov3[2][2];
  }
  return 0;
}

// Render pixels.  xy: n_pix (x, y) pairs, or NULL for the whole image in row-major order.
// rgb: [n_pix][3]; T, n_contrib, n_marks: [n_pix]; n_evals: [n_pix] candidates evaluated
// (Mahalanobis distance within the cutoff) up to the stop; ext: [n_pix][E] extra channels.
// Any output may be NULL.
int orc_frame_render(void* h, int n_pix, const int32_t* xy, double* rgb, double* T,
                     int32_t* n_contrib, int32_t* n_marks, int64_t* n_evals, double* ext) {
  Frame& f = *static_cast<Frame*>(h);
  const int W = f.vw.width;
  if (!xy) n_pix = W * f.vw.height;
#pragma omp parallel
  {
    std::vector<Cand> cands;
    PixelResult res;
#pragma omp for schedule(dynamic, 64)
    for (int p = 0; p < n_pix; ++p) {
      const int px = xy ? xy[2 * p] : p % W, py = xy ? xy[2 * p + 1] : p / W;
      render_pixel(f, px, py, res, cands);
      if (rgb)
        for (int ch = 0; ch < 3; ++ch) rgb[3 * (size_t)p + ch] = res.rgb[ch];
      if (T) T[p] = res.T;
      if (n_contrib) n_contrib[p] = res.n_contrib;
      if (n_marks) n_marks[p] = (int32_t)res.marks.size();
      if (n_evals) n_evals[p] = res.n_evals;
      if (ext)
        for (int c = 0; c < f.E; ++c) ext[(size_t)p * f.E + c] = res.ext[c];
    }
  }
  return 0;
}

// All admissible results of one pixel: every combination of its marked decisions taken either
// way (color, transmittance, extra channels and composited count of each).  Returns the number of variants written (2^marks), or -1 if the pixel has more than
// max_marks marked decisions (unverifiable), or -2 if the output buffer is too small.
int orc_frame_variants(void* h, int px, int py, int max_marks, int max_out, double* rgb,
                       double* T, double* ext, int32_t* n_contrib) {
  Frame& f = *static_cast<Frame*>(h);
  std::vector<Cand> cands;
  PixelResult base;
  render_pixel(f, px, py, base, cands);
  const int k = (int)base.marks.size();
  if (k > max_marks) return -1;
  const int nv = 1 << k;
  if (nv > max_out) return -2;
  for (int v = 0; v < nv; ++v) {
    PixelResult r;
    r.px = px;
    r.py = py;
    composite(f, cands, base.marks, (unsigned)v, false, r, nullptr);
    for (int ch = 0; ch < 3; ++ch) rgb[3 * v + ch] = r.rgb[ch];
    if (T) T[v] = r.T;
    if (n_contrib) n_contrib[v] = r.n_contrib;
    if (ext)
      for (int c = 0; c < f.E; ++c) ext[(size_t)v * f.E + c] = r.ext[c];
  }
  return nv;
}

// Backward of the whole image of this view: accumulates (+=) the gradient of
// L = <dL_drgb, image> + <dL_dext, extra channels> into `out`, `d_features` ([n][D]) and
// `d_gate` ([D]).  dL_drgb is planar [3][H][W]; dL_dext is planar [E][H][W] or NULL (its flow
// channels are ignored).  d_features and d_gate may be NULL when there are no features.
int orc_frame_backward(void* h, const double* dL_drgb, const double* dL_dext, orc_grads* out,
                       double* d_features, double* d_gate) {
  Frame& f = *static_cast<Frame*>(h);
  const int W = f.vw.width, H = f.vw.height, n = f.g.n;
  const bool has_ext = dL_dext && f.E > 0;
  const int E = has_ext ? f.E : 0;
  std::vector<double> acc((size_t)n * NQ, 0.0), acc_ext((size_t)n * E, 0.0);
#pragma omp parallel
  {
    std::vector<double> local((size_t)n * NQ, 0.0), local_ext((size_t)n * E, 0.0);
    std::vector<double> gx(E, 0.0);
    std::vector<Cand> cands;
    std::vector<Contrib> contrib;
#pragma omp for schedule(dynamic, 64)
    for (int p = 0; p < W * H; ++p) {
      const double g[3] = {dL_drgb[p], dL_drgb[(size_t)W * H + p], dL_drgb[2 * (size_t)W * H + p]};
      for (int c = 0; c < E; ++c) {
        const bool is_flow = f.off_flow >= 0 && c >= f.off_flow;
        gx[c] = is_flow ? 0.0 : dL_dext[(size_t)c * W * H + p];
      }
      pixel_backward(f, p % W, p / W, g, cands, contrib, local.data(),
                     has_ext ? gx.data() : nullptr, has_ext ? local_ext.data() : nullptr);
    }
#pragma omp critical
    {
      for (size_t k = 0; k < local.size(); ++k) acc[k] += local[k];
      for (size_t k = 0; k < local_ext.size(); ++k) acc_ext[k] += local_ext[k];
    }
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int i = 0; i < n; ++i) {
    const double* q = acc.data() + (size_t)i * NQ;
    const double q_depth = (has_ext && f.off_depth >= 0) ? acc_ext[(size_t)i * E + f.off_depth] : 0.0;
    bool any = q_depth != 0.0;
    for (int j = 0; j < NQ; ++j) any |= q[j] != 0.0;
    if (!any || !f.splats[i].alive) continue;
    gaussian_backward(f, i, q, *out, q_depth);
  }
  // Features: f_hat = s / |s|, s = gate * f.  dL/ds = (dL/df_hat - f_hat (f_hat . dL/df_hat)) / |s|,
  // dL/df = gate * dL/ds, dL/dgate = sum over Gaussians of f * dL/ds.  (Zero where |s| = 0.)
  if (has_ext && f.D > 0 && d_features) {
    for (int i = 0; i < n; ++i) {
      const double nrm = f.fnorm[i];
      if (!(nrm > 0.0)) continue;
      const double* gf = acc_ext.data() + (size_t)i * E;
      const double* fh = f.ext.data() + (size_t)i * f.E;
      double dot = 0.0;
      for (int c = 0; c < f.D; ++c) dot += fh[c] * gf[c];
      for (int c = 0; c < f.D; ++c) {
        const double ds = (gf[c] - fh[c] * dot) / nrm;
        d_features[(size_t)i * f.D + c] += f.gate[c] * ds;
        if (d_gate) d_gate[c] += f.features[(size_t)i * f.D + c] * ds;
      }
    }
  }
  return 0;
}

// Per-splat accumulated gradient of the 9 per-view quantities (for stage tests): [n][9].
int orc_frame_backward_splat(void* h, const double* dL_drgb, double* acc_out) {
  Frame& f = *static_cast<Frame*>(h);
  const int W = f.vw.width, H = f.vw.height, n = f.g.n;
  std::fill(acc_out, acc_out + (size_t)n * NQ, 0.0);
#pragma omp parallel
  {
    std::vector<double> local((size_t)n * NQ, 0.0);
    std::vector<Cand> cands;
    std::vector<Contrib> contrib;
#pragma omp for schedule(dynamic, 64)
    for (int p = 0; p < W * H; ++p) {
      const double g[3] = {dL_drgb[p], dL_drgb[(size_t)W * H + p], dL_drgb[2 * (size_t)W * H + p]};
      pixel_backward(f, p % W, p / W, g, cands, contrib, local.data());
    }
#pragma omp critical
    for (size_t k = 0; k < local.size(); ++k) acc_out[k] += local[k];
  }
  return 0;
}

// Sky image of a view: sky [H][W][3] = M_sky(r) of each pixel's ray.  Where the two largest
// |components| of r are within `margin` (relative) of each other the face choice is marked:
// near [H][W] = 1 and alt [H][W][3] holds the lookup on the other face (else alt = sky).
int orc_sky(const orc_view* vw, const double* cube, int R, double margin, double* sky,
            double* alt, int32_t* near) {
  const int W = vw->width, H = vw->height;
#pragma omp parallel for schedule(static)
  for (int p = 0; p < W * H; ++p) {
    double r[3];
    pixel_ray(*vw, p % W, p / W, r);
    const int ax = major_axis(r);
    cube_bilinear(cube_face(r, ax), R, cube, sky + 3 * (size_t)p, nullptr, nullptr);
    int other = -1;
    const double m = std::fabs(r[ax]);
    for (int k = 0; k < 3; ++k)
      if (k != ax && std::fabs(std::fabs(r[k]) - m) <= margin * m) other = k;
    if (near) near[p] = other >= 0;
    if (alt) {
      if (other >= 0)
        cube_bilinear(cube_face(r, other), R, cube, alt + 3 * (size_t)p, nullptr, nullptr);
      else
        for (int c = 0; c < 3; ++c) alt[3 * (size_t)p + c] = sky[3 * (size_t)p + c];
    }
  }
  return 0;
}

// Adjoint of orc_sky: d_cube [6][R][R][3] += the bilinear transpose of dsky [H][W][3].
int orc_sky_backward(const orc_view* vw, int R, const double* dsky, double* d_cube) {
  const int W = vw->width, H = vw->height;
  for (int p = 0; p < W * H; ++p) {
    double r[3];
    pixel_ray(*vw, p % W, p / W, r);
    cube_bilinear(cube_face(r, major_axis(r)), R, nullptr, nullptr, d_cube, dsky + 3 * (size_t)p);
  }
  return 0;
}

// Per-pixel background [H][W][3] used instead of the view's constant (NULL: back to it).
int orc_frame_set_background(void* h, const double* bg) {
  Frame& f = *static_cast<Frame*>(h);
  if (!bg) {
    f.bg_px.clear();
    return 0;
  }
  f.bg_px.assign(bg, bg + 3 * (size_t)f.vw.width * f.vw.height);
  return 0;
}

// Decode a compact model into full parameters (float64; see the file header).  mean4_h holds
// IEEE half bit patterns.  Codebooks: scale [6][64][4], rot [6][64][4], dc [6][64][3],
// rest [8][256][K - 3] with K = (t_degree + 1)(sh_degree + 1)^2 3; sh out [n][K] with the
// direct component (n = 0, l = 0) first.
int orc_decode_compact(int n, int sh_degree, int t_degree, const uint16_t* mean4_h,
                       const uint8_t* scale_idx, const uint8_t* rot_l_idx,
                       const uint8_t* rot_r_idx, const uint8_t* opacity_q, double op_lo,
                       double op_hi, const uint8_t* dc_idx, const uint8_t* rest_idx,
                       const double* scale_cb, const double* rot_cb, const double* dc_cb,
                       const double* rest_cb, double* mean4, double* scale4, double* rot_l,
                       double* rot_r, double* opacity, double* sh) {
  const int K = (t_degree + 1) * (sh_degree + 1) * (sh_degree + 1) * 3;
  const int KR = K - 3;
  auto half_to_double = [](uint16_t h) {
    const int sign = (h >> 15) & 1, e = (h >> 10) & 31, m = h & 1023;
    double v;
    if (e == 0)
      v = std::ldexp((double)m, -24);  // subnormal
    else if (e == 31)
      v = m ? NAN : INFINITY;
    else
      v = std::ldexp((double)(m + 1024), e - 25);
    return sign ? -v : v;
  };
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < 4; ++k) mean4[4 * i + k] = half_to_double(mean4_h[4 * i + k]);
    for (int k = 0; k < 4; ++k) {
      double ls = 0.0, ql = 0.0, qr = 0.0;
      for (int c = 0; c < 6; ++c) {
        ls += scale_cb[(c * 64 + scale_idx[6 * i + c]) * 4 + k];
        ql += rot_cb[(c * 64 + rot_l_idx[6 * i + c]) * 4 + k];
        qr += rot_cb[(c * 64 + rot_r_idx[6 * i + c]) * 4 + k];
      }
      scale4[4 * i + k] = std::exp(ls);
      rot_l[4 * i + k] = ql;
      rot_r[4 * i + k] = qr;
    }
    opacity[i] = op_lo + (op_hi - op_lo) * (double)opacity_q[i] / 255.0;
    double* o = sh + (size_t)i * K;
    for (int ch = 0; ch < 3; ++ch) {
      double v = 0.0;
      for (int c = 0; c < 6; ++c) v += dc_cb[(c * 64 + dc_idx[6 * i + c]) * 3 + ch];
      o[ch] = v;
    }
    for (int j = 0; j < KR; ++j) {
      double v = 0.0;
      for (int c = 0; c < 8; ++c) v += rest_cb[((size_t)c * 256 + rest_idx[8 * i + c]) * KR + j];
      o[3 + j] = v;
    }
  }
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
