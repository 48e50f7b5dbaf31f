// Per-Gaussian work of the extra render channels (Sec. 7 feature rendering, Sec. 5
// rendered depth, Sec. 8.1 rendered flow); their compositing lives in the raster kernels.
//
//   feature_normalize: f_hat = s / |s| with s = gate * f (0 when s = 0).
//   flow_forward:      per visible (view, Gaussian) slot, the image displacement of the
//                      conditional mean between t and t + dt.  The mean moves linearly in t,
//                      mu(t') = mu(t) + Sigma_{1:3,4} / Sigma_44 (t' - t), so one slice suffices.
//   feature_backward:  dL/ds = (dL/df_hat - f_hat (f_hat . dL/df_hat)) / |s|,
//                      dL/df = gate * dL/ds, dL/dgate = sum_i f_i * dL/ds_i (per-lane sums
//                      over the rows a wave visits, then one atomic per channel and wave).
//
// The two feature kernels map a row of D features to DP = (next power of two >= D) adjacent
// lanes, 64 / DP rows per wave step, so that each load and store of the [N, D] arrays is one
// contiguous run; the row's dot products are sums over its DP lanes.
#include <hip/hip_runtime.h>

#include "g4d_internal.h"

namespace g4d {
namespace {

// Sum over the DP-lane group of the lane (DP a power of two, at most 64).
template <int DP>
__device__ __forceinline__ float group_sum(float x) {
#pragma unroll
  for (int o = DP / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <int DP>
__global__ __launch_bounds__(256) void k_feature_normalize(int n, int d,
                                                           const float* __restrict__ f,
                                                           const float* __restrict__ gate,
                                                           float* __restrict__ fn,
                                                           float* __restrict__ fnorm) {
  constexpr int kRows = 64 / DP;
  const int lane = threadIdx.x & 63, c = lane % DP, sub = lane / DP;
  const float gc = c < d ? (gate ? gate[c] : 1.f) : 0.f;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t stride = ((int64_t)gridDim.x * blockDim.x >> 6) * kRows;
  for (int64_t r0 = wave * kRows; r0 < n; r0 += stride) {
    const int64_t i = r0 + sub;
    const bool ok = i < n && c < d;
    const float s = ok ? gc * f[i * d + c] : 0.f;
    const float nrm = sqrtf(group_sum<DP>(s * s));
    const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
    if (ok) fn[i * d + c] = s * inv;
    if (i < n && c == 0) fnorm[i] = nrm;
  }
}

__global__ __launch_bounds__(256) void k_flow(int n, int n_views, const float4* __restrict__ mean4,
                                              const float4* __restrict__ scale4,
                                              const float4* __restrict__ rot_l,
                                              const float4* __restrict__ rot_r,
                                              const DView* __restrict__ views,
                                              const uint32_t* __restrict__ tiles, float dt,
                                              float2* __restrict__ flow) {
  const int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= n) return;
  Geom g;
  geom_forward(rot_l[gi], rot_r[gi], scale4[gi], g);
  const float4 mean = mean4[gi];
  const float* m = g.M[3];
  const float s44 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2] + m[3] * m[3];
  const float inv_s = 1.f / s44;
  float sig[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float* Mi = g.M[i];
    sig[i] = Mi[0] * m[0] + Mi[1] * m[1] + Mi[2] * m[2] + Mi[3] * m[3];
  }
  for (int v = 0; v < n_views; ++v) {
    const size_t slot = (size_t)v * n + gi;
    if (tiles[slot] == 0) continue;
    const DView& V = views[v];
    const float k = (V.t - mean.w) * inv_s;
    const float mu[3] = {fmaf(sig[0], k, mean.x), fmaf(sig[1], k, mean.y), fmaf(sig[2], k, mean.z)};
    const float step = dt * inv_s;
    float x[3], y[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float* W = V.W + 3 * r;
      x[r] = fmaf(W[0], mu[0], fmaf(W[1], mu[1], fmaf(W[2], mu[2], V.tau[r])));
      // displacement of the mean over dt, mapped to camera axes
      y[r] = x[r] + step * fmaf(W[0], sig[0], fmaf(W[1], sig[1], W[2] * sig[2]));
    }
    float2 out = make_float2(0.f, 0.f);
    if (x[2] > 0.f && y[2] > 0.f) {
      const float ix = 1.f / x[2], iy = 1.f / y[2];
      out.x = V.fx * (y[0] * iy - x[0] * ix);
      out.y = V.fy * (y[1] * iy - x[1] * ix);
    }
    flow[slot] = out;
  }
}

template <int DP>
__global__ __launch_bounds__(256) void k_feature_backward(
    int n, int d, const float* __restrict__ f, const float* __restrict__ gate,
    const float* __restrict__ fn, const float* __restrict__ fnorm,
    const float* __restrict__ dfn, float* __restrict__ d_features, float* __restrict__ d_gate) {
  constexpr int kRows = 64 / DP;
  const int lane = threadIdx.x & 63, c = lane % DP, sub = lane / DP;
  const float gc = c < d ? (gate ? gate[c] : 1.f) : 0.f;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t stride = ((int64_t)gridDim.x * blockDim.x >> 6) * kRows;
  float gacc = 0.f;  // this lane's part of dL/dgate[c]
  for (int64_t r0 = wave * kRows; r0 < n; r0 += stride) {
    const int64_t i = r0 + sub;
    const bool ok = i < n && c < d;
    const float nrm = ok ? fnorm[i] : 0.f;
    const bool live = ok && nrm > 0.f;
    const float fh = live ? fn[i * d + c] : 0.f, dh = live ? dfn[i * d + c] : 0.f;
    const float dot = group_sum<DP>(fh * dh);
    const float ds = live ? (dh - fh * dot) * (1.f / nrm) : 0.f;
    if (ok) d_features[i * d + c] = gc * ds;
    if (d_gate && live) gacc = fmaf(f[i * d + c], ds, gacc);
  }
  if (d_gate) {
#pragma unroll
    for (int o = 32; o >= DP; o >>= 1) gacc += __shfl_xor(gacc, o, 64);
    if (sub == 0 && c < d && gacc != 0.f) atomicAdd(d_gate + c, gacc);
  }
}

// Lanes per feature row for D features.
int row_lanes(int d) {
  int dp = 1;
  while (dp < d) dp <<= 1;
  return dp;
}

// Waves for `rows` rows at 64 / DP rows per wave step, capped so that each wave visits several
// rows (fewer dL/dgate atomics).
unsigned feature_blocks(int64_t rows, int dp) {
  const int64_t waves = (rows * dp + 63) / 64;
  const int64_t blocks = (waves + 3) / 4;
  return (unsigned)(blocks < 1024 ? blocks : 1024);
}

template <int DP>
void launch_feature_normalize(int n, int d, const float* f, const float* gate, float* fn,
                              float* fnorm, hipStream_t st) {
  hipLaunchKernelGGL(k_feature_normalize<DP>, dim3(feature_blocks(n, DP)), dim3(256), 0, st, n, d,
                     f, gate, fn, fnorm);
}

template <int DP>
void launch_feature_backward(int n, int d, const float* f, const float* gate, const float* fn,
                             const float* fnorm, const float* dfn, float* d_features,
                             float* d_gate, hipStream_t st) {
  hipLaunchKernelGGL(k_feature_backward<DP>, dim3(feature_blocks(n, DP)), dim3(256), 0, st, n, d,
                     f, gate, fn, fnorm, dfn, d_features, d_gate);
}

}  // namespace

void feature_normalize(int n, int d, const float* f, const float* gate, float* fn, float* fnorm,
                       hipStream_t st) {
  if (n <= 0 || d <= 0) return;
  switch (row_lanes(d)) {
    case 1: launch_feature_normalize<1>(n, d, f, gate, fn, fnorm, st); break;
    case 2: launch_feature_normalize<2>(n, d, f, gate, fn, fnorm, st); break;
    case 4: launch_feature_normalize<4>(n, d, f, gate, fn, fnorm, st); break;
    case 8: launch_feature_normalize<8>(n, d, f, gate, fn, fnorm, st); break;
    case 16: launch_feature_normalize<16>(n, d, f, gate, fn, fnorm, st); break;
    case 32: launch_feature_normalize<32>(n, d, f, gate, fn, fnorm, st); break;
    default: launch_feature_normalize<64>(n, d, f, gate, fn, fnorm, st); break;
  }
}

void flow_forward(const GaussPtrs& g, const DView* views, int n_views, const uint32_t* tiles,
                  float dt, float* flow, hipStream_t st) {
  if (g.n <= 0) return;
  hipLaunchKernelGGL(k_flow, dim3((g.n + 255) / 256), dim3(256), 0, st, g.n, n_views,
                     reinterpret_cast<const float4*>(g.mean4),
                     reinterpret_cast<const float4*>(g.scale4),
                     reinterpret_cast<const float4*>(g.rot_l),
                     reinterpret_cast<const float4*>(g.rot_r), views, tiles, dt,
                     reinterpret_cast<float2*>(flow));
}

void feature_backward(int n, int d, const float* f, const float* gate, const float* fn,
                      const float* fnorm, const float* dfn, float* d_features, float* d_gate,
                      hipStream_t st) {
  if (n <= 0 || d <= 0) return;
#define G4D_FB(DP) launch_feature_backward<DP>(n, d, f, gate, fn, fnorm, dfn, d_features, d_gate, st)
  switch (row_lanes(d)) {
    case 1: G4D_FB(1); break;
    case 2: G4D_FB(2); break;
    case 4: G4D_FB(4); break;
    case 8: G4D_FB(8); break;
    case 16: G4D_FB(16); break;
    case 32: G4D_FB(32); break;
    default: G4D_FB(64); break;
  }
#undef G4D_FB
}

}  // namespace g4d
