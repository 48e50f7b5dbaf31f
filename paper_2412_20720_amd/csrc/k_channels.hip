// Per-Gaussian work of the extra render channels (Sec. 7 feature rendering, Sec. 5
// rendered depth, Sec. 8.1 rendered flow); their compositing lives in the raster kernels.
//
//   feature_normalize: f_hat = s / |s| with s = gate * f (0 when s = 0), one thread per Gaussian.
//   flow_forward:      per visible (view, Gaussian) slot, the image displacement of the
//                      conditional mean between t and t + dt.  The mean moves linearly in t,
//                      mu(t') = mu(t) + Sigma_{1:3,4} / Sigma_44 (t' - t), so one slice suffices.
//   feature_backward:  dL/ds = (dL/df_hat - f_hat (f_hat . dL/df_hat)) / |s|,
//                      dL/df = gate * dL/ds, dL/dgate = sum_i f_i * dL/ds_i (wave sums, then
//                      one atomic per channel and wave).
#include <hip/hip_runtime.h>

#include "g4d_internal.h"

namespace g4d {
namespace {

__global__ __launch_bounds__(256) void k_feature_normalize(int n, int d,
                                                           const float* __restrict__ f,
                                                           const float* __restrict__ gate,
                                                           float* __restrict__ fn,
                                                           float* __restrict__ fnorm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* fi = f + (size_t)i * d;
  float n2 = 0.f;
  for (int c = 0; c < d; ++c) {
    const float s = (gate ? gate[c] : 1.f) * fi[c];
    n2 = fmaf(s, s, n2);
  }
  const float nrm = sqrtf(n2);
  const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
  float* o = fn + (size_t)i * d;
  for (int c = 0; c < d; ++c) o[c] = (gate ? gate[c] : 1.f) * fi[c] * inv;
  fnorm[i] = nrm;
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

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__global__ __launch_bounds__(256) void k_feature_backward(
    int n, int d, const float* __restrict__ f, const float* __restrict__ gate,
    const float* __restrict__ fn, const float* __restrict__ fnorm,
    const float* __restrict__ dfn, float* __restrict__ d_features, float* __restrict__ d_gate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const float nrm = valid ? fnorm[i] : 0.f;
  const bool live = valid && nrm > 0.f;
  const size_t row = live ? (size_t)i * d : 0;
  float dot = 0.f;
  for (int c = 0; c < d; ++c)
    if (live) dot = fmaf(fn[row + c], dfn[row + c], dot);
  const float inv = live ? 1.f / nrm : 0.f;
  // every lane stays in the loop (the wave sums below need all 64)
  for (int c = 0; c < d; ++c) {
    const float ds = live ? (dfn[row + c] - fn[row + c] * dot) * inv : 0.f;
    if (valid) d_features[(size_t)i * d + c] = (gate ? gate[c] : 1.f) * ds;
    if (d_gate) {
      const float part = wave_sum(live ? f[(size_t)i * d + c] * ds : 0.f);
      if ((threadIdx.x & 63) == 0 && part != 0.f) atomicAdd(d_gate + c, part);
    }
  }
}

}  // namespace

void feature_normalize(int n, int d, const float* f, const float* gate, float* fn, float* fnorm,
                       hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_feature_normalize, dim3((n + 255) / 256), dim3(256), 0, st, n, d, f, gate,
                     fn, fnorm);
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
  hipLaunchKernelGGL(k_feature_backward, dim3((n + 255) / 256), dim3(256), 0, st, n, d, f, gate,
                     fn, fnorm, dfn, d_features, d_gate);
}

}  // namespace g4d
