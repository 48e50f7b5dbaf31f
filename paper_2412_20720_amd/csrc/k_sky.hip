// Sky composite of urban scenes (Sec. 5): I = I_gs + (1 - O_gs) M_sky(r), where M_sky is a
// learnable cube map queried by the world direction r of each pixel's ray.  With
// O_gs = 1 - T_final this is the image with M_sky(r) as a per-pixel background, so the forward
// writes that background (k_sky) and the raster kernels read it; the adjoint of the lookup,
// dL/dM_sky += T_final dL/dI spread with the bilinear weights, is k_sky_backward.
//
// Cube-map convention (OpenGL): faces +x, -x, +y, -y, +z, -z picked by the largest |component|
// of r (ties to x, then y); face coordinates s = (sc / |ma| + 1) / 2, t = (tc / |ma| + 1) / 2;
// texel (i, j) centred at ((i + 1/2) / R, (j + 1/2) / R); bilinear within the face, clamped at
// its edges.  Grid y = view; the lookup takes one thread per pixel.
#include <hip/hip_runtime.h>

#include "g4d_internal.h"

namespace g4d {
namespace {

struct CubeTap {
  int idx[4];   // float offsets of the four texels (channel 0)
  float w[4];   // their bilinear weights
  int base;     // texel (face, y0, x0) before clamping, the same for a whole footprint
};

__device__ __forceinline__ CubeTap cube_tap(const DView& V, int px, int py, int R) {
  const float dx = ((float)px + 0.5f - V.cx) / V.fx, dy = ((float)py + 0.5f - V.cy) / V.fy;
  float r[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) r[j] = fmaf(V.W[j], dx, fmaf(V.W[3 + j], dy, V.W[6 + j]));
  const float ax = fabsf(r[0]), ay = fabsf(r[1]), az = fabsf(r[2]);
  int face;
  float sc, tc, ma;
  if (ax >= ay && ax >= az) {
    face = r[0] >= 0.f ? 0 : 1;
    ma = ax;
    sc = r[0] >= 0.f ? -r[2] : r[2];
    tc = -r[1];
  } else if (ay >= az) {
    face = r[1] >= 0.f ? 2 : 3;
    ma = ay;
    sc = r[0];
    tc = r[1] >= 0.f ? r[2] : -r[2];
  } else {
    face = r[2] >= 0.f ? 4 : 5;
    ma = az;
    sc = r[2] >= 0.f ? r[0] : -r[0];
    tc = -r[1];
  }
  const float im = 1.f / ma;
  const float x = 0.5f * fmaf(sc, im, 1.f) * (float)R - 0.5f;
  const float y = 0.5f * fmaf(tc, im, 1.f) * (float)R - 0.5f;
  const float fx = floorf(x), fy = floorf(y);
  const float wx = x - fx, wy = y - fy;
  const int x0 = (int)fx, y0 = (int)fy;
  const int xa = min(max(x0, 0), R - 1), xb = min(max(x0 + 1, 0), R - 1);
  const int ya = min(max(y0, 0), R - 1), yb = min(max(y0 + 1, 0), R - 1);
  CubeTap t;
  const int fb = face * R * R;
  t.idx[0] = 3 * (fb + ya * R + xa);
  t.idx[1] = 3 * (fb + ya * R + xb);
  t.idx[2] = 3 * (fb + yb * R + xa);
  t.idx[3] = 3 * (fb + yb * R + xb);
  t.w[0] = (1.f - wx) * (1.f - wy);
  t.w[1] = wx * (1.f - wy);
  t.w[2] = (1.f - wx) * wy;
  t.w[3] = wx * wy;
  t.base = (face * (R + 2) + (y0 + 1)) * (R + 2) + (x0 + 1);
  return t;
}

__global__ __launch_bounds__(256) void k_sky(const DView* __restrict__ views,
                                             const float* __restrict__ cube, int R,
                                             float* __restrict__ bg) {
  const DView& V = views[blockIdx.y];
  const int64_t hw = (int64_t)V.width * V.height;
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= hw) return;
  const int px = (int)(pix % V.width), py = (int)(pix / V.width);
  const CubeTap t = cube_tap(V, px, py, R);
  float* o = bg + 3 * (int64_t)V.pix_base + pix;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float v = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) v = fmaf(t.w[k], cube[t.idx[k] + c], v);
    o[c * hw] = v;
  }
}

// Adjoint: each thread walks a kPatchX x kPatchY patch of pixels row by row and keeps the 12
// partial sums (4 texels x 3 channels) of up to kSlots bilinear footprints; a footprint's sums
// are added to the cube-map gradient when its slot is reused (round robin) or at the end.
// Texels are larger than pixels, so a patch meets few footprints and the device-scope atomics
// drop to a fraction of one per pixel.  Slots are indexed with compile-time constants only
// (selects, no dynamic register indexing).  Measured on the 300k/16-view workload with a 256^2
// cube map (texels of about 10 pixels): 8 x 8 patches with 4 slots are fastest (sky step 6.62
// ms against 7.25 at 16 x 8, 8.1 at 32 x 8 with 6 slots, 7.05 at 8 x 8 with 2 slots).
#ifndef G4D_SKY_PATCH_X
#define G4D_SKY_PATCH_X 8
#endif
#ifndef G4D_SKY_PATCH_Y
#define G4D_SKY_PATCH_Y 8
#endif
#ifndef G4D_SKY_SLOTS
#define G4D_SKY_SLOTS 4
#endif
constexpr int kPatchX = G4D_SKY_PATCH_X, kPatchY = G4D_SKY_PATCH_Y, kSlots = G4D_SKY_SLOTS;

__device__ __forceinline__ void flush(float* d_cube, const int* idx, const float acc[4][3]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (acc[k][c] != 0.f) atomicAdd(d_cube + idx[k] + c, acc[k][c]);
}

__global__ __launch_bounds__(256) void k_sky_backward(const DView* __restrict__ views, int R,
                                                      const float* __restrict__ px_T,
                                                      const float* __restrict__ dL,
                                                      float* __restrict__ d_cube) {
  const DView& V = views[blockIdx.y];
  const int64_t hw = (int64_t)V.width * V.height;
  const int px_per_row = (V.width + kPatchX - 1) / kPatchX;
  const int64_t patch = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t patches = (int64_t)px_per_row * ((V.height + kPatchY - 1) / kPatchY);
  if (patch >= patches) return;
  const int x0 = (int)(patch % px_per_row) * kPatchX, y0 = (int)(patch / px_per_row) * kPatchY;
  int base[kSlots], idx[kSlots][4];
  float acc[kSlots][4][3];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    base[s] = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      idx[s][k] = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[s][k][c] = 0.f;
    }
  }
  int next = 0;  // slot to reuse next
  for (int dy = 0; dy < kPatchY; ++dy) {
    const int py = y0 + dy;
    if (py >= V.height) break;
    for (int dx = 0; dx < kPatchX; ++dx) {
      const int px = x0 + dx;
      if (px >= V.width) break;
      const int64_t pix = (int64_t)py * V.width + px;
      const CubeTap t = cube_tap(V, px, py, R);
      int hit = -1;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) hit = base[s] == t.base ? s : hit;
      if (hit < 0) {
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
          if (s == next) {
            if (base[s] >= 0) flush(d_cube, idx[s], acc[s]);
            base[s] = t.base;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              idx[s][k] = t.idx[k];
#pragma unroll
              for (int c = 0; c < 3; ++c) acc[s][k][c] = 0.f;
            }
          }
        }
        hit = next;
        next = next + 1 == kSlots ? 0 : next + 1;
      }
      const float T = px_T[V.pix_base + pix];
      const float* d = dL + 3 * (int64_t)V.pix_base + pix;
      float g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = T * d[c * hw];
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const bool h = s == hit;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float w = h ? t.w[k] : 0.f;
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[s][k][c] = fmaf(w, g[c], acc[s][k][c]);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < kSlots; ++s)
    if (base[s] >= 0) flush(d_cube, idx[s], acc[s]);
}

}  // namespace

void sky_forward(const DView* views, int n_views, int max_pixels, const float* cube, int R,
                 float* bg, hipStream_t st) {
  if (n_views <= 0 || max_pixels <= 0) return;
  hipLaunchKernelGGL(k_sky, dim3((unsigned)((max_pixels + 255) / 256), (unsigned)n_views),
                     dim3(256), 0, st, views, cube, R, bg);
}

void sky_backward(const DView* views, int n_views, int max_width, int max_height, int R,
                  const float* px_T, const float* dL, float* d_cube, hipStream_t st) {
  if (n_views <= 0 || max_width <= 0 || max_height <= 0) return;
  const int64_t patches = (int64_t)((max_width + kPatchX - 1) / kPatchX) *
                          ((max_height + kPatchY - 1) / kPatchY);
  hipLaunchKernelGGL(k_sky_backward, dim3((unsigned)((patches + 255) / 256), (unsigned)n_views),
                     dim3(256), 0, st, views, R, px_T, dL, d_cube);
}

}  // namespace g4d
