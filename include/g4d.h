/* g4d: differentiable render of native 4D Gaussians on AMD Instinct MI355X (gfx950).
 *
 * Method: "4D Gaussian Splatting: Modeling Dynamic Scenes with Native 4D Primitives"
 * (arXiv 2412.20720).  A pixel (u, v) of a view with extrinsic E, intrinsic K and time t is
 *   I(u, v, t) = sum_i p_i(t) p_i(u, v | t) alpha_i c_i(d, dt) prod_{j<i} (1 - p_j(t) p_j(u, v | t) alpha_j)
 * (Sec. 3.2, eq:4dblending), where p_i(t) is the temporal marginal and p_i(u, v | t) the EWA
 * splat (Sec. 3.1, eq:meansplatting / eq:covsplatting) of the conditional 3D Gaussian of the
 * 4D Gaussian i at time t (Sec. 3.2, conditional mean and covariance), whose covariance is
 * R S S^T R^T with R = L(q_l) R(q_r) built from two rotors (Sec. 3.2, 4D rotation), and
 * c_i is a 4D spherindrical-harmonic color (Sec. 3.2).
 *
 * Conventions of this ABI:
 *   - Pointers are device pointers (hipMalloc / PyTorch CUDA tensors) unless marked (host).
 *   - Arrays are float32, row-major, structure of arrays.  Nothing is ever freed or kept by
 *     the library beyond the call except inside the context.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default stream).
 *   - Errors are returned as g4d_status; no exception crosses the ABI.  The message of the last
 *     error is g4d_last_error(ctx).  One context must not be used by two threads at once, and
 *     its calls should stay on one stream (the context keeps device state between calls, for
 *     instance the view table, and reuses it in stream order).
 */
#ifndef G4D_H
#define G4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define G4D_VERSION 1
/* Floats per (view, Gaussian) record written by g4d_preprocess (layout below). */
#define G4D_RECORD_FLOATS 12
/* Maximum views in one call, maximum image side, and maximum SH / Fourier degrees. */
#define G4D_MAX_VIEWS 256
#define G4D_MAX_SIDE 8192
#define G4D_MAX_SH_DEGREE 3
#define G4D_MAX_T_DEGREE 2

typedef struct g4d_ctx g4d_ctx;

typedef enum {
  G4D_OK = 0,
  G4D_EINVAL = -1,    /* an argument failed a host-side check; nothing was enqueued */
  G4D_ENOMEM = -2,    /* a device allocation failed */
  G4D_ECAPACITY = -3, /* more (Gaussian, tile) pairs than the fixed capacity of a captured graph,
                         or more than 2^31 - 1 in one call */
  G4D_EHIP = -4,      /* a HIP runtime call failed */
  G4D_ESTATE = -5     /* backward without a matching forward in this context */
} g4d_status;

/* A set of N 4D Gaussians (Sec. 3.2, "Representation of 4D Gaussian"):
 *   mean4   [N,4]  (mu_x, mu_y, mu_z, mu_t)
 *   scale4  [N,4]  (s_x, s_y, s_z, s_t) > 0, already activated
 *   rot_l   [N,4]  left rotor (a, b, c, d); any nonzero length, normalized inside
 *   rot_r   [N,4]  right rotor (p, q, r, s); any nonzero length, normalized inside
 *   opacity [N]    in [0, 1], already activated
 *   sh      [N, t_degree+1, (sh_degree+1)^2, 3]  4DSH coefficients k[n, l*l+l+m, channel]
 *           (Sec. 3.2, Z = cos(2 pi n dt / T) Y_l^m; real Y without Condon-Shortley phase).
 *   mask    [N]    optional (NULL: none) significance M of the volume mask (Sec. 4.3,
 *           eq. mask_prune), already activated: the forward uses M_hat = 1{M > mask_threshold},
 *           scales and opacity multiplied by M_hat, so a Gaussian with M <= mask_threshold is
 *           removed; the backward's dL/dM is straight-through (dM_hat/dM = 1).
 * sh_degree in 0..3, t_degree in 0..2, N >= 0.  A Gaussian with a non-finite value in any of
 * its arrays is culled in every view and gets zero gradient. */
typedef struct {
  int32_t n, sh_degree, t_degree;
  const float *mean4, *scale4, *rot_l, *rot_r, *opacity, *sh;
  const float *mask;
  float mask_threshold;
} g4d_gaussians;

/* Gradients, same shapes as g4d_gaussians; overwritten (not accumulated) with the sum over
 * the call's views.  Any pointer may be NULL to skip that group.
 *   mask     [N]    dL/dM = sum_j s_j dL/ds_j + opacity dL/d(opacity) for a kept Gaussian, 0
 *                   for a removed one (without g4d_gaussians.mask every Gaussian is kept);
 *   densify  [N,3]  densification statistics of the call (Sec. 3.3, densification in
 *                   spacetime): sum over the views where the Gaussian is listed in a tile of
 *                   |dL/d(u, v)| (screen-space mean, pixels), |dL/d mu_t| (of the summed
 *                   gradient), and the number of such views. */
typedef struct {
  float *mean4, *scale4, *rot_l, *rot_r, *opacity, *sh;
  float *mask, *densify;
} g4d_grads;

/* (host) One view: pinhole intrinsics K = (fx, fy, cx, cy), extrinsic world->camera
 * E = [R | tau] row-major 3x4 with OpenCV axes (x right, y down, z forward), time t and
 * background color (Sec. 3.1 renders a pixel (u, v) of a view from its extrinsic E and
 * intrinsic K; Sec. 3.2 adds the timestamp t).  Pixel (i, j) is sampled at (i + 0.5, j + 0.5). */
typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float world_to_cam[12];
  float t;
  float background[3];
} g4d_view;

/* (host) Render settings.  The paper leaves these unstated except the marginal filter
 * (p(t) threshold, Sec. 8.1 implementation details); g4d_default_settings fills in:
 *   near_z 0.2        cull when the camera-space depth of the sliced mean is <= near_z (> 0)
 *   marginal_min 1/255 cull when p(t) < marginal_min (the paper quotes 0.05)
 *   cutoff_sigma 3    a splat covers pixels with Mahalanobis distance <= cutoff_sigma
 *   blur 0.3          EWA low-pass: added to both diagonal entries of the 2D covariance (px^2)
 *   jacobian_margin 0.15  the perspective Jacobian is evaluated at x/z, y/z clamped to the
 *                     image widened by this fraction on each side
 *   alpha_min 1/255   contributions with alpha below this are skipped (must be > 0)
 *   alpha_max 0.99    alpha = min(alpha_max, opacity p(t) p(u, v | t)); alpha_min <=
 *                     alpha_max < 1 (the backward divides by 1 - alpha)
 *   T_min 1e-4        a pixel stops before the Gaussian that would take T below T_min
 *   color_offset 0.5, color_min 0   c = max(color_min, color_offset + 4DSH sum)
 *   time_period 1     the period T of the Fourier basis of the 4DSH
 *   tile_size 16      screen tile side in pixels (8, 16 or 32)
 *   lds_batch 0       list entries a wave stages in LDS at a time: 32, 64 or 128
 *                     (0 = library default, 64)
 *   px_per_lane 0     pixels per lane of the raster waves: 1 (8x8 block per wave), 2 (16x8)
 *                     or 4 (16x16); 2 and 4 need tile_size >= 16 (0 = library default:
 *                     4, or 1 for 8-pixel tiles)
 *   bwd_px_per_lane 0 pixels per lane of the backward raster waves: 1, 2, 4 as above, or 8
 *                     (32x16 blocks, tile_size 32 only); 0 = library default: 8 at 32-pixel
 *                     tiles when the forward takes 4, else the forward's value.  The backward
 *                     reads only per-pixel state of the forward, so the two may differ.
 * Tile size, batch and pixels per lane change the work decomposition only, never the image. */
typedef struct {
  float near_z, marginal_min, cutoff_sigma, blur, jacobian_margin;
  float alpha_min, alpha_max, T_min, color_offset, color_min, time_period;
  int32_t tile_size, lds_batch, px_per_lane, bwd_px_per_lane;
} g4d_settings;

/* Work counters of the last forward (host). */
typedef struct {
  int64_t n_slots;      /* N * n_views */
  int64_t n_visible;    /* (view, Gaussian) slots that survived every cull and touch a tile */
  int64_t n_pairs;      /* (Gaussian, tile) pairs sorted */
  int64_t n_tiles;      /* screen tiles over all views */
  int64_t n_pixels;     /* pixels over all views */
  int64_t pair_capacity;
  int64_t n_clamped_batches; /* LDS batches of the last backward that ran the raster's entry loop
                                with the alpha_max clamp (an entry's opacity p(t) reaches it);
                                counted only while g4d_eval_counters is enabled, else -1 */
} g4d_stats;

/* Fill *s with the defaults listed above.  Returns G4D_EINVAL if s is NULL. */
g4d_status g4d_default_settings(g4d_settings *s);

/* Create a context on HIP device `device`.  The context owns all scratch memory (grown on
 * demand) and the state a forward leaves for its backward.  *out is NULL on failure. */
g4d_status g4d_create(g4d_ctx **out, int device);

/* Free the context and everything it owns (synchronizes its device first). */
g4d_status g4d_destroy(g4d_ctx *ctx);

/* Message of the last error on this context (never NULL; "" if none). */
const char *g4d_last_error(const g4d_ctx *ctx);

/* Per-(view, Gaussian) slice and splat only (Sec. 3.2 conditional Gaussian and marginal p(t);
 * Sec. 3.1 eq:meansplatting, eq:covsplatting; 4DSH color).  Writes
 *   records [n_views][N][G4D_RECORD_FLOATS]:
 *     0 u, 1 v (screen mean, px), 2..4 conic (a, b, c) = inverse 2D covariance,
 *     5 opacity * p(t), 6..8 rgb, 9..10 half extents (px) of the box of the reach ellipse
 *     (where alpha can still reach alpha_min, within the cutoff), 11 camera-space depth;
 *   tiles [n_views][N] int32: number of screen tiles with a pixel centre inside the reach
 *     ellipse, 0 if culled or if the splat can reach no pixel.
 * Either output may be NULL. */
g4d_status g4d_preprocess(g4d_ctx *ctx, const g4d_gaussians *g, const g4d_view *views,
                          int32_t n_views, const g4d_settings *s, float *records, int32_t *tiles,
                          void *stream);

/* Forward render of n_views views in one batch (Sec. 3.2, eq:4dblending, composited with the
 * tile-based rasterizer that Sec. 3.2 takes over from 3D Gaussian splatting):
 *   out_rgb: per view planar [3][H][W], views concatenated in order;
 *   out_T:   per view [H][W] final transmittance (may be NULL).
 * Saves the state its backward needs in ctx. */
g4d_status g4d_render_forward(g4d_ctx *ctx, const g4d_gaussians *g, const g4d_view *views,
                              int32_t n_views, const g4d_settings *s, float *out_rgb,
                              float *out_T, void *stream);

/* Backward of the last forward on this context with the same g, views and settings
 * (else G4D_ESTATE): given dL/d(out_rgb) in the out_rgb layout, writes dL/d(parameters),
 * summed over the views, into *out (derivative of eq:4dblending through the splat, the
 * slice, the rotors and their normalization, and the 4DSH color; discrete decisions frozen). */
g4d_status g4d_render_backward(g4d_ctx *ctx, const g4d_gaussians *g, const g4d_view *views,
                               int32_t n_views, const g4d_settings *s, const float *dL_drgb,
                               const g4d_grads *out, void *stream);

/* Extra channels rendered with the same weights T alpha as the image (Sec. 7: the 2D feature
 * map of 4D segmentation, the color replaced by the normalized scale-gated feature; Sec. 5: the
 * rendered depth of the urban LiDAR loss; Sec. 8.1: the rendered optical flow, the image
 * displacement of each conditional mean between t and t + flow_dt).  The channels of a pixel
 * are, in order: n_features feature channels, then the depth channel (if depth), then du, dv
 * (if flow); E = n_features + depth + 2 flow <= G4D_MAX_CHANNELS.  Their background is 0.
 *   features: device [N][n_features] float32, row-major (NULL iff n_features = 0); each
 *             Gaussian's f is gated and normalized, f_hat = (gate * f) / |gate * f| (0 when
 *             gate * f = 0);
 *   gate:     device [n_features] float32 (the scale gate S(s)), or NULL for all ones;
 *   depth:    camera-space z of the sliced mean;
 *   flow:     (u, v)(t + flow_dt) - (u, v)(t) of the projected conditional mean, 0 where the
 *             moved mean is not in front of the camera.  Flow is forward only. */
#define G4D_MAX_CHANNELS 36
typedef struct {
  int32_t n_features;
  const float *features, *gate;
  int32_t depth, flow;
  float flow_dt;
} g4d_channels;

/* g4d_render_forward plus the extra channels of *ch:
 *   out_ch: per view planar [E][H][W], views concatenated in order (caller-owned device memory).
 * Rasterization uses 64-entry LDS batches whatever s->lds_batch says and two pixels per lane
 * (one if s->px_per_lane is 1 or tile_size is 8); tile_size is honored.  out_rgb and out_T are
 * bit-identical to g4d_render_forward's.  Saves the state g4d_render_channels_backward needs. */
g4d_status g4d_render_channels_forward(g4d_ctx *ctx, const g4d_gaussians *g,
                                       const g4d_view *views, int32_t n_views,
                                       const g4d_settings *s, const g4d_channels *ch,
                                       float *out_rgb, float *out_T, float *out_ch, void *stream);

/* Backward of the last g4d_render_channels_forward on this context with the same g, views,
 * settings and *ch (else G4D_ESTATE): given dL/d(out_rgb) and dL/d(out_ch) (same layout as
 * out_ch, or NULL for zero; its flow channels are ignored), writes dL/d(parameters) into *out,
 * dL/d(features) [N][n_features] into d_features and dL/d(gate) [n_features] into d_gate, all
 * summed over the views and overwritten.  d_features may be NULL only when n_features is 0;
 * d_gate may be NULL (then not computed).  The depth channel's gradient reaches the Gaussians
 * through the sliced mean.  g4d_render_backward after g4d_render_channels_forward gives the
 * image gradients alone. */
g4d_status g4d_render_channels_backward(g4d_ctx *ctx, const g4d_gaussians *g,
                                        const g4d_view *views, int32_t n_views,
                                        const g4d_settings *s, const g4d_channels *ch,
                                        const float *dL_drgb, const float *dL_dch,
                                        const g4d_grads *out, float *d_features, float *d_gate,
                                        void *stream);

/* Sky of urban scenes (Sec. 5): I = I_gs + (1 - O_gs) M_sky(r) = C + T_final M_sky(r), a
 * learnable cube map M_sky queried by the world direction r of each pixel's ray.
 *   cube:       device [6][R][R][3] float32, faces +x, -x, +y, -y, +z, -z (OpenGL convention:
 *               the largest |component| of r picks the face, ties to x then y; face coordinates
 *               s = (sc / |ma| + 1) / 2, t = (tc / |ma| + 1) / 2; texel [face][j][i] centred at
 *               ((i + 1/2) / R, (j + 1/2) / R); bilinear within the face, clamped at its edges);
 *   resolution: R, 1 <= R <= G4D_MAX_SKY_RES.
 * The sky replaces the views' constant background. */
#define G4D_MAX_SKY_RES 4096
typedef struct {
  const float *cube;
  int32_t resolution;
} g4d_sky;

/* g4d_render_forward with the sky as each pixel's background.  Saves the state
 * g4d_render_sky_backward needs. */
g4d_status g4d_render_sky_forward(g4d_ctx *ctx, const g4d_gaussians *g, const g4d_view *views,
                                  int32_t n_views, const g4d_settings *s, const g4d_sky *sky,
                                  float *out_rgb, float *out_T, void *stream);

/* Backward of the last g4d_render_sky_forward with the same inputs and *sky (else
 * G4D_ESTATE): the parameter gradients into *out as g4d_render_backward, and dL/d(cube)
 * [6][R][R][3] into d_cube (overwritten; may be NULL), summed over the views. */
g4d_status g4d_render_sky_backward(g4d_ctx *ctx, const g4d_gaussians *g, const g4d_view *views,
                                   int32_t n_views, const g4d_settings *s, const g4d_sky *sky,
                                   const float *dL_drgb, const g4d_grads *out, float *d_cube,
                                   void *stream);

/* Compact 4DGS (Sec. 4.2 parameter compression; codebook sizes of Sec. 8.3).  Residual vector
 * quantization stores per Gaussian one index into each codebook of a model and decodes the
 * sum of the selected codewords:
 *   scale4  = exp(sum_k scale_cb[k][scale_idx[i][k]])   (6 codebooks of 64 x 4, log space)
 *   rot_l   = sum_k rot_cb[k][rot_l_idx[i][k]], rot_r likewise with rot_r_idx (one model of 6
 *             codebooks of 64 x 4 shared by both rotors)
 *   sh[i][0][0][:] = sum_k dc_cb[k][dc_idx[i][k]]   (6 x 64 x 3, the direct component)
 *   the other K - 3 coefficients of sh[i], in order, = sum_k rest_cb[k][rest_idx[i][k]]
 *             (8 codebooks of 256 x (K - 3)), K = (t_degree + 1)(sh_degree + 1)^2 3
 *   mean4   = the IEEE half values mean4_h[i][0..3]
 *   opacity = opacity_lo + (opacity_hi - opacity_lo) opacity_q[i] / 255 (8-bit min-max).
 * Index arrays are row-major uint8 [N][6] ([N][8] for rest_idx), codebooks row-major float32;
 * all arrays are device memory. */
typedef struct {
  int32_t n, sh_degree, t_degree;
  const uint16_t *mean4_h;
  const uint8_t *scale_idx, *rot_l_idx, *rot_r_idx, *opacity_q, *dc_idx, *rest_idx;
  float opacity_lo, opacity_hi;
  const float *scale_cb, *rot_cb, *dc_cb, *rest_cb;
} g4d_compact;

/* Decode a compact model into the full parameter arrays of g4d_gaussians (device, caller
 * owned; for training or fine-tuning with g4d_render_forward/_backward). */
g4d_status g4d_decode_compact(g4d_ctx *ctx, const g4d_compact *c, float *mean4, float *scale4,
                              float *rot_l, float *rot_r, float *opacity, float *sh,
                              void *stream);

/* Forward render of a compact model, decoding inside the per-Gaussian preprocess (no full
 * parameter arrays are read or written).  Same outputs as g4d_render_forward; it leaves no
 * state for a backward (decode first to train). */
g4d_status g4d_render_compact_forward(g4d_ctx *ctx, const g4d_compact *c, const g4d_view *views,
                                      int32_t n_views, const g4d_settings *s, float *out_rgb,
                                      float *out_T, void *stream);

/* Flags of g4d_render_step. */
#define G4D_STEP_GRAPH 1

/* One training-style step: g4d_render_forward then g4d_render_backward with dL_drgb (the
 * whole differentiable render of Sec. 3.2 and its derivative for a batch of views).  With
 * flags & G4D_STEP_GRAPH the step is captured once into a hipGraph and replayed on later calls
 * with the same inputs, views, settings and buffer addresses (parameter and dL values may
 * change between calls): no host synchronization, allocation or per-kernel launch happens in
 * a replay.  The first call (and any call whose key changed) runs one eager step on a private
 * context to size the buffers, then captures with pair and row-run capacities 25% above the
 * counts it found; if a later replay finds more, g4d_sync_status reports G4D_ECAPACITY, the
 * outputs of that replay are undefined, and the graph is dropped so that the next call with
 * G4D_STEP_GRAPH sizes and captures it again. */
g4d_status g4d_render_step(g4d_ctx *ctx, const g4d_gaussians *g, const g4d_view *views,
                           int32_t n_views, const g4d_settings *s, const float *dL_drgb,
                           float *out_rgb, float *out_T, const g4d_grads *grads, int32_t flags,
                           void *stream);

/* For callers that cannot allocate device memory (code that must not call hipMalloc, such as
 * tight serving loops or harnesses that forbid it): g4d_render_step without G4D_STEP_GRAPH,
 * with the same arguments, outputs and numerics, whose every scratch buffer is a slice of one
 * fixed device array of G4D_NOALLOC_SCRATCH_BYTES bytes.  Each GPU the library runs on holds
 * its own copy of that array from the first g4d_create on it until the process ends; the call
 * allocates no device memory and no pinned host memory (no hipMalloc, hipHostMalloc, hipFree).
 *   Limit: the records, counts and sort buffers of N * n_views slots, the per-pixel state of
 *   all views and the (Gaussian, tile) pairs must fit in the array together (about
 *   124 B per slot + 8 B per pixel + 8 B per tile + 40 B per tile row + 16 B per pair, the
 *   pair list and the binning's row runs, of which there may be up to half as many as pairs;
 *   a 100k-Gaussian view of 1352x1014 fits).  Sizes known before launching are rejected at
 *   once with G4D_ECAPACITY and nothing enqueued; a pair or run count above what remains is
 *   found when the call reads it (it waits on the host once, as g4d_render_forward does) and
 *   returned as G4D_ECAPACITY, the outputs then undefined.
 *   All calls on one GPU share its array and leave their contents in it: the call clears what
 *   must start at zero itself, and calls that overlap on one GPU (other streams, threads or
 *   contexts) race and give undefined results.  The call keeps no state for g4d_render_backward
 *   and does not touch the context's own forward state.  g4d_sync_status(ctx) also reports
 *   device-detected errors of the last such call on the device. */
#define G4D_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
g4d_status g4d_render_step_noalloc(g4d_ctx *ctx, const g4d_gaussians *g, const g4d_view *views,
                                   int32_t n_views, const g4d_settings *s, const float *dL_drgb,
                                   float *out_rgb, float *out_T, const g4d_grads *grads,
                                   void *stream);

/* Wait for the context's work on `stream` and report errors found on the device
 * (G4D_ECAPACITY when a pair or row-run capacity was exceeded; outputs are then
 * undefined).  An error is reported once: the flag is cleared. */
g4d_status g4d_sync_status(g4d_ctx *ctx, void *stream);

/* Counters of the last forward; synchronizes `stream`. */
g4d_status g4d_get_stats(g4d_ctx *ctx, g4d_stats *out, void *stream);

/* Binning of the last forward on this context, for checks and tools (the depth-ordered,
 * tile-sorted list that the tile-based rasterizer of Sec. 3.2 walks): copies into caller device
 * buffers, each of which may be NULL,
 *   tile_ids [n_pairs] uint32: global tile id of every (tile, splat) pair, sorted ascending
 *            (tiles of all views numbered consecutively, view by view, row-major in a view);
 *   slots    [n_pairs] uint32: the (view, Gaussian) slot view * N + g of each pair; within a tile
 *            the slots are in ascending camera depth, ties by ascending slot;
 *   ranges   [n_tiles][2] uint32: [first, end) of each tile's pairs (0, 0 for an empty tile).
 * n_pairs and n_tiles are those of g4d_get_stats.  G4D_ESTATE if the context holds no forward
 * whose binning is kept (a later g4d_preprocess or a compact forward discards it). */
g4d_status g4d_get_pairs(g4d_ctx *ctx, uint32_t *tile_ids, uint32_t *slots, uint32_t *ranges,
                         void *stream);

/* Per-pixel work counters of eq:4dblending: bits 0-15 hold the number of (Gaussian, pixel)
 * pairs that the pixel evaluates before its transmittance stop, bits 16-31 the number of those
 * that were composited (both saturate at 65535).  enable = 1 makes later forwards count them
 * (one extra store per pixel), counting the pairs within each splat's reach (the cutoff, or
 * the smaller radius beyond which alpha < alpha_min: the pairs the backward evaluates);
 * enable = 2 counts every pair within the plain cutoff instead, binning the splats by the
 * cutoff for those forwards (more (Gaussian, tile) pairs, the same image); 0 stops.
 * If `out` (device, [total pixels] uint32, views concatenated) is not NULL, the counters of
 * the last counted forward are copied there (G4D_ESTATE if there is none). */
g4d_status g4d_eval_counters(g4d_ctx *ctx, int enable, uint32_t *out, void *stream);

/* Autotuner: picks tile_size, lds_batch and px_per_lane for this problem shape (N, SH and
 * Fourier degrees, view count and sizes, cutoff and thresholds) by timing `reps` forward +
 * backward passes of every valid combination with HIP events on `stream`, and writes the
 * fastest into *s (other fields are kept).  The choice changes the work decomposition only,
 * never the image (eq:4dblending is evaluated per pixel with the same cutoff).  Results are
 * cached in the context per shape; a cached shape returns at once.  out_rgb, out_T (may be
 * NULL), dL_drgb and grads are caller buffers of the g4d_render_forward / backward layouts,
 * overwritten.  *best_ms (may be NULL) receives the time of the chosen setting. */
g4d_status g4d_autotune(g4d_ctx *ctx, const g4d_gaussians *g, const g4d_view *views,
                        int32_t n_views, g4d_settings *s, const float *dL_drgb, float *out_rgb,
                        float *out_T, const g4d_grads *grads, int32_t reps, double *best_ms,
                        void *stream);

/* Pipeline stages timed by g4d_profile (index: name). */
#define G4D_NUM_STAGES 8
/* Stage timing with HIP events recorded on the call's stream around each kernel group:
 *   0 preprocess, 1 depth_sort (each view's listed slots), 2 splat_rows (splats to
 *   per-tile-row runs), 3 row_tiles (runs to the tile lists), 4 raster_fwd, 5 clear_grad,
 *   6 raster_bwd, 7 preprocess_bwd.
 * enable = 1 starts recording for later calls, 0 stops.  If ms / launches are not NULL
 * (host arrays of G4D_NUM_STAGES), the context's device is synchronized, every recorded
 * interval is added in and the totals since the last reset are returned; reset = 1 then
 * clears the totals. */
g4d_status g4d_profile(g4d_ctx *ctx, int enable, double *ms, int64_t *launches, int reset);

/* Stages that g4d_profile records while enabled: bit s for stage s (the default, set at
 * g4d_create, is every stage).  Each recorded stage adds two HIP event records to the stream,
 * and each leaves the GPU idle for some microseconds between kernels, so timed work records
 * only the stages it reports.  Bits of nonexistent stages are ignored. */
g4d_status g4d_profile_mask(g4d_ctx *ctx, uint32_t stage_mask);

/* Name of a stage index of g4d_profile ("" if out of range). */
const char *g4d_stage_name(int stage);

#ifdef __cplusplus
}
#endif
#endif /* G4D_H */
