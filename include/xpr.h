/*
 * xpr.h - C-ABI of the MI355X (gfx950) tile-splatting hot path for 3D
 * Gaussians: projection, binning (count, prefix sum, duplicate, radix sort,
 * tile ranges), compositing forward and compositing + projection backward.
 *
 * The operations follow the paper "XPR: An Extensible Cross-Platform
 * Point-Based Differentiable Renderer" (arxiv 2606.11529):
 *   - Background section: the 3DGS primitive (mean, covariance R S S^T R^T,
 *     opacity, SH colour) and alpha blending c = sum_i c_i a_i T_i with
 *     T_i = prod_{j<i} (1 - a_j), ending on low transmittance;
 *   - Listing "Implementation of XPR-3DGS" (functions project and evaluate);
 *   - section "Rasterizer" (replicate by prefix sum, tile id, sort by
 *     (tile id, depth), segment bounds);
 *   - section "Shader", Algorithm 1 (per-pixel front-to-back loop over the
 *     tile's depth-sorted list in batches, exit checks at batch boundaries).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - All pointers named as device buffers are device memory of the current
 *   HIP device; every call only enqueues work on `stream` and returns.
 *   Host structs (xpr_views, xpr_config and what they point to) are read
 *   during the call only. The library never allocates device memory: the
 *   caller passes buffers, including the workspaces sized by the
 *   *_workspace queries.
 * - A batch is described by xpr_views: n_views cameras, each rendering one of
 *   n_scenes scenes (view_scene[v]). Per-view buffers are concatenated over
 *   views in view order:
 *     records  (projection outputs): view v starts at R_v = sum_{u<v} n(scene(u))
 *     tiles    (tile ranges):        view v starts at G_v = sum_{u<v} tx_u * ty_u
 *              with tx = ceil(W / tile_w), ty = ceil(H / tile_h), row-major
 *     pixels   (T_final, n_contrib): view v starts at X_v = sum_{u<v} W_u H_u,
 *              row-major [H][W]
 *     images   (image, dL/dimage):   view v starts at 3 X_v, planar [3][H][W]
 * - Errors: arguments are checked on the host before anything is enqueued
 *   (XPR_ERR_INVALID_ARG, nothing launched); a failed launch returns
 *   XPR_ERR_HIP. xpr_last_error() returns a thread-local message for the last
 *   non-OK status. No C++ exception crosses this interface.
 */
#ifndef XPR_H
#define XPR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XPR_VERSION 1
#define XPR_MAX_VIEWS 32  /* views per call */
#define XPR_MAX_SCENES 8  /* scenes per call */

typedef enum {
  XPR_OK = 0,
  XPR_ERR_INVALID_ARG = 1,
  XPR_ERR_CAPACITY = 2,   /* more tile-Gaussian pairs than isect_capacity */
  XPR_ERR_HIP = 3,
  XPR_ERR_UNSUPPORTED = 4
} xpr_status;

/* Methods (listings "Implementation of XPR-3DGS" and "...XPR-3DGUT"). */
#define XPR_METHOD_3DGS 0  /* EWA projection, 2D Gaussian evaluate; forward and backward */
#define XPR_METHOD_3DGUT 1 /* unscented-transform projection, ray evaluate; forward and
                              backward */
#define XPR_METHOD_LINPRIM 2 /* octahedra (scales = half-extents), slab chords, Beer-Lambert;
                                forward and backward */

/* Sort strategies of xpr_bin_sort; both produce the identical list. */
#define XPR_SORT_PRESORT 0 /* sort Gaussians by depth, then pairs by tile */
#define XPR_SORT_FULL 1    /* one radix sort of 64-bit (tile, depth) keys */
#define XPR_SORT_BANDS 2   /* depth presort, then records binned per band of 16 tiles and
                              placed per tile by counting (same output; falls back to
                              XPR_SORT_PRESORT beyond 65536 bands or 2^23 records) */
#define XPR_SORT_ONESWEEP 3 /* XPR_SORT_PRESORT with single-pass radix passes: digit counts
                              of every pass taken up front, each pass one kernel whose
                              blocks find their digit offsets by decoupled look-back (same
                              output; XPR_SORT_PRESORT with tile_cull or for capacities of
                              2^30 pairs or more) */

/* Pinhole camera, world -> camera x_c = R x_w + t (R row-major), camera axes
 * x right, y down, z forward. (cx, cy) is the principal point in continuous
 * pixel coordinates; pixel (i, j) is sampled at (i, j) + 0.5. The camera
 * "view" of the paper's project(p, cam, view). */
typedef struct xpr_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height; /* 1 .. 16384 */
} xpr_camera;

/* Method constants and tuning knobs. Defaults: xpr_config_default(). */
typedef struct xpr_config {
  int32_t tile_w, tile_h; /* 8x8, 16x16 or 32x32 */
  int32_t lds_batch;      /* Gaussians staged per LDS batch (forward): 64,128,256,512 */
  int32_t sh_degree;      /* 0..3 */
  float lowpass;          /* added to both diagonal entries of cov2D (0.3) */
  float alpha_min;        /* alpha_thresh of the listing (1/255) */
  float alpha_max;        /* alpha clamp (0.99) */
  float t_min;            /* stop before blending when T (1 - a) < t_min (1e-4) */
  float z_near;           /* cull when camera-space z <= z_near (> 0; 0.2) */
  float fov_clip;         /* Jacobian clamp at fov_clip * W / (2 fx) (1.3; 0 = off) */
  float bg[3];            /* background colour (0, 0, 0) */
  int32_t sort_mode;      /* XPR_SORT_PRESORT, _FULL, _BANDS or _ONESWEEP */
  int32_t no_sync;        /* 1: never read back to the host (graph capture) */
  int32_t fwd_ppt;        /* pixels per thread in the forward: 1, 2 or 4 (16x16 tiles;
                           * 8x8 tiles use 1, 32x32 tiles 4) */
  int32_t bwd_ppt;        /* pixels per thread in the backward: 1, 2 or 4 (16x16 tiles;
                           * 8x8 tiles use 1, 32x32 tiles 4) */
  int32_t bwd_lds_batch;  /* LDS batch of the backward (0: same as lds_batch) */
  int32_t persistent;     /* 1: persistent render grids pulling from tile_order */
  int32_t tile_cull;      /* 1: per-(Gaussian, tile) cull in xpr_bin_sort (0) */
  int32_t opacity_extents; /* 1: rect from the alpha >= alpha_min extents, not 3 sigma (0) */
  int32_t method;         /* XPR_METHOD_3DGS (0), XPR_METHOD_3DGUT or XPR_METHOD_LINPRIM */
  int32_t bwd_split_walk; /* 16x16 tiles, bwd_ppt 4, not persistent: a tile whose walk (its
                           * largest n_contrib) reaches this is walked backward as four
                           * 16x4 bands by four workgroups, one pixel per lane (at most 64
                           * tiles per call); 0 = never (default 2048) */
} xpr_config;

/* One scene of n Gaussians, structure of arrays with leading dimension ld:
 *   means [3][ld], scales [3][ld] (activated, > 0), quats [4][ld] (w,x,y,z,
 *   any non-zero norm, normalised inside), opacities [ld] (activated, in
 *   (0,1)), sh [sh_coeffs][3][ld] (coefficient-major, RGB inner), with
 *   sh_coeffs >= (sh_degree+1)^2. Device memory, read only. The paper's
 *   PrimitiveParams (mu, s, q, sh, o). */
typedef struct xpr_scene {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacities;
  const float* sh;
  int64_t n;  /* 0 .. 2^31-1 */
  int64_t ld; /* >= n */
  int32_t sh_coeffs;
} xpr_scene;

/* Gradient buffers of one scene, same layout (ld, sh_coeffs) as xpr_scene;
 * gradients are with respect to the activated scales and opacities and the
 * raw (unnormalised) quaternion. */
typedef struct xpr_scene_grad {
  float* means;
  float* scales;
  float* quats;
  float* opacities;
  float* sh;
} xpr_scene_grad;

typedef struct xpr_views {
  const xpr_scene* scenes;   /* host array [n_scenes] */
  int32_t n_scenes;          /* 1 .. XPR_MAX_SCENES */
  const xpr_camera* cams;    /* host array [n_views] */
  const int32_t* view_scene; /* host array [n_views], values < n_scenes */
  int32_t n_views;           /* 1 .. XPR_MAX_VIEWS */
} xpr_views;

/* Per-record projection outputs (device buffers, concatenated over views,
 * one record per (view, Gaussian)). The paper's ProjectResult:
 *   splat [total][12] float: u, v, A, B | C, o, r, g | b, 0, 0, 0 where
 *         (u, v) is mean2D and A = -0.5 con00, B = -con01, C = -0.5 con11
 *         the scaled conic (the listing's shader data), (r, g, b) the colour;
 *         with XPR_METHOD_3DGUT [total][24] float: the same 9 values (o the
 *         adjusted opacity o', (u, v) = UT mean2D - 1/2 and the conic of the
 *         UT covariance: the listing's tile cull data), then ro (3), the
 *         camera position in the Gaussian's canonical frame, M = S^-1 R^T
 *         (9, row-major) (the listing's shader data), then two words whose
 *         bit patterns hold int16 pairs X0 | X1 << 16 and Y0 | Y1 << 16, the
 *         pixel columns and rows that can hold the record's contributions
 *         (a bound the compositing uses for its per-wave record lists, not
 *         part of the paper's record), and a zero;
 *         with XPR_METHOD_LINPRIM [total][20] float: u, v (mu_2D - 1/2),
 *         sigma, r | g, b, ex, ey | c0 (3), c1 (3), c2 (3), 3 zeros with
 *         c_k the rows of A^-1 (the listing's shader data)
 *   depth [total] float: camera-space z
 *   rect  [total][4] int16: tile-space box x0, y0, x1, y1 (half-open)
 *   tiles_touched [total] int32: (x1-x0)(y1-y0) if visible else 0 */
typedef struct xpr_projected {
  float* splat;
  float* depth;
  int16_t* rect;
  int32_t* tiles_touched;
} xpr_projected;

/* Sizes of a batch: records, tiles and pixels over all views. */
typedef struct xpr_sizes {
  int64_t records, tiles, pixels;
  int32_t tile_bits; /* bits needed for a global tile id */
} xpr_sizes;

/* Fills *cfg with the defaults listed in xpr_config. */
void xpr_config_default(xpr_config* cfg);

/* Sizes of the concatenated buffers of a batch (host only). */
xpr_status xpr_batch_sizes(const xpr_views* views, const xpr_config* cfg, xpr_sizes* out);

/* Projection (listing XPR-3DGS, project), one record per (view, Gaussian):
 * world->camera; 3D covariance from the normalised quaternion and scales;
 * EWA 2D covariance J W Sigma W^T J^T + lowpass I with J the perspective
 * Jacobian at the clamped direction; conic = inverse; mean2D = f X/Z + c - 1/2;
 * radius ceil(3 sqrt(lambda_max)); tile rect [floor((u-r)/tw),
 * floor((u+r)/tw)+1) clamped to the grid (likewise v); visibility
 * det > 0, o >= alpha_min, r > 0, area > 0, z > z_near. With
 * cfg->opacity_extents = 1 the extents are opacity-aware (compute_extents of
 * the listing takes the opacity): the half-widths of the ellipse where
 * o G = alpha_min, ex = sqrt(2 ln(o / alpha_min) cov_xx) and
 * ey = sqrt(2 ln(o / alpha_min) cov_yy) (cov with the low-pass), the rect is
 * [floor((u-ex)/tw), floor((u+ex)/tw)+1) x [floor((v-ey)/th),
 * floor((v+ey)/th)+1) and r = max(ex, ey); every pixel whose alpha can pass
 * the alpha_min gate then lies in the rect.
 * With cfg->method = XPR_METHOD_3DGUT (listing XPR-3DGUT, project): the
 * unscented transform of n = 3 with alpha = 1, beta = 2, kappa = 0 (sigma
 * points mu and mu +- sqrt(3) s_j R e_j; mean weights 0 and 1/6, covariance
 * weights 2 and 1/6) through the pinhole projection; invisible when a sigma
 * point has z <= z_near; cov2D + lowpass I; o' = o sqrt(det_orig / det);
 * rect as above around (u, v) = mean2D - 1/2; visibility also needs
 * o' > alpha_min; ro and M as in the record layout above.
 * With cfg->method = XPR_METHOD_LINPRIM (listing XPR-LinPrim, project; the
 * scene's scales are the octahedra's half-extents): A = J3 R_w2c R diag(s)
 * with J3 the perspective Jacobian rows over mu_c / |mu_c|; c_k the rows of
 * A^-1; ex = max_k |A_0k|, ey = max_k |A_1k|; rect around (u, v) = mu_2D -
 * 1/2 from (ex, ey) with the rounding above; depth = |mu_c|;
 * sigma = -log(1 - 0.99 o) / (2 s_min), o clipped to [0, 0.999]; visible
 * when z > z_near, A is invertible, s_min > 0 and the rect is not empty.
 * Colour
 * max(0, 0.5 + sum_lm sh_lm Y_lm(dir)) with the real SH basis (Condon-Shortley
 * phase) and dir = (mu - campos) / |mu - campos|. Writes every field of
 * *out for all records (invisible: tiles_touched = 0). */
xpr_status xpr_project(const xpr_views* views, const xpr_config* cfg, const xpr_projected* out,
                       hipStream_t stream);

/* Pair lists and tile ranges produced by xpr_bin_sort (device buffers).
 *   keys  [capacity] uint64 (may be NULL): tile << 32 | float bits of depth
 *   vals  [capacity] int32: record index of each sorted pair
 *   tile_ranges [tiles][2] int32: [start, end) per global tile, (0,0) if empty
 *   n_isect  int64: total number of pairs I (written also when I > capacity)
 *   tile_order [tiles + 1] int32 (may be NULL): the tiles by decreasing list
 *   length (ties by tile id), the order in which the render calls schedule
 *   them; the last entry is queue state the render calls reset and use.
 *   capacity  length of keys and vals (<= 2^31 - 1) */
typedef struct xpr_bins {
  uint64_t* keys;
  int32_t* vals;
  int32_t* tile_ranges;
  int64_t* n_isect;
  int32_t* tile_order;
  int64_t capacity;
} xpr_bins;

/* Workspace bytes xpr_bin_sort needs for this batch and capacity. */
xpr_status xpr_bin_sort_workspace(const xpr_views* views, const xpr_config* cfg,
                                  int64_t isect_capacity, size_t* bytes);

/* Binning (section Rasterizer): exclusive prefix sum of tiles_touched, one
 * pair per (record, tile of its rect) with tile id G_v + y tx + x enumerated
 * row-major in the rect, stable sort by (tile id, depth) so that ties keep
 * the lower record index, per-tile [start, end), and (if requested) the
 * longest-list-first tile order.
 * With cfg->tile_cull = 1 a pair is kept only if it passes tile_cull of the
 * listing XPR-3DGS: the smallest power 0.5 d^T conic d over the tile's
 * pixel-sample box [x tw, x tw + tw - 1] x [y th, y th + th - 1] (clipped
 * to the image) is at most log(o / alpha_min), evaluated in float64 from the
 * float32 splat (a conic that is not positive definite keeps its rect). The
 * lists, ranges and *n_isect then hold the kept pairs only (the listing's
 * sentinel tile for culled pairs is never materialised), the image is the
 * same up to alpha values at the 1/255 threshold, and the presort strategy
 * is used whatever cfg->sort_mode says. For XPR_METHOD_3DGUT the tile box
 * is first extended by one pixel in x and y (tile_max += 1 of its
 * tile_cull). For XPR_METHOD_LINPRIM the test is the tile_cull of the
 * listing XPR-LinPrim: with the slab data (h_i = 1 / |n_iz|, m_i the slab
 * midpoint in tau at a pixel) the longest chord over the same pixel-sample
 * box is bounded by max(0, min over ordered slab pairs (i, j) of
 * [max over the box corners of (m_i - m_j) + h_i + h_j]) (slabs with
 * |n_iz| < 1e-10 dropped), and the pair is kept iff sigma times that bound
 * is at least -log(1 - alpha_min).
 *   out     buffers as described at xpr_bins
 *   ws / ws_bytes   workspace of at least xpr_bin_sort_workspace() bytes
 * With cfg->no_sync == 0 the call reads I back (one stream sync) and returns
 * XPR_ERR_CAPACITY when I > capacity (outputs then undefined, *n_isect
 * valid). With no_sync == 1 nothing is read back and grids are sized from
 * the capacity; if I > capacity the lists are undefined and the caller checks
 * *n_isect after the stream completes. */
xpr_status xpr_bin_sort(const xpr_views* views, const xpr_config* cfg, const xpr_projected* proj,
                        const xpr_bins* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* Forward compositing (Algorithm 1 with the 3DGS evaluate): for each pixel
 * (x, y), over its tile's list front to back, P = A dx^2 + B dx dy + C dy^2
 * (dx = x - u, dy = y - v); skip if P > 0; a = min(alpha_max, o e^P); skip
 * if a < alpha_min; stop without blending if T (1 - a) < t_min; else
 * C += c a T, T *= 1 - a. Reads bins->vals, tile_ranges and (if not NULL)
 * tile_order. Writes
 *   image [3][H][W] per view: C + T bg
 *   T_final [H][W] per view: final transmittance
 *   n_contrib [H][W] per view: 1-based list position of the last blended
 *   entry (0 if none), used by the backward;
 *   tile_work [tiles][2] int32 (may be NULL): the work the definition
 *   performs in each tile, summed over its pixels: the list entries a pixel
 *   evaluates (up to and including the one that stops it, else the whole
 *   list), then the entries it blends. Given, the call runs a counting
 *   instantiation in index order (tile_order, persistent and the
 *   lds_batch / fwd_ppt knobs are then ignored; the outputs are the same).
 * Tiles are scheduled in tile_order when given; with cfg->persistent a grid
 * sized to fill the device pulls tiles from that order through an atomic
 * counter (then tile_order is required).
 * XPR_METHOD_3DGUT (pixel_info and evaluate of listing XPR-3DGUT): per pixel
 * the world ray direction through (x + 1/2, y + 1/2); per entry the largest
 * response exp(-d^2 / 2) of the Gaussian along that ray, d^2 the squared
 * canonical distance at tau_max; skipped unless the response > 0.0113; then
 * alpha = min(alpha_max, o' response) with the gates, stop rule and
 * blending above. Evaluated with d^2 in float64. cfg->lds_batch, fwd_ppt
 * and persistent do not apply (256 / 64 / 1024 threads per 16x16 / 8x8 /
 * 32x32 tile).
 * XPR_METHOD_LINPRIM (evaluate of listing XPR-LinPrim): the chord of the
 * ray through (x + 1/2, y + 1/2) inside the slabs |n_i . (dx, dy, tau)|
 * <= 1, n_i = c0 +- c1 +- c2, alpha = 1 - exp(-sigma chord) for a
 * positive chord, then the gates, stop rule and blending above (chord in
 * float64; same launch shape as 3DGUT). */
xpr_status xpr_render_fwd(const xpr_views* views, const xpr_config* cfg, const xpr_projected* proj,
                          const xpr_bins* bins, float* image, float* T_final, int32_t* n_contrib,
                          int32_t* tile_work, hipStream_t stream);

/* Workspace bytes xpr_render_bwd needs: the tile data of the split backward
 * (bwd_split_walk; 4 bytes per tile plus 512) followed by the per-record
 * shader-data gradients (36 bytes per record for XPR_METHOD_3DGS, 64 for
 * XPR_METHOD_3DGUT and XPR_METHOD_LINPRIM; used when grad2d is NULL). */
xpr_status xpr_render_bwd_workspace(const xpr_views* views, const xpr_config* cfg, size_t* bytes);

/* Backward of compositing and projection: the derivative of the blending
 * sum of the Background section, c(x, y) = sum_i c_i a_i T_i with
 * T_i = prod_{j<i} (1 - a_j), through evaluate and project of the listing
 * "Implementation of XPR-3DGS". The paper obtains this derivative by
 * automatic differentiation of its four interface functions (section Key
 * Interfaces: gradients flow through project, tile_cull, pixel_info and
 * evaluate); here it is written out, with the gates, the stop rule and the
 * rect rounding piecewise constant (zero derivative) and the clamps
 * (alpha <= alpha_max, colour >= 0, the Jacobian clamp) differentiated on
 * the side they take, which is what automatic differentiation of the
 * forward gives.
 * Given dL/dimage (laid out like
 * image) and the forward's T_final and n_contrib, accumulates the gradient of
 * L with respect to every scene's parameters, summed over the views that
 * render it:
 *   grads [n_scenes] host array of device gradient buffers, or NULL to stop
 *   after the compositing backward (then grad2d is required);
 *   accumulate 0: overwrite, 1: add to the existing contents;
 *   grad2d float (may be NULL): receives the derivative with respect to the
 *   shader data per record, [records][9] dL/d(u, v, A, B, C, o, r, g, b)
 *   for XPR_METHOD_3DGS, [records][16] dL/d(o', r, g, b, ro (3), M (9,
 *   row-major)) for XPR_METHOD_3DGUT (the values its evaluate reads, M's
 *   derivative taken with the Gaussian's centre fixed; the 2D mean and
 *   conic only place the rect), [records][16] dL/d(u, v, sigma, r, g, b,
 *   c0 (3), c1 (3), c2 (3)) and a zero for XPR_METHOD_LINPRIM (ex, ey only
 *   place the rect); when NULL the workspace holds it.
 * The compositing backward walks each pixel's list in reverse from its last
 * blended entry (T_i recovered as T_{i+1} / (1 - a_i)); tiles are scheduled
 * as in xpr_render_fwd. Gradient sums use float atomics, so the last bits
 * vary from run to run. For XPR_METHOD_3DGUT the same derivative is taken
 * through evaluate and project of the listing "Implementation of XPR-3DGUT"
 * (the response along the ray, the unscented transform's 2D covariance in
 * the Mip-Splatting opacity factor, ro and M = S^-1 R^T); cfg->lds_batch,
 * bwd_ppt, persistent and bwd_split_walk do not apply to it (one thread per
 * pixel). For XPR_METHOD_LINPRIM the derivative of evaluate and project of
 * the listing "Implementation of XPR-LinPrim": the Beer-Lambert alpha, the
 * chord through its entry and exit slabs, sigma, and A^-1 =
 * (J3 R_w2c R diag(s))^-1 (same launch shape as 3DGUT). */
xpr_status xpr_render_bwd(const xpr_views* views, const xpr_config* cfg, const xpr_projected* proj,
                          const xpr_bins* bins, const float* dL_dimage, const float* T_final,
                          const int32_t* n_contrib, const xpr_scene_grad* grads,
                          int32_t accumulate, float* grad2d, void* ws, size_t ws_bytes,
                          hipStream_t stream);

/* xpr_render_bwd for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation with grads required and grad2d / the workspace
 * replaced by a file-scope static device array of 64 MiB per device (1 MiB
 * of split-backward tile data, used for batches of up to 200,000 tiles,
 * then the per-record shader-data gradients, 36 bytes per record for
 * XPR_METHOD_3DGS, at most 1,835,008 records, 64 for XPR_METHOD_3DGUT and
 * XPR_METHOD_LINPRIM, at most 1,032,192; more fail with XPR_ERR_CAPACITY before anything is
 * enqueued). Calls no
 * hipMalloc, hipFree or other allocating routine; the caller still owns
 * every input and the gradient buffers. Every call on a device shares that
 * device's array, which is zero-filled at the start of each call by a
 * kernel on the given stream: calls that overlap on one device (different
 * streams, or threads) race on it and must be serialised by the caller.
 * The array's address is looked up once per device on its first call. */
xpr_status xpr_render_bwd_noalloc(const xpr_views* views, const xpr_config* cfg,
                                  const xpr_projected* proj, const xpr_bins* bins,
                                  const float* dL_dimage, const float* T_final,
                                  const int32_t* n_contrib, const xpr_scene_grad* grads,
                                  int32_t accumulate, hipStream_t stream);

/* Backward of the projection alone (the derivative of project of the listing
 * "Implementation of XPR-3DGS" -- world to camera, R(q) S^2 R(q)^T, the EWA
 * covariance with its low-pass, the conic, mean2D and the SH colour of the
 * Background section -- obtained in the paper by automatic differentiation,
 * section Key Interfaces): from grad2d [records][9] (as written by
 * xpr_render_bwd) to the parameter gradients of every scene, summed over the
 * views that render it (one thread per Gaussian loops over those views, so
 * the sum is deterministic). Records with tiles_touched == 0 contribute
 * nothing. grads and accumulate as in xpr_render_bwd. For XPR_METHOD_3DGUT
 * grad2d is [records][16] and the derivative is that of the listing
 * "Implementation of XPR-3DGUT", project: ro = M (campos - mu),
 * M = S^-1 R(q)^T, the opacity factor sqrt(det_orig / det) through the
 * seven projected sigma points, and the SH colour. For XPR_METHOD_LINPRIM
 * (grad2d [records][16]) that of its project: mean2D, sigma through the
 * clipped opacity and the smallest scale, A^-1 through J3, R_w2c, R(q) and
 * the scales, and the SH colour. */
xpr_status xpr_project_bwd(const xpr_views* views, const xpr_config* cfg, const xpr_projected* proj,
                           const float* grad2d, const xpr_scene_grad* grads, int32_t accumulate,
                           hipStream_t stream);

/* The training loss of the benchmarked step (the L1 photometric term of the
 * 3DGS objective, Background section): over n colour values (3HW for one
 * view, image and target laid out alike),
 *   *loss = (1/n) sum |image - target|,
 *   dL_dimage = sign(image - target) / n   (sign(0) = 0),
 * ready to pass to xpr_render_bwd. loss is one device float (overwritten);
 * all pointers are device memory, 4-byte aligned (16-byte alignment of all
 * three arrays takes a vector path). The sum uses float atomics across
 * workgroups, so its last bits vary from run to run; dL_dimage is exact. */
xpr_status xpr_l1_loss(const float* image, const float* target, int64_t n, float* loss,
                       float* dL_dimage, hipStream_t stream);

/* Message of the last non-OK status on this thread ("" if none). */
const char* xpr_last_error(void);

/* XPR_VERSION of the library. */
int32_t xpr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XPR_H */
