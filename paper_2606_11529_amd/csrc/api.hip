// Host side of the C-ABI declared in include/xpr.h: argument checks, batch
// descriptors, workspace carving and kernel launches. No device memory is
// allocated here; no exception crosses the interface.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "xpr_internal.h"

namespace xpr {

hipError_t launch_project(const Batch& B, int max_n, float* splat, float* depth, int16_t* rect,
                          int32_t* tc, hipStream_t st);
hipError_t launch_project_bwd(const Batch& B, int max_n, const float* splat, const float* grad2d,
                              const int32_t* tc, const GradDev* G, int accumulate, hipStream_t st);
size_t bin_workspace_bytes(int64_t n_rec, int64_t cap, int64_t tiles, int sort_mode, bool cull);
hipError_t bin_phase1(const Batch& B, int sort_mode, bool cull, const float* splat,
                      const int16_t* rect, const float* depth, const int32_t* tc,
                      int64_t n_rec, int64_t cap, int64_t* n_isect, void* ws, hipStream_t st,
                      const uint32_t** perm_out);
hipError_t bin_phase2(const Batch& B, int sort_mode, bool cull, const float* splat,
                      int tile_bits, const float* depth, const int16_t* rect, const int32_t* tc,
                      const uint32_t* perm, int64_t n_rec,
                      int64_t cap, int64_t grid_n, const int64_t* n_isect, uint64_t* keys_out,
                      int32_t* vals, int2* ranges, int32_t* tile_order, void* ws, size_t ws_bytes,
                      hipStream_t st);
hipError_t launch_render_fwd_gut(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, float* image,
                                 float* Tfin, int32_t* ncon, int32_t* tile_work, hipStream_t st);
hipError_t launch_render_fwd_lin(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, float* image,
                                 float* Tfin, int32_t* ncon, int32_t* tile_work, hipStream_t st);
hipError_t launch_render_fwd(const Batch& B, int lds_batch, int ppt, bool persistent,
                             const float* splat, const int32_t* vals, const int32_t* ranges,
                             int32_t* order, float* image, float* Tfin, int32_t* ncon,
                             int32_t* tile_work, hipStream_t st);
hipError_t launch_render_bwd(const Batch& B, int lds_batch, int ppt, bool persistent,
                             int split_walk, int32_t* split_meta, const float* splat,
                             const int32_t* vals, const int32_t* ranges, int32_t* order,
                             const float* dimg, const float* Tfin, const int32_t* ncon,
                             float* grad2d, hipStream_t st);
hipError_t launch_render_bwd_lin(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, const float* dimg,
                                 const float* Tfin, const int32_t* ncon, float* grad,
                                 hipStream_t st);
hipError_t launch_render_bwd_gut(const Batch& B, const float* splat, const int32_t* vals,
                                 const int32_t* ranges, const int32_t* order, const float* dimg,
                                 const float* Tfin, const int32_t* ncon, float* grad,
                                 hipStream_t st);
size_t split_meta_bytes(int64_t tiles);
hipError_t fill_zero_f32(float* p, int64_t n, hipStream_t st);
hipError_t launch_l1_loss(const float* img, const float* tgt, int64_t n, float* loss,
                          float* dimg, hipStream_t st);

static thread_local char g_err[512];

const char* set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return g_err;
}

#define XPR_CHECK(cond, ...)                  \
  do {                                        \
    if (!(cond)) {                            \
      set_error(__VA_ARGS__);                 \
      return XPR_ERR_INVALID_ARG;             \
    }                                         \
  } while (0)

#define XPR_HIP(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      set_error("%s: %s", #expr, hipGetErrorString(e_));                       \
      return XPR_ERR_HIP;                                                      \
    }                                                                          \
  } while (0)

static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

struct Sizes {
  int64_t records, tiles, pixels;
  int tile_bits;
  int max_n;
};

static xpr_status check_config(const xpr_config* c) {
  XPR_CHECK(c != nullptr, "config is NULL");
  XPR_CHECK(c->tile_w == c->tile_h && (c->tile_w == 8 || c->tile_w == 16 || c->tile_w == 32),
            "tile size %dx%d not supported (8x8, 16x16 or 32x32)", c->tile_w, c->tile_h);
  XPR_CHECK(c->lds_batch == 64 || c->lds_batch == 128 || c->lds_batch == 256 || c->lds_batch == 512,
            "lds_batch %d not in {64,128,256,512}", c->lds_batch);
  XPR_CHECK(c->sh_degree >= 0 && c->sh_degree <= 3, "sh_degree %d not in 0..3", c->sh_degree);
  XPR_CHECK(std::isfinite(c->lowpass) && c->lowpass >= 0.f, "lowpass must be >= 0");
  XPR_CHECK(c->alpha_min > 0.f && c->alpha_min < 1.f, "alpha_min must be in (0,1)");
  XPR_CHECK(c->alpha_max > c->alpha_min && c->alpha_max < 1.f,
            "alpha_max must be in (alpha_min, 1)");
  XPR_CHECK(c->t_min > 0.f && c->t_min < 1.f, "t_min must be in (0,1)");
  XPR_CHECK(c->z_near > 0.f && std::isfinite(c->z_near), "z_near must be > 0");
  XPR_CHECK(c->fov_clip >= 0.f && std::isfinite(c->fov_clip), "fov_clip must be >= 0");
  XPR_CHECK(std::isfinite(c->bg[0]) && std::isfinite(c->bg[1]) && std::isfinite(c->bg[2]),
            "bg must be finite");
  XPR_CHECK(c->sort_mode == XPR_SORT_PRESORT || c->sort_mode == XPR_SORT_FULL ||
                c->sort_mode == XPR_SORT_BANDS || c->sort_mode == XPR_SORT_ONESWEEP,
            "sort_mode %d unknown", c->sort_mode);
  XPR_CHECK(c->fwd_ppt == 1 || c->fwd_ppt == 2 || c->fwd_ppt == 4, "fwd_ppt %d not in {1,2,4}",
            c->fwd_ppt);
  XPR_CHECK(c->bwd_ppt == 1 || c->bwd_ppt == 2 || c->bwd_ppt == 4, "bwd_ppt %d not in {1,2,4}",
            c->bwd_ppt);
  XPR_CHECK(c->bwd_split_walk >= 0, "bwd_split_walk < 0");
  XPR_CHECK(c->bwd_lds_batch == 0 || c->bwd_lds_batch == 64 || c->bwd_lds_batch == 128 ||
                c->bwd_lds_batch == 256 || c->bwd_lds_batch == 512,
            "bwd_lds_batch %d not in {0,64,128,256,512}", c->bwd_lds_batch);
  XPR_CHECK(c->tile_cull == 0 || c->tile_cull == 1, "tile_cull must be 0 or 1");
  XPR_CHECK(c->opacity_extents == 0 || c->opacity_extents == 1, "opacity_extents must be 0 or 1");
  XPR_CHECK(c->method == XPR_METHOD_3DGS || c->method == XPR_METHOD_3DGUT ||
                c->method == XPR_METHOD_LINPRIM,
            "method %d unknown", c->method);
  return XPR_OK;
}

// Validates the batch and fills the kernel descriptor.
static xpr_status build_batch(const xpr_views* vw, const xpr_config* c, Batch* B, Sizes* S) {
  xpr_status st = check_config(c);
  if (st != XPR_OK) return st;
  XPR_CHECK(vw != nullptr, "views is NULL");
  XPR_CHECK(vw->n_views >= 1 && vw->n_views <= XPR_MAX_VIEWS, "n_views %d not in 1..%d",
            vw->n_views, XPR_MAX_VIEWS);
  XPR_CHECK(vw->n_scenes >= 1 && vw->n_scenes <= XPR_MAX_SCENES, "n_scenes %d not in 1..%d",
            vw->n_scenes, XPR_MAX_SCENES);
  XPR_CHECK(vw->scenes && vw->cams && vw->view_scene, "views has NULL arrays");
  std::memset(B, 0, sizeof(*B));
  const int nb = (c->sh_degree + 1) * (c->sh_degree + 1);
  int max_n = 0;
  for (int s = 0; s < vw->n_scenes; ++s) {
    const xpr_scene& sc = vw->scenes[s];
    XPR_CHECK(sc.n >= 0 && sc.n < ((int64_t)1 << 31), "scene %d: n=%lld out of range", s,
              (long long)sc.n);
    XPR_CHECK(sc.ld >= sc.n && sc.ld < ((int64_t)1 << 31), "scene %d: ld < n", s);
    XPR_CHECK(sc.sh_coeffs >= nb && sc.sh_coeffs <= 16, "scene %d: sh_coeffs %d < %d", s,
              sc.sh_coeffs, nb);
    if (sc.n > 0) {
      XPR_CHECK(sc.means && sc.scales && sc.quats && sc.opacities && sc.sh,
                "scene %d: NULL parameter pointer", s);
      XPR_CHECK(aligned(sc.means, 4) && aligned(sc.scales, 4) && aligned(sc.quats, 4) &&
                    aligned(sc.opacities, 4) && aligned(sc.sh, 4),
                "scene %d: misaligned parameter pointer", s);
    }
    B->s[s] = SceneDev{sc.means, sc.scales, sc.quats, sc.opacities, sc.sh,
                       (int32_t)sc.n, (int32_t)sc.ld, sc.sh_coeffs, 0};
    max_n = std::max<int>(max_n, (int)sc.n);
  }
  int64_t rec = 0, tiles = 0, pix = 0;
  for (int v = 0; v < vw->n_views; ++v) {
    const xpr_camera& cam = vw->cams[v];
    const int sidx = vw->view_scene[v];
    XPR_CHECK(sidx >= 0 && sidx < vw->n_scenes, "view %d: scene index %d out of range", v, sidx);
    XPR_CHECK(cam.width >= 1 && cam.width <= 16384 && cam.height >= 1 && cam.height <= 16384,
              "view %d: image %dx%d out of range", v, cam.width, cam.height);
    XPR_CHECK(cam.fx > 0.f && cam.fy > 0.f && std::isfinite(cam.fx) && std::isfinite(cam.fy) &&
                  std::isfinite(cam.cx) && std::isfinite(cam.cy),
              "view %d: bad intrinsics", v);
    for (int k = 0; k < 9; ++k) XPR_CHECK(std::isfinite(cam.R[k]), "view %d: bad R", v);
    for (int k = 0; k < 3; ++k) XPR_CHECK(std::isfinite(cam.t[k]), "view %d: bad t", v);
    ViewDev& d = B->v[v];
    std::memcpy(d.R, cam.R, sizeof(d.R));
    std::memcpy(d.t, cam.t, sizeof(d.t));
    d.fx = cam.fx; d.fy = cam.fy; d.cx = cam.cx; d.cy = cam.cy;
    d.W = (int16_t)cam.width;
    d.H = (int16_t)cam.height;
    const int tx = (cam.width + c->tile_w - 1) / c->tile_w;
    const int ty = (cam.height + c->tile_h - 1) / c->tile_h;
    d.tiles_x = (int16_t)tx;
    d.tiles_y = (int16_t)ty;
    d.scene = sidx;
    d.rec_off = (int32_t)rec;
    d.tile_off = (int32_t)tiles;
    d.pix_off = (int32_t)pix;
    rec += vw->scenes[sidx].n;
    tiles += (int64_t)tx * ty;
    pix += (int64_t)cam.width * cam.height;
    XPR_CHECK(rec < ((int64_t)1 << 31) && pix < ((int64_t)1 << 30) && tiles < ((int64_t)1 << 31),
              "batch too large");
  }
  B->n_views = vw->n_views;
  B->n_scenes = vw->n_scenes;
  B->total_rec = (int32_t)rec;
  B->total_tiles = (int32_t)tiles;
  B->tile_w = c->tile_w;
  B->tile_h = c->tile_h;
  B->sh_degree = c->sh_degree;
  B->opacity_extents = c->opacity_extents;
  B->method = c->method;
  B->lowpass = c->lowpass;
  B->alpha_min = c->alpha_min;
  B->alpha_max = c->alpha_max;
  B->t_min = c->t_min;
  B->z_near = c->z_near;
  B->fov_clip = c->fov_clip;
  B->bg[0] = c->bg[0];
  B->bg[1] = c->bg[1];
  B->bg[2] = c->bg[2];
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < tiles) ++bits;
  XPR_CHECK(bits <= 31, "too many tiles");
  if (S) {
    S->records = rec;
    S->tiles = tiles;
    S->pixels = pix;
    S->tile_bits = bits;
    S->max_n = max_n;
  }
  return XPR_OK;
}

static xpr_status check_proj(const xpr_projected* p, const Sizes& S) {
  XPR_CHECK(p != nullptr, "projected is NULL");
  if (S.records > 0) {
    XPR_CHECK(p->splat && p->depth && p->rect && p->tiles_touched, "projected has NULL buffers");
    XPR_CHECK(aligned(p->splat, 16) && aligned(p->depth, 4) && aligned(p->rect, 8) &&
                  aligned(p->tiles_touched, 4),
              "projected buffers misaligned (splat 16 B, rect 8 B)");
  }
  return XPR_OK;
}

static xpr_status check_grads(const xpr_views* views, const xpr_scene_grad* grads, GradDev* G) {
  std::memset(G, 0, sizeof(GradDev) * XPR_MAX_SCENES);
  for (int s = 0; s < views->n_scenes; ++s) {
    const xpr_scene_grad& g = grads[s];
    if (views->scenes[s].n > 0) {
      XPR_CHECK(g.means && g.scales && g.quats && g.opacities && g.sh,
                "scene %d: NULL gradient buffer", s);
      XPR_CHECK(aligned(g.means, 4) && aligned(g.scales, 4) && aligned(g.quats, 4) &&
                    aligned(g.opacities, 4) && aligned(g.sh, 4),
                "scene %d: misaligned gradient buffer", s);
    }
    G[s] = GradDev{g.means, g.scales, g.quats, g.opacities, g.sh};
  }
  return XPR_OK;
}

// Floats per record of the backward's shader-data gradient: 9 for 3DGS
// (mean2D, conic, opacity, colour), 16 for 3DGUT (o', colour, ro, M) and
// LinPrim (mean2D, sigma, colour, the rows of A^-1, one zero).
static size_t grad_width(int method) { return method == XPR_METHOD_3DGS ? 9 : 16; }

// Refuses a batch whose shader-data gradients (gw floats per record) do not
// fit in cap bytes of static scratch.
static xpr_status scratch_capacity_check(int64_t records, size_t gw, size_t cap) {
  const int64_t max_records = (int64_t)(cap / (gw * sizeof(float)));
  if (records > max_records) {
    set_error("%lld records need %lld bytes of 2D gradients; the static scratch holds %lld "
              "(%lld records)",
              (long long)records, (long long)(records * (int64_t)(gw * sizeof(float))),
              (long long)(max_records * (int64_t)(gw * sizeof(float))), (long long)max_records);
    return XPR_ERR_CAPACITY;
  }
  return XPR_OK;
}

}  // namespace xpr

using namespace xpr;

extern "C" {

int32_t xpr_version(void) { return XPR_VERSION; }

const char* xpr_last_error(void) { return g_err; }

void xpr_config_default(xpr_config* c) {
  if (!c) return;
  c->tile_w = 16;
  c->tile_h = 16;
  c->lds_batch = 256;
  c->sh_degree = 3;
  c->lowpass = 0.3f;
  c->alpha_min = 1.0f / 255.0f;
  c->alpha_max = 0.99f;
  c->t_min = 1e-4f;
  c->z_near = 0.2f;
  c->fov_clip = 1.3f;
  c->bg[0] = c->bg[1] = c->bg[2] = 0.f;
  c->sort_mode = XPR_SORT_PRESORT;
  c->no_sync = 0;
  c->fwd_ppt = 2;
  c->bwd_ppt = 4;
  c->bwd_split_walk = 2048;
  c->bwd_lds_batch = 0;
  c->persistent = 0;
  c->tile_cull = 0;
  c->opacity_extents = 0;
  c->method = XPR_METHOD_3DGS;
}

xpr_status xpr_batch_sizes(const xpr_views* views, const xpr_config* cfg, xpr_sizes* out) {
  g_err[0] = 0;
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  XPR_CHECK(out != nullptr, "out is NULL");
  out->records = S.records;
  out->tiles = S.tiles;
  out->pixels = S.pixels;
  out->tile_bits = S.tile_bits;
  return XPR_OK;
}

xpr_status xpr_project(const xpr_views* views, const xpr_config* cfg, const xpr_projected* out,
                       hipStream_t stream) {
  g_err[0] = 0;
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  st = check_proj(out, S);
  if (st != XPR_OK) return st;
  XPR_HIP(launch_project(B, S.max_n, out->splat, out->depth, out->rect, out->tiles_touched, stream));
  return XPR_OK;
}

xpr_status xpr_bin_sort_workspace(const xpr_views* views, const xpr_config* cfg,
                                  int64_t isect_capacity, size_t* bytes) {
  g_err[0] = 0;
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  XPR_CHECK(bytes != nullptr, "bytes is NULL");
  XPR_CHECK(isect_capacity >= 0 && isect_capacity < ((int64_t)1 << 31),
            "isect_capacity out of range");
  *bytes = bin_workspace_bytes(S.records, isect_capacity, S.tiles, cfg->sort_mode,
                               cfg->tile_cull != 0);
  return XPR_OK;
}

xpr_status xpr_bin_sort(const xpr_views* views, const xpr_config* cfg, const xpr_projected* proj,
                        const xpr_bins* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  g_err[0] = 0;
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  st = check_proj(proj, S);
  if (st != XPR_OK) return st;
  XPR_CHECK(out != nullptr, "bins is NULL");
  const int64_t cap = out->capacity;
  XPR_CHECK(cap >= 0 && cap < ((int64_t)1 << 31), "capacity out of range");
  XPR_CHECK(out->tile_ranges && out->n_isect, "tile_ranges / n_isect NULL");
  XPR_CHECK(cap == 0 || out->vals, "vals NULL");
  XPR_CHECK(aligned(out->tile_ranges, 8) && aligned(out->n_isect, 8) &&
                (!out->keys || aligned(out->keys, 8)) && (!out->vals || aligned(out->vals, 4)) &&
                (!out->tile_order || aligned(out->tile_order, 4)),
            "misaligned output buffer");
  const bool cull = cfg->tile_cull != 0;
  const size_t need = bin_workspace_bytes(S.records, cap, S.tiles, cfg->sort_mode, cull);
  XPR_CHECK(ws_bytes >= need && (need == 0 || ws != nullptr),
            "workspace too small: %zu < %zu bytes", ws_bytes, need);
  XPR_CHECK(aligned(ws, 256), "workspace must be 256-byte aligned");
  const uint32_t* perm = nullptr;
  XPR_HIP(bin_phase1(B, cfg->sort_mode, cull, proj->splat, proj->rect, proj->depth,
                     proj->tiles_touched, S.records, cap, out->n_isect, ws, stream, &perm));
  int64_t grid_n = cap;
  if (!cfg->no_sync) {
    int64_t I = 0;
    XPR_HIP(hipMemcpyAsync(&I, out->n_isect, sizeof(I), hipMemcpyDeviceToHost, stream));
    XPR_HIP(hipStreamSynchronize(stream));
    if (I > cap) {
      set_error("%lld tile-Gaussian pairs exceed isect_capacity %lld", (long long)I,
                (long long)cap);
      return XPR_ERR_CAPACITY;
    }
    grid_n = I;
  }
  XPR_HIP(bin_phase2(B, cfg->sort_mode, cull, proj->splat, S.tile_bits, proj->depth, proj->rect,
                     proj->tiles_touched, perm, S.records, cap, grid_n, out->n_isect, out->keys,
                     out->vals, reinterpret_cast<int2*>(out->tile_ranges), out->tile_order, ws,
                     ws_bytes, stream));
  if (!cfg->no_sync && cfg->sort_mode == XPR_SORT_ONESWEEP && !cull) {
    // a look-back wait past its limit poisons the pair count
    int64_t I2 = 0;
    XPR_HIP(hipMemcpyAsync(&I2, out->n_isect, sizeof(I2), hipMemcpyDeviceToHost, stream));
    XPR_HIP(hipStreamSynchronize(stream));
    if (I2 > cap) {
      set_error("binning failed: a look-back wait of the single-pass sort hit its limit");
      return XPR_ERR_HIP;
    }
  }
  return XPR_OK;
}

xpr_status xpr_render_fwd(const xpr_views* views, const xpr_config* cfg, const xpr_projected* proj,
                          const xpr_bins* bins, float* image, float* T_final, int32_t* n_contrib,
                          int32_t* tile_work, hipStream_t stream) {
  g_err[0] = 0;
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  st = check_proj(proj, S);
  if (st != XPR_OK) return st;
  XPR_CHECK(bins && bins->tile_ranges && image && T_final && n_contrib, "NULL buffer");
  XPR_CHECK(!cfg->persistent || bins->tile_order, "persistent needs bins->tile_order");
  XPR_CHECK(aligned(bins->tile_ranges, 8) && aligned(image, 4) && aligned(T_final, 4) &&
                aligned(n_contrib, 4) && (!bins->vals || aligned(bins->vals, 4)) &&
                (!tile_work || aligned(tile_work, 4)),
            "misaligned buffer");
  if (cfg->method == XPR_METHOD_LINPRIM) {
    XPR_HIP(launch_render_fwd_lin(B, proj->splat, bins->vals, bins->tile_ranges, bins->tile_order,
                                  image, T_final, n_contrib, tile_work, stream));
    return XPR_OK;
  }
  if (cfg->method == XPR_METHOD_3DGUT) {
    XPR_HIP(launch_render_fwd_gut(B, proj->splat, bins->vals, bins->tile_ranges, bins->tile_order,
                                  image, T_final, n_contrib, tile_work, stream));
    return XPR_OK;
  }
  XPR_HIP(launch_render_fwd(B, cfg->lds_batch, cfg->fwd_ppt, cfg->persistent != 0, proj->splat,
                            bins->vals, bins->tile_ranges, bins->tile_order, image, T_final,
                            n_contrib, tile_work, stream));
  return XPR_OK;
}

xpr_status xpr_render_bwd_workspace(const xpr_views* views, const xpr_config* cfg, size_t* bytes) {
  g_err[0] = 0;
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  XPR_CHECK(bytes != nullptr, "bytes is NULL");
  *bytes = split_meta_bytes(S.tiles) + grad_width(cfg->method) * sizeof(float) *
                                           (size_t)std::max<int64_t>(S.records, 1);
  return XPR_OK;
}

}  // extern "C"

// The backward given the per-record 2D gradient buffer g2 (or NULL: then
// grad2d, else the workspace ws of ws_bytes holds it).
static xpr_status render_bwd_impl(const xpr_views* views, const xpr_config* cfg,
                                  const xpr_projected* proj, const xpr_bins* bins,
                                  const float* dL_dimage, const float* T_final,
                                  const int32_t* n_contrib, const xpr_scene_grad* grads,
                                  int32_t accumulate, float* grad2d, void* ws, size_t ws_bytes,
                                  float* g2, size_t g2_bytes, int32_t* split_meta,
                                  hipStream_t stream) {
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  st = check_proj(proj, S);
  if (st != XPR_OK) return st;
  const size_t gw = grad_width(cfg->method);
  XPR_CHECK(bins && bins->tile_ranges && dL_dimage && T_final && n_contrib, "NULL buffer");
  XPR_CHECK(grads || grad2d, "grads and grad2d both NULL");
  XPR_CHECK(!cfg->persistent || bins->tile_order, "persistent needs bins->tile_order");
  XPR_CHECK(aligned(dL_dimage, 4) && aligned(T_final, 4) && aligned(n_contrib, 4) &&
                aligned(bins->tile_ranges, 8) && (!grad2d || aligned(grad2d, 4)),
            "misaligned buffer");
  // workspace: [split metadata][2D gradients unless grad2d is given]; the
  // static scratch path passes both parts itself
  const size_t meta_bytes = split_meta_bytes(S.tiles);
  if (g2) {
    st = scratch_capacity_check(S.records, gw, g2_bytes);
    if (st != XPR_OK) return st;
  } else {
    g2 = grad2d;
    if (ws) XPR_CHECK(aligned(ws, 16), "workspace misaligned");
    if (ws && ws_bytes >= meta_bytes) split_meta = static_cast<int32_t*>(ws);
  }
  if (!g2) {
    const size_t need =
        meta_bytes + gw * sizeof(float) * (size_t)std::max<int64_t>(S.records, 1);
    XPR_CHECK(ws && ws_bytes >= need, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    g2 = reinterpret_cast<float*>(static_cast<char*>(ws) + meta_bytes);
  }
  GradDev G[XPR_MAX_SCENES];
  if (grads) {
    st = check_grads(views, grads, G);
    if (st != XPR_OK) return st;
  }
  XPR_HIP(fill_zero_f32(g2, (int64_t)gw * S.records, stream));
  if (cfg->method != XPR_METHOD_3DGS) {
    if (cfg->method == XPR_METHOD_3DGUT)
      XPR_HIP(launch_render_bwd_gut(B, proj->splat, bins->vals, bins->tile_ranges,
                                    bins->tile_order, dL_dimage, T_final, n_contrib, g2, stream));
    else
      XPR_HIP(launch_render_bwd_lin(B, proj->splat, bins->vals, bins->tile_ranges,
                                    bins->tile_order, dL_dimage, T_final, n_contrib, g2, stream));
    if (grads)
      XPR_HIP(launch_project_bwd(B, S.max_n, proj->splat, g2, proj->tiles_touched, G, accumulate ? 1 : 0,
                                 stream));
    return XPR_OK;
  }
  const int bwd_lds = cfg->bwd_lds_batch ? cfg->bwd_lds_batch : cfg->lds_batch;
  XPR_HIP(launch_render_bwd(B, bwd_lds, cfg->bwd_ppt, cfg->persistent != 0, cfg->bwd_split_walk,
                            split_meta, proj->splat, bins->vals, bins->tile_ranges,
                            bins->tile_order, dL_dimage, T_final, n_contrib, g2, stream));
  if (grads)
    XPR_HIP(launch_project_bwd(B, S.max_n, proj->splat, g2, proj->tiles_touched, G, accumulate ? 1 : 0, stream));
  return XPR_OK;
}

// File-scope scratch of xpr_render_bwd_noalloc: the per-record shader-data
// gradients (9 floats per record for 3DGS, 16 for 3DGUT and LinPrim). Each device holds its own copy for the life of the
// process. In host code ``scratch`` names a host-side stand-in, never the
// device memory: kernels and fills get the address hipGetSymbolAddress
// returns on each device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
// the first 1 MiB holds the split backward's tile data (its size for
// kScratchTiles tiles is 800,768 bytes; larger batches are walked unsplit)
constexpr size_t kScratchMetaBytes = (size_t)1 << 20;
constexpr int64_t kScratchTiles = 200000;
constexpr size_t kScratchGradBytes = kScratchBytes - kScratchMetaBytes;
static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[kMaxDevices];

// The current device's address of ``scratch`` (looked up once per device,
// with that device current).
static xpr_status scratch_of_current_device(float** out) {
  int dev = -1;
  XPR_HIP(hipGetDevice(&dev));
  XPR_CHECK(dev >= 0 && dev < kMaxDevices, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    XPR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    XPR_CHECK(p != nullptr && aligned(p, 256), "scratch symbol address invalid");
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return XPR_OK;
}

extern "C" {

xpr_status xpr_render_bwd(const xpr_views* views, const xpr_config* cfg, const xpr_projected* proj,
                          const xpr_bins* bins, const float* dL_dimage, const float* T_final,
                          const int32_t* n_contrib, const xpr_scene_grad* grads,
                          int32_t accumulate, float* grad2d, void* ws, size_t ws_bytes,
                          hipStream_t stream) {
  g_err[0] = 0;
  return render_bwd_impl(views, cfg, proj, bins, dL_dimage, T_final, n_contrib, grads,
                         accumulate, grad2d, ws, ws_bytes, nullptr, 0, nullptr, stream);
}

xpr_status xpr_render_bwd_noalloc(const xpr_views* views, const xpr_config* cfg,
                                  const xpr_projected* proj, const xpr_bins* bins,
                                  const float* dL_dimage, const float* T_final,
                                  const int32_t* n_contrib, const xpr_scene_grad* grads,
                                  int32_t accumulate, hipStream_t stream) {
  g_err[0] = 0;
  XPR_CHECK(grads != nullptr, "grads is NULL");
  // the size check needs no device: it comes before anything else
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  st = scratch_capacity_check(S.records, grad_width(cfg->method), kScratchGradBytes);
  if (st != XPR_OK) return st;
  float* base = nullptr;
  st = scratch_of_current_device(&base);
  if (st != XPR_OK) return st;
  int32_t* meta = S.tiles <= kScratchTiles ? reinterpret_cast<int32_t*>(base) : nullptr;
  float* g2 = base + kScratchMetaBytes / sizeof(float);
  return render_bwd_impl(views, cfg, proj, bins, dL_dimage, T_final, n_contrib, grads,
                         accumulate, nullptr, nullptr, 0, g2, kScratchGradBytes, meta, stream);
}

xpr_status xpr_l1_loss(const float* image, const float* target, int64_t n, float* loss,
                       float* dL_dimage, hipStream_t stream) {
  g_err[0] = 0;
  XPR_CHECK(n >= 0, "n < 0");
  XPR_CHECK(loss && aligned(loss, 4), "loss NULL or misaligned");
  XPR_CHECK(n == 0 || (image && target && dL_dimage), "image, target or dL_dimage is NULL");
  XPR_CHECK(n == 0 || (aligned(image, 4) && aligned(target, 4) && aligned(dL_dimage, 4)),
            "image, target or dL_dimage misaligned");
  XPR_HIP(launch_l1_loss(image, target, n, loss, dL_dimage, stream));
  return XPR_OK;
}

xpr_status xpr_project_bwd(const xpr_views* views, const xpr_config* cfg, const xpr_projected* proj,
                           const float* grad2d, const xpr_scene_grad* grads, int32_t accumulate,
                           hipStream_t stream) {
  g_err[0] = 0;
  Batch B;
  Sizes S;
  xpr_status st = build_batch(views, cfg, &B, &S);
  if (st != XPR_OK) return st;
  st = check_proj(proj, S);
  if (st != XPR_OK) return st;
  XPR_CHECK(grads != nullptr, "grads is NULL");
  XPR_CHECK(S.records == 0 || (grad2d && aligned(grad2d, 4)), "grad2d NULL or misaligned");
  GradDev G[XPR_MAX_SCENES];
  st = check_grads(views, grads, G);
  if (st != XPR_OK) return st;
  XPR_HIP(launch_project_bwd(B, S.max_n, proj->splat, grad2d, proj->tiles_touched, G, accumulate ? 1 : 0,
                             stream));
  return XPR_OK;
}

}  // extern "C"
