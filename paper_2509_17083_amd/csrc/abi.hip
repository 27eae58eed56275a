// C ABI of the HyRF render step: host-side validation, workspace carving
// and kernel launches.  No allocation, no global state except the
// thread-local error string.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>

#include "backward.h"
#include "bin.h"
#include "block.h"
#include "composite.h"
#include "kernels.h"
#include "project.h"
#include "query.h"

namespace {
// Points one decoder-adjoint workgroup stages per round: 4 waves of 16
// Gaussians, 8 waves of 16 background pixels.
constexpr int64_t BWD_PPR_GAUSS = 64, BWD_PPR_BG = 128;
}

using namespace hyrf;

namespace {

thread_local std::string g_err;

hyrf_status fail(hyrf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

hyrf_status launch_error(hipError_t e) {
  return fail(HYRF_ERR_LAUNCH, "kernel launch failed: %s", hipGetErrorString(e));
}

#define REQ(cond, ...)                                                  \
  do {                                                                  \
    if (!(cond)) return fail(HYRF_ERR_INVALID_ARGUMENT, __VA_ARGS__);   \
  } while (0)

hyrf_status check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return launch_error(e);
  g_err.clear();
  return HYRF_OK;
}

hyrf_status check_cams(const hyrf_camera* cams, int V) {
  REQ(cams, "cams is NULL");
  REQ(V >= 1 && V <= HYRF_MAX_VIEWS, "n_views = %d outside [1, %d]", V, HYRF_MAX_VIEWS);
  for (int v = 0; v < V; ++v) {
    const hyrf_camera& c = cams[v];
    REQ(c.width > 0 && c.height > 0, "camera %d: width/height must be positive", v);
    REQ(c.width == cams[0].width && c.height == cams[0].height, "camera %d: all views must share width and height", v);
    REQ((int64_t)c.width * c.height * V < (int64_t)1 << 31, "image too large");
    REQ(c.fx > 0.f && c.fy > 0.f, "camera %d: focal lengths must be positive", v);
    REQ(c.z_near > 0.f, "camera %d: z_near must be positive", v);
    REQ(c.cull_tol >= 0.f, "camera %d: cull_tol must be >= 0", v);
  }
  return HYRF_OK;
}

Cams make_cams(const hyrf_camera* cams, int V) {
  Cams c{};
  for (int v = 0; v < V; ++v) c.c[v] = to_camp(cams[v]);
  c.V = V;
  return c;
}

hyrf_status check_gauss(const hyrf_gaussians* g) {
  REQ(g, "gaussians is NULL");
  REQ(g->n >= 0, "gaussian count must be >= 0");
  if (g->n > 0) REQ(g->pos && g->scale_e && g->opac_e && g->col_e, "a gaussian array is NULL");
  REQ(g->pos_dtype == HYRF_F32 || g->pos_dtype == HYRF_F16, "pos_dtype = %d must be HYRF_F32 or HYRF_F16",
      g->pos_dtype);
  return HYRF_OK;
}

hyrf_status check_fields(const hyrf_fields* f) {
  REQ(f, "fields is NULL");
  REQ(f->levels == 4 || f->levels == 8 || f->levels == 12 || f->levels == 16, "levels = %d must be 4, 8, 12 or 16", f->levels);
  REQ(f->features == 2, "features per entry must be 2");
  REQ((f->single_field || (f->log2_T_geo >= 10 && f->log2_T_geo <= 24)) && f->log2_T_rad >= 10 &&
          f->log2_T_rad <= 24,
      "log2 table sizes must be in [10, 24]");
  REQ(f->base_res >= 2.f && f->growth >= 1.f, "base_res must be >= 2 and growth >= 1");
  REQ((f->single_field || f->table_geo) && f->table_rad && f->mlp_geo && f->mlp_col, "a field array is NULL");
  REQ(f->hidden == 16 || f->hidden == 32 || f->hidden == 48 || f->hidden == 64, "hidden width must be 16, 32, 48 or 64");
  REQ(f->n_hidden == 1 || f->n_hidden == 2, "n_hidden must be 1 or 2");
  REQ(f->bg_radius > 0.f, "bg_radius must be positive");
  for (int d = 0; d < 3; ++d) REQ(f->aabb_inv_half[d] > 0.f, "aabb_inv_half must be positive");
  REQ(f->scatter_merge >= 0 && f->scatter_merge <= 2, "scatter_merge = %d must be 0, 1 or 2", f->scatter_merge);
  if (!(f->table_dtype == HYRF_F32 || f->table_dtype == HYRF_F16 || f->table_dtype == HYRF_U8))
    return fail(HYRF_ERR_UNSUPPORTED, "table dtype %d not supported (F32, F16 or U8)", f->table_dtype);
  REQ(f->table_dtype != HYRF_U8 || ((f->single_field || f->qparams_geo) && f->qparams_rad),
      "8-bit tables need qparams_geo and qparams_rad");
  if (!(f->mlp_dtype == HYRF_F32 || f->mlp_dtype == HYRF_BF16))
    return fail(HYRF_ERR_UNSUPPORTED, "mlp dtype %d not supported (F32 or BF16)", f->mlp_dtype);
  if (!shape_supported(f->levels, f->hidden, f->n_hidden))
    return fail(HYRF_ERR_UNSUPPORTED, "no kernel for levels=%d hidden=%d n_hidden=%d "
                "(built: 16/64/2, 16/64/1, 8/32/1, 8/64/2)", f->levels, f->hidden, f->n_hidden);
  if (!precision_supported(f->levels, f->hidden, f->n_hidden, f->table_dtype, f->mlp_dtype == HYRF_BF16))
    return fail(HYRF_ERR_UNSUPPORTED, "float16 tables and bfloat16 decoders are built for levels=16 "
                "hidden=64 n_hidden=2 only");
  return HYRF_OK;
}

// The geometry field's table: the radiance table in the single-field model.
const void* geo_table(const hyrf_fields* f) { return f->single_field ? f->table_rad : f->table_geo; }

GridP make_grid(const hyrf_fields* f) {
  GridP g{};
  const int log2_T_geo = f->single_field ? f->log2_T_rad : f->log2_T_geo;
  g.single = f->single_field ? 1 : 0;
  g.L = f->levels;
  g.log2_T_geo = log2_T_geo;
  g.log2_T_rad = f->log2_T_rad;
  g.mask_geo = (1u << log2_T_geo) - 1u;
  g.mask_rad = (1u << f->log2_T_rad) - 1u;
  double s = (double)f->base_res;
  for (int l = 0; l < f->levels; ++l) {
    int res = (int)floor(s);
    g.res[l] = res;
    double side = (double)res + 1.0;
    if (side * side * side <= (double)(1u << log2_T_geo)) g.dense_geo |= 1u << l;
    if (side * side * side <= (double)(1u << f->log2_T_rad)) g.dense_rad |= 1u << l;
    s = s * (double)f->growth;
  }
  for (int d = 0; d < 3; ++d) {
    g.center[d] = f->aabb_center[d];
    g.inv_half[d] = f->aabb_inv_half[d];
  }
  g.bg_radius = f->bg_radius;
  g.tau_T = f->tau_T;
  g.qp_geo = f->table_dtype == HYRF_U8 ? (f->single_field ? f->qparams_rad : f->qparams_geo) : nullptr;
  g.qp_rad = f->table_dtype == HYRF_U8 ? f->qparams_rad : nullptr;
  return g;
}

size_t query_ws(int n, uint32_t** flag, uint32_t** pos, uint32_t** temp, void* base) {
  Carve c(base);
  uint32_t* a = c.take<uint32_t>(n > 0 ? n : 1);
  uint32_t* b = c.take<uint32_t>(n > 0 ? n : 1);
  uint32_t* t = c.take<uint32_t>(scan_temp_elems(n));
  if (flag) *flag = a;
  if (pos) *pos = b;
  if (temp) *temp = t;
  return c.off;
}

hyrf_status check_query(const hyrf_fields* fields, const hyrf_gaussians* g, const hyrf_camera* cams,
                        int32_t n_views, const hyrf_query_out* out) {
  hyrf_status s;
  if ((s = check_fields(fields)) != HYRF_OK) return s;
  if ((s = check_gauss(g)) != HYRF_OK) return s;
  if ((s = check_cams(cams, n_views)) != HYRF_OK) return s;
  REQ(out && out->vis_count && out->vis_idx, "query output: vis_count / vis_idx is NULL");
  REQ(g->n == 0 || (out->opacity && out->scale && out->quat && out->rgb), "query output: a property array is NULL");
  REQ((out->feat_geo == nullptr) == (out->feat_rad == nullptr), "feat_geo and feat_rad must both be set or both NULL");
  return HYRF_OK;
}

// Pre-cull, compaction and field query of validated arguments; `ws` holds
// query_ws(g->n) bytes (cull flags, their exclusive scan, scan partials).
void launch_query_all(const hyrf_fields* fields, const hyrf_gaussians* g, const hyrf_camera* cams,
                      int32_t n_views, const hyrf_query_out* out, void* ws, hipStream_t st) {
  uint32_t *flag, *pos, *temp;
  query_ws(g->n, &flag, &pos, &temp, ws);
  const Cams cc = make_cams(cams, n_views);
  launch_cull(g->pos, g->pos_dtype == HYRF_F16, g->n, cc, flag, pos, temp, out->vis_idx, out->vis_count, st);
  if (g->n > 0) {
    QueryArgs a{};
    a.grid = make_grid(fields);
    a.cams = cc;
    a.table_geo = geo_table(fields);
    a.table_rad = fields->table_rad;
    a.w_geo = fields->mlp_geo;
    a.w_col = fields->mlp_col;
    a.n = g->n;
    a.count = out->vis_count;
    a.vis_idx = out->vis_idx;
    a.pos = g->pos;
    a.pos_f16 = g->pos_dtype == HYRF_F16;
    a.scale_e = g->scale_e;
    a.rot_e = g->rot_e;
    a.opac_e = g->opac_e;
    a.col_e = g->col_e;
    a.opacity = out->opacity;
    a.scale = out->scale;
    a.quat = out->quat;
    a.rgb = out->rgb;
    a.feat_geo = out->feat_geo;
    a.feat_rad = out->feat_rad;
    a.dbg = out->dbg_index;
    a.jac = out->feat_jac;
    launch_query(fields->levels, fields->hidden, fields->n_hidden, fields->table_dtype,
                 fields->mlp_dtype == HYRF_BF16, a, g->n, st);
  }
}

}  // namespace

extern "C" {

const char* hyrf_last_error(void) { return g_err.c_str(); }
const char* hyrf_version(void) { return "hyrf-gfx950 0.1"; }

size_t hyrf_query_workspace_bytes(int32_t n) { return query_ws(n, nullptr, nullptr, nullptr, nullptr); }

hyrf_status hyrf_query_fields(const hyrf_fields* fields, const hyrf_gaussians* g,
                              const hyrf_camera* cams, int32_t n_views, const hyrf_query_out* out,
                              void* ws, size_t ws_bytes, void* stream) {
  hyrf_status s;
  if ((s = check_query(fields, g, cams, n_views, out)) != HYRF_OK) return s;
  const size_t need = hyrf_query_workspace_bytes(g->n);
  REQ(ws && ws_bytes >= need, "query workspace too small: %zu < %zu bytes", ws_bytes, need);
  launch_query_all(fields, g, cams, n_views, out, ws, (hipStream_t)stream);
  return check_launch();
}

hyrf_status hyrf_project(const hyrf_gaussians* g, const hyrf_query_out* q, const hyrf_camera* cams,
                         int32_t n_views, const hyrf_splats* sp, void* stream) {
  hyrf_status s;
  if ((s = check_gauss(g)) != HYRF_OK) return s;
  if ((s = check_cams(cams, n_views)) != HYRF_OK) return s;
  REQ(q && q->vis_count && q->vis_idx && q->opacity && q->scale && q->quat && q->rgb, "query output incomplete");
  REQ(sp && sp->rec && sp->rect && sp->depth && sp->total, "splats: an array is NULL");
  REQ(sp->n_max >= g->n, "splats.n_max (%d) must be >= the gaussian count (%d)", sp->n_max, g->n);
  REQ(((uintptr_t)sp->rec & 15) == 0 && ((uintptr_t)sp->rect & 15) == 0, "splats.rec / rect must be 16-byte aligned");
  ProjArgs a{};
  a.cams = make_cams(cams, n_views);
  a.n = g->n;
  a.n_max = sp->n_max;
  a.tiles_x = (cams[0].width + TILE - 1) / TILE;
  a.tiles_y = (cams[0].height + TILE - 1) / TILE;
  a.count = q->vis_count;
  a.vis_idx = q->vis_idx;
  a.pos = g->pos;
  a.pos_f16 = g->pos_dtype == HYRF_F16;
  a.opacity = q->opacity;
  a.scale = q->scale;
  a.quat = q->quat;
  a.rgb = q->rgb;
  a.rec = sp->rec;
  a.rect = sp->rect;
  a.depth = sp->depth;
  a.total = sp->total;
  launch_project(a, g->n, n_views, (hipStream_t)stream);
  return check_launch();
}

size_t hyrf_bin_sort_workspace_bytes(int32_t n_views, int32_t n_max, int64_t capacity, int32_t width,
                                     int32_t height) {
  const int tiles = ((width + TILE - 1) / TILE) * ((height + TILE - 1) / TILE);
  return carve_bin_ws(nullptr, n_views, n_max, capacity, tiles * n_views).bytes;
}

hyrf_status hyrf_bin_sort(const hyrf_splats* sp, const hyrf_camera* cams, int32_t n_views,
                          int64_t n_entries, int64_t capacity, uint32_t* keys, uint32_t* vals,
                          uint32_t* tile_ranges, void* ws, size_t ws_bytes, void* stream) {
  hyrf_status s;
  if ((s = check_cams(cams, n_views)) != HYRF_OK) return s;
  REQ(sp && sp->count && sp->rect && sp->depth, "splats: count / rect / depth is NULL");
  REQ(sp->n_max >= 0, "splats.n_max must be >= 0");
  REQ(((uintptr_t)sp->rect & 15) == 0, "splats.rect must be 16-byte aligned");
  REQ(vals && tile_ranges, "vals / tile_ranges is NULL");
  REQ(n_entries >= 0 && capacity >= 0, "n_entries / capacity must be >= 0");
  REQ((int64_t)n_views * sp->n_max < ((int64_t)1 << 31), "too many splats");
  if (n_entries > capacity)
    return fail(HYRF_ERR_CAPACITY, "tile entries %lld exceed capacity %lld", (long long)n_entries, (long long)capacity);
  if (n_entries >= ((int64_t)1 << 31)) return fail(HYRF_ERR_CAPACITY, "more than 2^31 - 1 tile entries");
  const int tx = (cams[0].width + TILE - 1) / TILE, ty = (cams[0].height + TILE - 1) / TILE;
  const size_t need = hyrf_bin_sort_workspace_bytes(n_views, sp->n_max, capacity, cams[0].width, cams[0].height);
  REQ(ws && ws_bytes >= need, "bin_sort workspace too small: %zu < %zu bytes", ws_bytes, need);
  BinWs w = carve_bin_ws(ws, n_views, sp->n_max, capacity, tx * ty * n_views);
  BinArgs a{};
  a.V = n_views;
  a.n_max = sp->n_max;
  a.tiles_x = tx;
  a.tiles_y = ty;
  a.count = sp->count;
  a.depth = sp->depth;
  a.rect = sp->rect;
  a.n_entries = n_entries;
  a.keys = keys;
  a.vals = vals;
  a.ranges = tile_ranges;
  launch_bin_sort(a, w, (hipStream_t)stream);
  return check_launch();
}

size_t hyrf_composite_workspace_bytes(int32_t n_views, int32_t width, int32_t height) {
  Carve c(nullptr);
  c.take<uint32_t>((size_t)n_views * width * height);
  c.take<uint32_t>(1);
  return c.off;
}

hyrf_status hyrf_composite(const hyrf_splats* sp, const uint32_t* vals, const uint32_t* tile_ranges,
                           const hyrf_camera* cams, int32_t n_views, const hyrf_fields* fields,
                           int32_t mode, float* out_rgb, float* out_T, int32_t* out_last, float* out_bg,
                           float* out_bg_feat,
                           void* ws, size_t ws_bytes, void* stream) {
  hyrf_status s;
  if ((s = check_cams(cams, n_views)) != HYRF_OK) return s;
  REQ(mode == HYRF_RENDER || mode == HYRF_TRAIN, "mode must be HYRF_RENDER or HYRF_TRAIN");
  REQ(sp && sp->rec, "splats.rec is NULL");
  REQ(sp->n_max >= 0 && (int64_t)n_views * sp->n_max < ((int64_t)1 << 31), "splats.n_max out of range");
  REQ(((uintptr_t)sp->rec & 15) == 0, "splats.rec must be 16-byte aligned");
  REQ(vals && tile_ranges && out_rgb && out_T, "vals / tile_ranges / out_rgb / out_T is NULL");
  if (mode == HYRF_TRAIN) REQ(out_last && (out_bg || !fields), "TRAIN mode needs out_last and out_bg");
  if (fields && (s = check_fields(fields)) != HYRF_OK) return s;
  const int W = cams[0].width, H = cams[0].height;
  const size_t need = hyrf_composite_workspace_bytes(n_views, W, H);
  REQ(ws && ws_bytes >= need, "composite workspace too small: %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  Carve c(ws);
  uint32_t* list = c.take<uint32_t>((size_t)n_views * W * H);
  uint32_t* list_count = c.take<uint32_t>(1);
  CompArgs a{};
  a.W = W;
  a.H = H;
  a.tiles_x = (W + TILE - 1) / TILE;
  a.tiles_y = (H + TILE - 1) / TILE;
  a.rec = sp->rec;
  a.n_rec = (uint32_t)((int64_t)n_views * sp->n_max);
  a.vals = vals;
  a.ranges = tile_ranges;
  a.tau_T = fields ? fields->tau_T : 0.f;
  a.out_rgb = out_rgb;
  a.out_T = out_T;
  a.out_last = out_last;
  const bool render_bg = fields && mode == HYRF_RENDER;
  a.list = render_bg ? list : nullptr;
  a.list_count = render_bg ? list_count : nullptr;
  launch_composite(a, n_views, st);
  if (fields) {
    BgArgs b{};
    b.grid = make_grid(fields);
    b.cams = make_cams(cams, n_views);
    b.table_rad = fields->table_rad;
    b.w_col = fields->mlp_col;
    b.W = W;
    b.H = H;
    b.list = render_bg ? list : nullptr;
    b.list_count = render_bg ? list_count : nullptr;
    b.T = out_T;
    b.out_rgb = out_rgb;
    b.bg_save = mode == HYRF_TRAIN ? out_bg : nullptr;
    b.feat_save = mode == HYRF_TRAIN ? out_bg_feat : nullptr;
    launch_bg(fields->levels, fields->hidden, fields->n_hidden, fields->table_dtype,
              fields->mlp_dtype == HYRF_BF16, b, n_views * W * H, st);
  }
  return check_launch();
}

hyrf_status hyrf_background(const hyrf_fields* fields, const hyrf_camera* cams, int32_t n_views, float* out_bg,
                            float* out_bg_feat, void* stream) {
  hyrf_status s;
  if ((s = check_cams(cams, n_views)) != HYRF_OK) return s;
  if ((s = check_fields(fields)) != HYRF_OK) return s;
  REQ(out_bg, "out_bg is NULL");
  const int W = cams[0].width, H = cams[0].height;
  BgArgs b{};
  b.grid = make_grid(fields);
  b.cams = make_cams(cams, n_views);
  b.table_rad = fields->table_rad;
  b.w_col = fields->mlp_col;
  b.W = W;
  b.H = H;
  b.bg_save = out_bg;
  b.feat_save = out_bg_feat;
  launch_bg(fields->levels, fields->hidden, fields->n_hidden, fields->table_dtype, fields->mlp_dtype == HYRF_BF16,
            b, n_views * W * H, (hipStream_t)stream);
  return check_launch();
}

hyrf_status hyrf_blend_background(const float* bg, const float* T, float* rgb, int32_t n_views, int32_t width,
                                  int32_t height, void* stream) {
  REQ(bg && T && rgb, "bg / T / rgb is NULL");
  REQ(n_views >= 1 && width > 0 && height > 0, "sizes must be positive");
  REQ((int64_t)n_views * 3 * width * height < ((int64_t)1 << 40), "image too large");
  launch_blend_bg(bg, T, rgb, n_views, width * height, (hipStream_t)stream);
  return check_launch();
}

size_t hyrf_l1_workspace_bytes(int64_t n) { return l1_ws_elems(n) * sizeof(float); }

hyrf_status hyrf_l1_loss(const float* img, const float* target, int64_t n, float* loss, float* grad,
                         void* ws, size_t ws_bytes, void* stream) {
  REQ(img && target && loss, "img / target / loss is NULL");
  REQ(n > 0, "n must be positive");
  REQ(ws && ws_bytes >= hyrf_l1_workspace_bytes(n), "l1 workspace too small");
  launch_l1(img, target, n, loss, grad, (float*)ws, (hipStream_t)stream);
  return check_launch();
}

size_t hyrf_l1_dssim_workspace_bytes(int32_t planes, int32_t height, int32_t width) {
  if (planes <= 0 || height <= 0 || width <= 0) return 0;
  return l1_dssim_ws_elems(planes, height, width) * sizeof(float);
}

hyrf_status hyrf_l1_dssim_loss(const float* img, const float* target, int32_t planes, int32_t height,
                               int32_t width, float lambda, float* loss, float* grad, void* ws,
                               size_t ws_bytes, void* stream) {
  REQ(img && target && loss, "img / target / loss is NULL");
  REQ(planes > 0 && height > 0 && width > 0, "planes / height / width must be positive");
  REQ(planes <= 65535, "planes = %d exceeds 65535", planes);
  REQ((int64_t)planes * height * width < (int64_t)1 << 31, "image too large");
  REQ(lambda >= 0.f && lambda <= 1.f, "lambda = %g outside [0, 1]", (double)lambda);
  REQ(ws && ws_bytes >= hyrf_l1_dssim_workspace_bytes(planes, height, width), "l1_dssim workspace too small");
  launch_l1_dssim(img, target, planes, height, width, lambda, loss, grad, (float*)ws, (hipStream_t)stream);
  return check_launch();
}

namespace {
constexpr int BWD_MAX_BLOCKS = 256;   // persistent: one 8-wave workgroup per CU

struct BwdWs {
  float *gs, *dgeo, *dcol, *dfeat_geo, *dfeat_rad, *wf_geo, *wf_col, *wb_geo, *wb_col, *dw_part;
  size_t bytes;
};

BwdWs carve_bwd(void* base, const hyrf_fields* f, int V, int n_max) {
  size_t fg = 0, fc = 0, bg = 0, bc = 0, nw = 0;
  bwd_weight_floats(f->levels, f->hidden, f->n_hidden, &fg, &fc, &bg, &bc, &nw);
  Carve c(base);
  BwdWs w;
  const size_t nm = n_max > 0 ? (size_t)n_max : 1;
  w.gs = c.take<float>((size_t)V * nm * 9);
  w.dgeo = c.take<float>(nm * 8);
  w.dcol = c.take<float>(nm * V * 3);
  w.dfeat_geo = c.take<float>(nm * 2 * f->levels);
  w.dfeat_rad = c.take<float>(nm * 2 * f->levels);
  w.wf_geo = c.take<float>(fg);
  w.wf_col = c.take<float>(fc);
  w.wb_geo = c.take<float>(bg);
  w.wb_col = c.take<float>(bc);
  w.dw_part = c.take<float>((size_t)2 * BWD_MAX_BLOCKS * nw);
  w.bytes = c.off;
  return w;
}
}  // namespace

size_t hyrf_backward_workspace_bytes(const hyrf_fields* fields, int32_t n_views, int32_t n_max, int32_t width,
                                     int32_t height) {
  if (!fields || !shape_supported(fields->levels, fields->hidden, fields->n_hidden) || n_views < 1) return 0;
  return carve_bwd(nullptr, fields, n_views, n_max).bytes;
}

static hyrf_status backward_impl(int stages, const hyrf_fields* fields, const hyrf_gaussians* g,
                                 const hyrf_camera* cams, int32_t n_views, const hyrf_fwd_state* saved,
                                 const float* dL_drgb, const hyrf_grads* grads, void* ws, size_t ws_bytes,
                                 void* stream) {
  hyrf_status s;
  if ((s = check_fields(fields)) != HYRF_OK) return s;
  if (fields->table_dtype == HYRF_U8)
    return fail(HYRF_ERR_UNSUPPORTED, "8-bit quantised tables are a render-only format (no backward)");
  if ((s = check_gauss(g)) != HYRF_OK) return s;
  if (g->pos_dtype != HYRF_F32)
    return fail(HYRF_ERR_UNSUPPORTED, "float16 positions are a render-only format (no backward)");
  if ((s = check_cams(cams, n_views)) != HYRF_OK) return s;
  REQ(saved && saved->query && saved->splats, "saved forward state is incomplete");
  const hyrf_query_out* q = saved->query;
  const hyrf_splats* sp = saved->splats;
  REQ(q->vis_count && q->vis_idx && q->opacity && q->scale && q->quat && q->rgb,
      "saved query output is incomplete");
  REQ(q->feat_geo && q->feat_rad, "backward needs the features saved by a TRAIN-mode query");
  REQ(sp->rec && sp->rect && sp->n_max >= g->n && sp->n_max >= 1, "saved splats are incomplete");
  REQ(((uintptr_t)sp->rec & 15) == 0 && ((uintptr_t)sp->rect & 15) == 0, "splats.rec / rect must be 16-byte aligned");
  REQ(saved->vals && saved->tile_ranges && saved->T_final && saved->last && saved->bg_rgb,
      "saved composite state (vals, tile_ranges, T_final, last, bg_rgb) is incomplete");
  REQ(dL_drgb && grads, "dL_drgb / grads is NULL");
  REQ(!grads->dens_accum == !grads->dens_count, "dens_accum and dens_count must both be set or both NULL");
  REQ((int64_t)n_views * sp->n_max < ((int64_t)1 << 31), "too many splats");
  const size_t need = hyrf_backward_workspace_bytes(fields, n_views, sp->n_max, cams[0].width, cams[0].height);
  REQ(ws && ws_bytes >= need, "backward workspace too small: %zu < %zu bytes", ws_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  BwdWs w = carve_bwd(ws, fields, n_views, sp->n_max);
  const int W = cams[0].width, H = cams[0].height;
  BwdLaunch L{};
  L.stages = stages;
  L.V = n_views;
  L.comp.W = W;
  L.comp.H = H;
  L.comp.tiles_x = (W + TILE - 1) / TILE;
  L.comp.tiles_y = (H + TILE - 1) / TILE;
  L.comp.rec = sp->rec;
  L.comp.n_rec = (uint32_t)((int64_t)n_views * sp->n_max);
  L.comp.vals = saved->vals;
  L.comp.ranges = saved->tile_ranges;
  L.comp.T_final = saved->T_final;
  L.comp.last = saved->last;
  L.comp.bg = saved->bg_rgb;
  L.field.bg_feat = saved->bg_feat;
  L.comp.dL = dL_drgb;
  L.comp.gs = w.gs;
  L.n_gs = (int64_t)n_views * sp->n_max * 9;
  const Cams cc = make_cams(cams, n_views);
  L.proj.cams = cc;
  L.proj.n = g->n;
  L.proj.n_max = sp->n_max;
  L.proj.count = q->vis_count;
  L.proj.vis_idx = q->vis_idx;
  L.proj.pos = static_cast<const float*>(g->pos);
  L.proj.opacity = q->opacity;
  L.proj.scale = q->scale;
  L.proj.quat = q->quat;
  L.proj.rgb = q->rgb;
  L.proj.rect = sp->rect;
  L.proj.gs = w.gs;
  L.proj.g_pos = grads->pos;
  L.proj.g_scale_e = grads->scale_e;
  L.proj.g_opac_e = grads->opac_e;
  L.proj.g_col_e = grads->col_e;
  L.proj.dgeo = w.dgeo;
  L.proj.dcol = w.dcol;
  L.proj.dens_accum = grads->dens_accum;
  L.proj.dens_count = grads->dens_accum ? grads->dens_count : nullptr;
  FieldBwdArgs& F = L.field;
  F.grid = make_grid(fields);
  F.cams = cc;
  F.table_geo = geo_table(fields);
  F.table_rad = fields->table_rad;
  F.n = g->n;
  F.count = q->vis_count;
  F.vis_idx = q->vis_idx;
  F.pos = static_cast<const float*>(g->pos);
  F.rot_e = g->rot_e;
  F.feat_geo = q->feat_geo;
  F.feat_rad = q->feat_rad;
  F.jac = q->feat_jac;
  F.merge = fields->scatter_merge == 2 ? 0 : 1;
  F.dgeo = w.dgeo;
  F.dcol = w.dcol;
  F.n_max = sp->n_max;
  F.dfeat_geo = w.dfeat_geo;
  F.dfeat_rad = w.dfeat_rad;
  F.g_pos = grads->pos;
  F.g_rot_e = grads->rot_e;
  F.g_table_geo = fields->single_field ? nullptr : grads->table_geo;
  F.g_table_rad = grads->table_rad;
  F.dw_part = w.dw_part;
  F.W = W;
  F.H = H;
  F.T_final = saved->T_final;
  F.dL = dL_drgb;
  L.w_geo = fields->mlp_geo;
  L.w_col = fields->mlp_col;
  L.wf_geo = w.wf_geo;
  L.wf_col = w.wf_col;
  L.wb_geo = w.wb_geo;
  L.wb_col = w.wb_col;
  const int64_t rg = ((int64_t)g->n + BWD_PPR_GAUSS - 1) / BWD_PPR_GAUSS;
  const int64_t rr = ((int64_t)n_views * W * H + BWD_PPR_BG - 1) / BWD_PPR_BG;
  L.blocks_g = (int)(rg < 1 ? 1 : (rg > BWD_MAX_BLOCKS ? BWD_MAX_BLOCKS : rg));
  L.blocks_r = (int)(rr < 1 ? 1 : (rr > BWD_MAX_BLOCKS ? BWD_MAX_BLOCKS : rr));
  L.with_bg = true;
  L.f16 = fields->table_dtype == HYRF_F16;
  L.bf = fields->mlp_dtype == HYRF_BF16;
  L.g_mlp_geo = grads->mlp_geo;
  L.g_mlp_col = grads->mlp_col;
  launch_backward(fields->levels, fields->hidden, fields->n_hidden, L, st);
  return check_launch();
}

hyrf_status hyrf_render_backward(const hyrf_fields* fields, const hyrf_gaussians* g, const hyrf_camera* cams,
                                 int32_t n_views, const hyrf_fwd_state* saved, const float* dL_drgb,
                                 const hyrf_grads* grads, void* ws, size_t ws_bytes, void* stream) {
  return backward_impl(BWD_STAGE_ALL, fields, g, cams, n_views, saved, dL_drgb, grads, ws, ws_bytes, stream);
}

hyrf_status hyrf_render_backward_stage(int32_t stage, const hyrf_fields* fields, const hyrf_gaussians* g,
                                       const hyrf_camera* cams, int32_t n_views, const hyrf_fwd_state* saved,
                                       const float* dL_drgb, const hyrf_grads* grads, void* ws, size_t ws_bytes,
                                       void* stream) {
  REQ(stage >= 0 && stage <= 6, "stage = %d outside [0, 6]", stage);
  return backward_impl(1 << stage, fields, g, cams, n_views, saved, dL_drgb, grads, ws, ws_bytes, stream);
}

size_t hyrf_spatial_order_workspace_bytes(int32_t n) { return order_ws_bytes(n); }

hyrf_status hyrf_adam_step(const hyrf_adam_group* groups, int32_t n_groups, int32_t step, float beta1,
                           float beta2, float eps, int32_t zero_grad, void* stream) {
  REQ(groups, "groups is NULL");
  REQ(n_groups >= 1 && n_groups <= HYRF_ADAM_MAX_GROUPS, "n_groups = %d outside [1, %d]", n_groups,
      HYRF_ADAM_MAX_GROUPS);
  REQ(step >= 1, "step must be >= 1");
  REQ(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f, "betas must be in [0, 1)");
  REQ(eps >= 0.f, "eps must be >= 0");
  for (int k = 0; k < n_groups; ++k) {
    const hyrf_adam_group& g = groups[k];
    REQ(g.n >= 0, "group %d: n < 0", k);
    if (g.n == 0) continue;
    REQ(g.param && g.grad && g.m && g.v, "group %d: param / grad / m / v is NULL", k);
    REQ((((uintptr_t)g.param | (uintptr_t)g.grad | (uintptr_t)g.m | (uintptr_t)g.v) & 15) == 0,
        "group %d: pointers must be 16-byte aligned", k);
    REQ(((uintptr_t)g.param_half & 1) == 0, "group %d: param_half must be 2-byte aligned", k);
  }
  if (adam_launch(groups, n_groups, step, beta1, beta2, eps, zero_grad, (hipStream_t)stream) != 0)
    return fail(HYRF_ERR_INVALID_ARGUMENT, "too many parameters for one launch");
  return check_launch();
}

hyrf_status hyrf_densify_masks(const hyrf_query_out* q, int32_t n, int32_t n_max, const float* dens_accum,
                               const float* dens_count, float grad_threshold, float dense_extent,
                               float min_opacity, uint8_t* flags, void* stream) {
  REQ(q && q->vis_count && q->vis_idx && q->opacity && q->scale, "query output is incomplete");
  REQ(n >= 1 && n_max >= n, "need 1 <= n <= n_max");
  REQ(dens_accum && dens_count && flags, "dens_accum / dens_count / flags is NULL");
  launch_densify_masks(n, n_max, q->vis_count, q->vis_idx, q->opacity, q->scale, dens_accum, dens_count,
                       grad_threshold, dense_extent, min_opacity, flags, (hipStream_t)stream);
  return check_launch();
}

hyrf_status hyrf_reset_opacity(float* opac_e, int32_t n, float value, void* stream) {
  REQ(opac_e, "opac_e is NULL");
  REQ(n >= 1, "n must be >= 1");
  REQ(value > 0.f && value < 1.f, "value must be in (0, 1)");
  launch_reset_opacity(opac_e, n, value, (hipStream_t)stream);
  return check_launch();
}

size_t hyrf_quantize_workspace_bytes(int32_t levels, int32_t log2_T) {
  if (levels < 1 || levels > 16 || log2_T < 1 || log2_T > 24) return 0;
  return quant_ws_elems(levels, log2_T) * sizeof(float);
}

hyrf_status hyrf_quantize_table(const float* table, int32_t levels, int32_t log2_T, uint8_t* codes,
                                float* qparams, void* ws, size_t ws_bytes, void* stream) {
  REQ(table && codes && qparams, "table / codes / qparams is NULL");
  REQ(levels >= 1 && levels <= 16, "levels = %d outside [1, 16]", levels);
  REQ(log2_T >= 1 && log2_T <= 24, "log2_T = %d outside [1, 24]", log2_T);
  REQ(((uintptr_t)table & 15) == 0 && ((uintptr_t)codes & 3) == 0,
      "table must be 16-byte and codes 4-byte aligned");
  REQ(ws && ws_bytes >= hyrf_quantize_workspace_bytes(levels, log2_T), "quantize workspace too small");
  launch_quantize(table, levels, log2_T, codes, qparams, (float*)ws, (hipStream_t)stream);
  return check_launch();
}

hyrf_status hyrf_spatial_order(const hyrf_fields* fields, const float* pos, int32_t n, uint32_t* perm, void* ws,
                               size_t ws_bytes, void* stream) {
  REQ(fields, "fields is NULL");
  REQ(n >= 0, "n must be >= 0");
  REQ(n == 0 || (pos && perm), "pos / perm is NULL");
  for (int d = 0; d < 3; ++d) REQ(fields->aabb_inv_half[d] > 0.f, "aabb_inv_half must be positive");
  REQ(ws && ws_bytes >= order_ws_bytes(n), "spatial_order workspace too small");
  GridP g{};
  for (int d = 0; d < 3; ++d) {
    g.center[d] = fields->aabb_center[d];
    g.inv_half[d] = fields->aabb_inv_half[d];
  }
  const hipError_t e = launch_order(pos, n, g, perm, ws, (hipStream_t)stream);
  if (e != hipSuccess) return launch_error(e);
  return check_launch();
}

}  // extern "C"

// ---------------------------------------------------------------- query without a workspace
// The query's scratch (cull flags, their exclusive scan and the scan's
// per-workgroup partials) in a device array that the library holds, for
// callers that cannot allocate.  Each GPU that loads the library holds its
// own copy of the array until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that device (the
// array's name on the host is a stand-in, not a device address).
namespace {

constexpr int64_t NOALLOC_MAX_N = HYRF_QUERY_NOALLOC_MAX_GAUSSIANS;

constexpr size_t scan_temp_elems_bound(int64_t n) {
  size_t s = 0;
  while (n > SCAN_ITEMS) {
    const int64_t nb = (n + SCAN_ITEMS - 1) / SCAN_ITEMS;
    s += (size_t)nb;
    n = nb;
  }
  return s + 1;
}

// query_ws of the largest accepted n: two arrays of n words, each start
// rounded up to 256 bytes (64 words), then the scan partials
constexpr size_t NOALLOC_WORDS = 2 * (size_t)NOALLOC_MAX_N + 64 + scan_temp_elems_bound(NOALLOC_MAX_N);

}  // namespace

static __device__ __align__(256) uint32_t scratch[NOALLOC_WORDS];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the calling thread's current device,
// looked up once per device.
hyrf_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HYRF_ERR_LAUNCH, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(HYRF_ERR_UNSUPPORTED, "device %d outside the %d devices the scratch table covers", dev,
                NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HYRF_ERR_LAUNCH, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return HYRF_OK;
}

}  // namespace

extern "C" {

size_t hyrf_query_noalloc_scratch_bytes(void) { return sizeof(scratch); }

hyrf_status hyrf_query_fields_noalloc(const hyrf_fields* fields, const hyrf_gaussians* g,
                                      const hyrf_camera* cams, int32_t n_views, const hyrf_query_out* out,
                                      void* stream) {
  hyrf_status s;
  if ((s = check_query(fields, g, cams, n_views, out)) != HYRF_OK) return s;
  if (g->n > NOALLOC_MAX_N)
    return fail(HYRF_ERR_CAPACITY, "hyrf_query_fields_noalloc: n = %d exceeds the %lld Gaussians its scratch holds",
                g->n, (long long)NOALLOC_MAX_N);
  if (query_ws(g->n, nullptr, nullptr, nullptr, nullptr) > sizeof(scratch))
    return fail(HYRF_ERR_CAPACITY, "hyrf_query_fields_noalloc: scratch too small for n = %d", g->n);
  void* ptr = nullptr;
  if ((s = scratch_address(&ptr)) != HYRF_OK) return s;
  // nothing in the scratch needs to start at zero: the cull writes every
  // flag, the scan every position and partial it reads
  launch_query_all(fields, g, cams, n_views, out, ptr, (hipStream_t)stream);
  return check_launch();
}

}  // extern "C"
