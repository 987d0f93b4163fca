// C ABI of the rasterizer library: argument checks, view tables, dispatch.
// Every entry point validates its arguments before enqueuing anything and
// never throws; kernels are enqueued on the caller's stream only.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gs_internal.hpp"

namespace gsk {

// ------------------------------------------------------------ event tracing
bool g_profile_on = false;
namespace {
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
  bool failed;  // an event could not be recorded: the collection reports an error
};
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;
hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

void profile_begin(const char* name, hipStream_t st) {
  ProfRec r{name, take_event(), nullptr, false};
  if (r.a && hipEventRecord(r.a, st) != hipSuccess) r.failed = true;
  g_recs.push_back(r);
}

void profile_end(hipStream_t st) {
  if (g_recs.empty()) return;
  ProfRec& r = g_recs.back();
  r.b = take_event();
  if (r.b && hipEventRecord(r.b, st) != hipSuccess) r.failed = true;
}

bool build_views(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg, Views* out) {
  if (!cams || !cfg || !out || n_views < 1 || n_views > GS_MAX_VIEWS) return false;
  if (cfg->tile != 8 && cfg->tile != 16 && cfg->tile != 32) return false;
  if (cfg->lds_batch != 128 && cfg->lds_batch != 256 && cfg->lds_batch != 512) return false;
  if (cfg->mip2d != 0 && cfg->mip2d != 1) return false;
  std::memset(out, 0, sizeof(Views));
  out->n_views = n_views;
  out->tile = cfg->tile;
  out->mip2d = cfg->mip2d;
  out->filter3d = cfg->filter3d;
  // a device camera table drives view 0 of a one-view call
  if ((cfg->cam_table == nullptr) != (cfg->cam_index == nullptr)) return false;
  if (cfg->cam_table && n_views != 1) return false;
  out->cam_table = cfg->cam_table;
  out->cam_index = cfg->cam_index;
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const gs_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384) return false;
    if (!(c.near_plane > 0.0f) || !std::isfinite(c.fx) || !std::isfinite(c.fy)) return false;
    DevView& d = out->v[v];
    for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
    for (int k = 0; k < 3; ++k)  // -R^T t in double, rounded once
      d.campos[k] = float(-(double(c.R[k]) * c.t[0] + double(c.R[3 + k]) * c.t[1] +
                            double(c.R[6 + k]) * c.t[2]));
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    d.near_plane = c.near_plane;
    d.W = c.width;
    d.H = c.height;
    d.gw = (c.width + cfg->tile - 1) / cfg->tile;
    d.gh = (c.height + cfg->tile - 1) / cfg->tile;
    d.tile_base = int32_t(tiles);
    d.pix_base = pix;
    tiles += int64_t(d.gw) * d.gh;
    pix += int64_t(c.width) * c.height;
  }
  if (tiles >= (int64_t(1) << 31)) return false;
  out->total_tiles = int32_t(tiles);
  return true;
}

}  // namespace gsk

using namespace gsk;

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

gs_status from_hip(hipError_t e) { return e == hipSuccess ? GS_OK : GS_ERR_DEVICE; }

bool n_ok(int32_t n_views, int32_t n) {
  return n >= 0 && n_views >= 1 && int64_t(n) * n_views < (int64_t(1) << 31);
}

}  // namespace

extern "C" {

int32_t gs_version(void) { return 1; }

void gs_profile_enable(int32_t on) { gsk::g_profile_on = on != 0; }

int32_t gs_profile_collect(gs_kernel_time* out, int32_t max_entries) {
  using gsk::g_recs;
  std::vector<gs_kernel_time> agg;
  bool err = false;
  for (auto& r : g_recs) {
    float ms = 0.0f;
    if (r.failed || !r.a || !r.b || hipEventSynchronize(r.b) != hipSuccess ||
        hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      err = true;
    }
    std::string nm(r.name);
    size_t k = 0;
    while (k < agg.size() && nm != agg[k].name) ++k;
    if (k == agg.size()) {
      gs_kernel_time t{};
      std::strncpy(t.name, r.name, sizeof(t.name) - 1);
      agg.push_back(t);
    }
    agg[k].launches += 1;
    agg[k].total_ms += ms;
    if (r.a) gsk::g_pool.push_back(r.a);
    if (r.b) gsk::g_pool.push_back(r.b);
  }
  g_recs.clear();
  if (err) return -1;
  const int32_t n = int32_t(agg.size()) < max_entries ? int32_t(agg.size()) : max_entries;
  for (int32_t i = 0; i < n && out; ++i) out[i] = agg[i];
  return n;
}

const char* gs_status_str(gs_status s) {
  switch (s) {
    case GS_OK: return "ok";
    case GS_ERR_ARG: return "invalid argument";
    case GS_ERR_CAPACITY: return "workspace or capacity too small";
    case GS_ERR_DEVICE: return "HIP launch failed";
    case GS_ERR_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

size_t gs_proj_bytes(int32_t n_views, int32_t n) {
  if (!n_ok(n_views, n) || n_views > GS_MAX_VIEWS) return 0;
  return size_t(n_views) * ProjLayout(n).stride;
}

int64_t gs_total_tiles(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg) {
  Views V;
  if (!build_views(n_views, cams, cfg, &V)) return -1;
  return V.total_tiles;
}

gs_status gs_filter3d_variance(int32_t n_views, const gs_camera* cams, int32_t n,
                               const float* means, float scale, float* variance,
                               uint32_t* scratch, void* stream) {
  gs_raster_cfg cfg{};  // the cameras only: any valid tiling
  cfg.tile = 16;
  cfg.lds_batch = 128;
  if (n_views < 1 || !cams || n < 0) return GS_ERR_ARG;
  if (!(scale >= 0.0f) || !std::isfinite(scale)) return GS_ERR_ARG;
  if (n > 0 && (!means || !variance || !scratch)) return GS_ERR_ARG;
  // the views in chunks of at most GS_MAX_VIEWS (one kernel argument each)
  std::vector<Views> chunks;
  for (int v0 = 0; v0 < n_views; v0 += GS_MAX_VIEWS) {
    Views V;
    if (!build_views(std::min(GS_MAX_VIEWS, n_views - v0), cams + v0, &cfg, &V)) return GS_ERR_ARG;
    chunks.push_back(V);
  }
  hipStream_t st = as_stream(stream);
  for (size_t k = 0; k < chunks.size(); ++k) {
    const hipError_t e = launch_filter3d_rate(chunks[k], n, k == 0 ? 1 : 0, means, variance, st);
    if (e != hipSuccess) return from_hip(e);
  }
  return from_hip(launch_filter3d_var(n, scale, variance, scratch, st));
}

gs_status gs_preprocess(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                        int32_t n, const float* means, const float* log_scales,
                        const float* quats, const float* opacity_logits, const float* sh,
                        int32_t sh_degree, void* proj, void* stream) {
  Views V;
  if (!n_ok(n_views, n) || !build_views(n_views, cams, cfg, &V)) return GS_ERR_ARG;
  if (sh_degree < 0 || sh_degree > 3) return GS_ERR_ARG;
  if (n > 0 && (!means || !log_scales || !quats || !opacity_logits || !sh || !proj))
    return GS_ERR_ARG;
  if (n > 0 && (!aligned16(quats) || !aligned16(sh) || !aligned16(proj))) return GS_ERR_ARG;
  return from_hip(launch_preprocess(V, n, sh_degree, means, log_scales, quats, opacity_logits, sh,
                                    static_cast<char*>(proj), as_stream(stream)));
}

size_t gs_bin_sort_workspace_bytes(int32_t n_views, int32_t n, int64_t capacity_pairs) {
  if (!n_ok(n_views, n) || capacity_pairs < 0 || capacity_pairs >= (int64_t(1) << 32)) return 0;
  return bin_sort_ws_bytes(n_views, n, capacity_pairs);
}

gs_status gs_bin_sort(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                      int32_t n, void* proj, int64_t capacity_pairs, void* ws,
                      size_t ws_bytes, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                      int64_t* n_pairs_dev, void* stream) {
  Views V;
  if (!n_ok(n_views, n) || !build_views(n_views, cams, cfg, &V)) return GS_ERR_ARG;
  if (capacity_pairs < 0 || capacity_pairs >= (int64_t(1) << 32)) return GS_ERR_ARG;
  if (!ws || !ranges || !n_pairs_dev || (n > 0 && !proj) || (capacity_pairs > 0 && !vals))
    return GS_ERR_ARG;
  if (ws_bytes < bin_sort_ws_bytes(n_views, n, capacity_pairs)) return GS_ERR_CAPACITY;
  if (!aligned16(ws) || (n > 0 && !aligned16(proj))) return GS_ERR_ARG;
  return from_hip(launch_bin_sort(V, n, static_cast<char*>(proj), capacity_pairs, ws, keys,
                                  vals, ranges, n_pairs_dev, as_stream(stream)));
}

gs_status gs_bin_sort_noalloc(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                              int32_t n, void* proj, int64_t capacity_pairs,
                              uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                              int64_t* n_pairs_dev, void* stream) {
  Views V;
  if (!n_ok(n_views, n) || !build_views(n_views, cams, cfg, &V)) return GS_ERR_ARG;
  if (capacity_pairs < 0) return GS_ERR_ARG;
  if (capacity_pairs > GS_BIN_SORT_NOALLOC_MAX_PAIRS ||
      int64_t(n_views) * n > GS_BIN_SORT_NOALLOC_MAX_ITEMS)
    return GS_ERR_CAPACITY;
  if (!ranges || !n_pairs_dev || (n > 0 && !proj) || (capacity_pairs > 0 && !vals))
    return GS_ERR_ARG;
  if (n > 0 && !aligned16(proj)) return GS_ERR_ARG;
  return from_hip(launch_bin_sort_noalloc(V, n, static_cast<char*>(proj), capacity_pairs,
                                          keys, vals, ranges, n_pairs_dev, as_stream(stream)));
}

size_t gs_spatial_order_workspace_bytes(int32_t n) {
  return n < 0 ? 0 : spatial_order_ws_bytes(n);
}

gs_status gs_spatial_order(int32_t n, const float* means, void* ws, size_t ws_bytes,
                           uint32_t* perm, void* stream) {
  if (n < 0 || (n > 0 && (!means || !ws || !perm))) return GS_ERR_ARG;
  if (ws_bytes < spatial_order_ws_bytes(n)) return GS_ERR_CAPACITY;
  return from_hip(launch_spatial_order(n, means, ws, perm, as_stream(stream)));
}

gs_status gs_gather_rows(int32_t n, const uint32_t* perm, int32_t n_arrays,
                         const float* const* src, float* const* dst, const int32_t* row_floats,
                         void* stream) {
  if (n < 0 || n_arrays < 0 || n_arrays > kGatherMaxArrays) return GS_ERR_ARG;
  if (n == 0 || n_arrays == 0) return GS_OK;
  if (!perm || !src || !dst || !row_floats) return GS_ERR_ARG;
  for (int a = 0; a < n_arrays; ++a) {
    if (!src[a] || !dst[a] || row_floats[a] < 1 || row_floats[a] > kGatherMaxRow) return GS_ERR_ARG;
    if (int64_t(n) * row_floats[a] >= (int64_t(1) << 40)) return GS_ERR_ARG;
  }
  return from_hip(launch_gather_rows(n, perm, n_arrays, src, dst, row_floats, as_stream(stream)));
}

size_t gs_bin_sort_radix_workspace_bytes(int32_t n_views, int32_t n, int64_t capacity_pairs) {
  if (!n_ok(n_views, n) || capacity_pairs < 0 || capacity_pairs >= (int64_t(1) << 32)) return 0;
  return bin_sort_radix_ws_bytes(n_views, n, capacity_pairs);
}

gs_status gs_bin_sort_radix(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                            int32_t n, void* proj, int64_t capacity_pairs, void* ws,
                            size_t ws_bytes, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                            int64_t* n_pairs_dev, void* stream) {
  Views V;
  if (!n_ok(n_views, n) || !build_views(n_views, cams, cfg, &V)) return GS_ERR_ARG;
  if (capacity_pairs < 0 || capacity_pairs >= (int64_t(1) << 32)) return GS_ERR_ARG;
  if (!ws || !ranges || !n_pairs_dev || (n > 0 && !proj) || (capacity_pairs > 0 && !vals))
    return GS_ERR_ARG;
  if (ws_bytes < bin_sort_radix_ws_bytes(n_views, n, capacity_pairs)) return GS_ERR_CAPACITY;
  if (!aligned16(ws) || (n > 0 && !aligned16(proj))) return GS_ERR_ARG;
  return from_hip(launch_bin_sort_radix(V, n, static_cast<char*>(proj), capacity_pairs, ws,
                                        keys, vals, ranges, n_pairs_dev, as_stream(stream)));
}

gs_status gs_render_fwd(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                        int32_t n, const void* proj, const uint32_t* ranges,
                        const uint32_t* vals, float* image, float* final_T,
                        uint32_t* last_contrib, void* stream) {
  Views V;
  if (!n_ok(n_views, n) || !build_views(n_views, cams, cfg, &V)) return GS_ERR_ARG;
  if (!ranges || !image || !final_T || !last_contrib || (n > 0 && !proj)) return GS_ERR_ARG;
  if (n > 0 && !aligned16(proj)) return GS_ERR_ARG;
  return from_hip(launch_render_fwd(V, n, *cfg, static_cast<const char*>(proj), ranges, vals,
                                    image, final_T, last_contrib, L1Fuse{}, as_stream(stream)));
}

gs_status gs_render_fwd_l1(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                           int32_t n, const void* proj, const uint32_t* ranges,
                           const uint32_t* vals, float* image, float* final_T,
                           uint32_t* last_contrib, const float* target, float scale,
                           float* dL_dimage, float* loss_sum, void* stream) {
  Views V;
  if (!n_ok(n_views, n) || !build_views(n_views, cams, cfg, &V)) return GS_ERR_ARG;
  if (!ranges || !image || !final_T || !last_contrib || (n > 0 && !proj)) return GS_ERR_ARG;
  if (!target || !dL_dimage) return GS_ERR_ARG;
  if (n > 0 && !aligned16(proj)) return GS_ERR_ARG;
  // with a camera table the target is the table's view's entry of a stack
  const L1Fuse l1{target, dL_dimage, loss_sum, scale, cfg->cam_index,
                  3 * int64_t(cams[0].width) * cams[0].height};
  return from_hip(launch_render_fwd(V, n, *cfg, static_cast<const char*>(proj), ranges, vals,
                                    image, final_T, last_contrib, l1, as_stream(stream)));
}

size_t gs_render_bwd_workspace_bytes(int32_t n_views, int32_t n, int64_t capacity_pairs) {
  if (!n_ok(n_views, n) || capacity_pairs < 0 || capacity_pairs >= (int64_t(1) << 32)) return 0;
  return render_bwd_ws_bytes(n_views, n, capacity_pairs);
}

gs_status gs_render_bwd(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                        int32_t n, const float* means, const float* log_scales,
                        const float* quats, const float* opacity_logits, const float* sh,
                        int32_t sh_degree, const void* proj, const uint32_t* ranges,
                        const uint32_t* vals, const float* final_T,
                        const uint32_t* last_contrib, const float* dL_dimage, float* d_means,
                        float* d_log_scales, float* d_quats, float* d_opacity_logits,
                        float* d_sh, float* d_mean2d_abs, int32_t accumulate,
                        int64_t capacity_pairs, void* ws, size_t ws_bytes, void* stream) {
  Views V;
  if (!n_ok(n_views, n) || !build_views(n_views, cams, cfg, &V)) return GS_ERR_ARG;
  if (sh_degree < 0 || sh_degree > 3) return GS_ERR_ARG;
  if (capacity_pairs < 0 || capacity_pairs >= (int64_t(1) << 32)) return GS_ERR_ARG;
  if (!ranges || !final_T || !last_contrib || !dL_dimage || !ws) return GS_ERR_ARG;
  if (n > 0 && (!means || !log_scales || !quats || !opacity_logits || !sh || !proj || !d_means ||
                !d_log_scales || !d_quats || !d_opacity_logits || !d_sh))
    return GS_ERR_ARG;
  if (n > 0 && (!aligned16(quats) || !aligned16(d_quats) || !aligned16(proj) || !aligned16(ws)))
    return GS_ERR_ARG;
  if (ws_bytes < render_bwd_ws_bytes(n_views, n, capacity_pairs)) return GS_ERR_CAPACITY;
  return from_hip(launch_render_bwd(V, n, *cfg, means, log_scales, quats, opacity_logits, sh,
                                    sh_degree, static_cast<const char*>(proj), ranges, vals,
                                    final_T, last_contrib, dL_dimage, d_means, d_log_scales,
                                    d_quats, d_opacity_logits, d_sh, d_mean2d_abs,
                                    accumulate != 0, capacity_pairs, ws, as_stream(stream)));
}

gs_status gs_adam_step(const gs_adam_group* groups, int32_t n_groups, int32_t step, float beta1,
                       float beta2, float eps, void* stream) {
  if (!groups || n_groups < 1 || n_groups > GS_MAX_ADAM_GROUPS || step < 1) return GS_ERR_ARG;
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f))
    return GS_ERR_ARG;
  for (int k = 0; k < n_groups; ++k) {
    const gs_adam_group& g = groups[k];
    if (g.numel < 0) return GS_ERR_ARG;
    if (g.numel > 0 && (!g.p || !g.g || !g.m || !g.v)) return GS_ERR_ARG;
  }
  return from_hip(
      launch_adam(groups, n_groups, step, beta1, beta2, eps, nullptr, as_stream(stream)));
}

gs_status gs_adam_step_device(const gs_adam_group* groups, int32_t n_groups, int32_t* step_dev,
                              float beta1, float beta2, float eps, void* stream) {
  if (!groups || !step_dev || n_groups < 1 || n_groups > GS_MAX_ADAM_GROUPS) return GS_ERR_ARG;
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f))
    return GS_ERR_ARG;
  for (int k = 0; k < n_groups; ++k) {
    const gs_adam_group& g = groups[k];
    if (g.numel < 0) return GS_ERR_ARG;
    if (g.numel > 0 && (!g.p || !g.g || !g.m || !g.v)) return GS_ERR_ARG;
  }
  return from_hip(
      launch_adam(groups, n_groups, 1, beta1, beta2, eps, step_dev, as_stream(stream)));
}

namespace {
gs_status render_bwd_adam(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                          int32_t n, float* means, float* log_scales, float* quats,
                          float* opacity_logits, float* sh, int32_t sh_degree, const void* proj,
                          const uint32_t* ranges, const uint32_t* vals, const float* final_T,
                          const uint32_t* last_contrib, const float* dL_dimage, float* const* m,
                          float* const* v, const float* lr, int32_t* step_dev, float beta1,
                          float beta2, float eps, float* d_mean2d_abs, int64_t capacity_pairs,
                          void* ws, size_t ws_bytes, void* stream, int sparse) {
  Views V;
  if (!n_ok(n_views, n) || !build_views(n_views, cams, cfg, &V)) return GS_ERR_ARG;
  if (sh_degree < 0 || sh_degree > 3) return GS_ERR_ARG;
  if (capacity_pairs < 0 || capacity_pairs >= (int64_t(1) << 32)) return GS_ERR_ARG;
  if (!ranges || !final_T || !last_contrib || !dL_dimage || !ws || !m || !v || !step_dev)
    return GS_ERR_ARG;
  if (!lr && !cfg->adam_lr) return GS_ERR_ARG;
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f))
    return GS_ERR_ARG;
  FusedAdam A{};
  for (int k = 0; k < 5; ++k) {
    if (n > 0 && (!m[k] || !v[k])) return GS_ERR_ARG;
    A.m[k] = m[k];
    A.v[k] = v[k];
  }
  for (int k = 0; k < 6; ++k) A.lr[k] = lr ? lr[k] : 0.0f;
  A.lr_dev = cfg->adam_lr;
  if (n > 0 && (!means || !log_scales || !quats || !opacity_logits || !sh || !proj))
    return GS_ERR_ARG;
  if (n > 0 && (!aligned16(quats) || !aligned16(sh) || !aligned16(proj) || !aligned16(ws) ||
                !aligned16(m[2]) || !aligned16(v[2]) || !aligned16(m[4]) || !aligned16(v[4])))
    return GS_ERR_ARG;
  if (ws_bytes < render_bwd_ws_bytes(n_views, n, capacity_pairs)) return GS_ERR_CAPACITY;
  A.b1 = beta1;
  A.b2 = beta2;
  A.eps = eps;
  A.step_dev = step_dev;
  A.sparse = sparse;
  return from_hip(launch_render_bwd_adam(V, n, *cfg, means, log_scales, quats, opacity_logits, sh,
                                         sh_degree, static_cast<const char*>(proj), ranges, vals,
                                         final_T, last_contrib, dL_dimage, A, d_mean2d_abs,
                                         capacity_pairs, ws, as_stream(stream)));
}
}  // namespace

gs_status gs_render_bwd_adam(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                             int32_t n, float* means, float* log_scales, float* quats,
                             float* opacity_logits, float* sh, int32_t sh_degree,
                             const void* proj, const uint32_t* ranges, const uint32_t* vals,
                             const float* final_T, const uint32_t* last_contrib,
                             const float* dL_dimage, float* const* m, float* const* v,
                             const float* lr, int32_t* step_dev, float beta1, float beta2,
                             float eps, float* d_mean2d_abs, int64_t capacity_pairs, void* ws,
                             size_t ws_bytes, void* stream) {
  return render_bwd_adam(n_views, cams, cfg, n, means, log_scales, quats, opacity_logits, sh,
                         sh_degree, proj, ranges, vals, final_T, last_contrib, dL_dimage, m, v, lr,
                         step_dev, beta1, beta2, eps, d_mean2d_abs, capacity_pairs, ws, ws_bytes,
                         stream, 0);
}

gs_status gs_render_bwd_sparse_adam(int32_t n_views, const gs_camera* cams,
                                    const gs_raster_cfg* cfg, int32_t n, float* means,
                                    float* log_scales, float* quats, float* opacity_logits,
                                    float* sh, int32_t sh_degree, const void* proj,
                                    const uint32_t* ranges, const uint32_t* vals,
                                    const float* final_T, const uint32_t* last_contrib,
                                    const float* dL_dimage, float* const* m, float* const* v,
                                    const float* lr, int32_t* step_dev, float beta1, float beta2,
                                    float eps, float* d_mean2d_abs, int64_t capacity_pairs,
                                    void* ws, size_t ws_bytes, void* stream) {
  return render_bwd_adam(n_views, cams, cfg, n, means, log_scales, quats, opacity_logits, sh,
                         sh_degree, proj, ranges, vals, final_T, last_contrib, dL_dimage, m, v, lr,
                         step_dev, beta1, beta2, eps, d_mean2d_abs, capacity_pairs, ws, ws_bytes,
                         stream, 1);
}

size_t gs_frequency_map_workspace_bytes(int32_t H, int32_t W) {
  if (H < 1 || W < 1 || H > kDftMax || W > kDftMax) return 0;
  return frequency_map_ws_bytes(H, W);
}

gs_status gs_frequency_map(int32_t n_images, int32_t H, int32_t W, const float* images,
                           double* mag, void* ws, size_t ws_bytes, void* stream) {
  if (n_images < 1 || H < 1 || W < 1 || H > kDftMax || W > kDftMax) return GS_ERR_ARG;
  if (!images || !mag || !ws) return GS_ERR_ARG;
  if (ws_bytes < frequency_map_ws_bytes(H, W)) return GS_ERR_CAPACITY;
  if (!aligned16(ws)) return GS_ERR_ARG;
  return from_hip(launch_frequency_map(n_images, H, W, images, mag, ws, as_stream(stream)));
}

gs_status gs_resolution_schedule(const double* mag_host, int32_t H, int32_t W, double S, double a,
                                 int32_t m, double r_max, int32_t per_pixel, double* r_knots,
                                 double* s_knots) {
  if (!mag_host || !r_knots || !s_knots || H < 1 || W < 1 || m < 1 || !(a > 1.0) || !(S > 0.0))
    return GS_ERR_ARG;
  if (r_max <= 0.0) r_max = double(H < W ? H : W);
  if (r_max < 1.0) return GS_ERR_ARG;
  resolution_schedule(mag_host, H, W, S, a, m, r_max, per_pixel, r_knots, s_knots, nullptr);
  return GS_OK;
}

double gs_schedule_resolution(double k, int32_t m, const double* r_knots, const double* s_knots) {
  if (!r_knots || !s_knots || m < 1) return 1.0;
  if (k >= s_knots[0]) return 1.0;
  for (int i = 1; i <= m; ++i) {
    if (k >= s_knots[i]) {
      const double t = (k - s_knots[i]) / (s_knots[i - 1] - s_knots[i]);
      const double a = 1.0 / (r_knots[i] * r_knots[i]), b = 1.0 / (r_knots[i - 1] * r_knots[i - 1]);
      return 1.0 / std::sqrt(a + t * (b - a));
    }
  }
  return r_knots[m];
}

gs_status gs_downsample_aa(int32_t n_planes, int32_t H, int32_t W, int32_t h, int32_t w,
                           const float* src, float* dst, void* stream) {
  if (n_planes < 0 || H < 1 || W < 1 || h < 1 || w < 1 || H > 16384 || W > 16384 || h > 16384 ||
      w > 16384)
    return GS_ERR_ARG;
  if (n_planes > 0 && (!src || !dst)) return GS_ERR_ARG;
  return from_hip(launch_downsample(n_planes, H, W, h, w, src, dst, as_stream(stream)));
}

double gs_primitive_target(double i, double S, double r, double p_init, double p_fin) {
  return p_init + (p_fin - p_init) / std::pow(r, 2.0 - i / S);
}

double gs_primitive_budget(double p_fin_prev, double p_add, double gamma, double eta) {
  const double x = gamma * p_fin_prev + eta * p_add;
  return x > p_fin_prev ? x : p_fin_prev;
}

size_t gs_densify_workspace_bytes(int32_t n) {
  return n < 0 || n >= kDensifyMaxN ? 0 : densify_ws_bytes(n);
}

gs_status gs_densify_stats(int32_t n_views, int32_t n, const void* proj,
                           const float* d_mean2d_abs, float scale, float* accum, float* count,
                           void* stream) {
  if (!n_ok(n_views, n)) return GS_ERR_ARG;
  if (n > 0 && (!proj || !d_mean2d_abs || !accum || !count || !aligned16(proj))) return GS_ERR_ARG;
  return from_hip(launch_densify_stats(n_views, n, static_cast<const char*>(proj), d_mean2d_abs,
                                       scale, accum, count, as_stream(stream)));
}

gs_status gs_densify_classify(int32_t n, const float* accum, const float* count,
                              const float* opacity_logits, float grad_thr, float min_opacity,
                              void* ws, size_t ws_bytes, int64_t* counts_dev, void* stream) {
  if (n < 0 || n >= kDensifyMaxN || !ws || !counts_dev ||
      (n > 0 && (!accum || !count || !opacity_logits)))
    return GS_ERR_ARG;
  if (ws_bytes < densify_ws_bytes(n)) return GS_ERR_CAPACITY;
  if (!aligned16(ws)) return GS_ERR_ARG;
  return from_hip(launch_densify_classify(n, accum, count, opacity_logits, grad_thr, min_opacity,
                                          ws, counts_dev, as_stream(stream)));
}

gs_status gs_densify_plan(int32_t n, int64_t k, int64_t n_candidates, const float* log_scales,
                          float max_scale, void* ws, size_t ws_bytes, int64_t* n_new_dev,
                          void* stream) {
  if (n < 0 || n >= kDensifyMaxN || n_candidates < 0 || n_candidates > n || !ws || !n_new_dev ||
      (n > 0 && !log_scales))
    return GS_ERR_ARG;
  if (ws_bytes < densify_ws_bytes(n)) return GS_ERR_CAPACITY;
  if (!aligned16(ws)) return GS_ERR_ARG;
  return from_hip(launch_densify_plan(n, k, n_candidates, log_scales, max_scale, ws, n_new_dev,
                                      as_stream(stream)));
}

gs_status gs_densify_apply(int32_t n, const float* const* params, const float* const* m,
                           const float* const* v, const float* z, const void* ws,
                           size_t ws_bytes, float* const* params_out, float* const* m_out,
                           float* const* v_out, void* stream) {
  if (n < 0 || n >= kDensifyMaxN || !params || !m || !v || !params_out || !m_out || !v_out ||
      !ws)
    return GS_ERR_ARG;
  if (n > 0 && !z) return GS_ERR_ARG;
  for (int t = 0; t < 5; ++t)
    if (n > 0 && (!params[t] || !m[t] || !v[t] || !params_out[t] || !m_out[t] || !v_out[t]))
      return GS_ERR_ARG;
  if (ws_bytes < densify_ws_bytes(n)) return GS_ERR_CAPACITY;
  return from_hip(launch_densify_apply(n, params, m, v, z, ws, params_out, m_out, v_out,
                                       as_stream(stream)));
}

gs_status gs_l1_loss_grad(int64_t numel, const float* image, const float* target, float scale,
                          float* dL_dimage, float* loss_sum, void* stream) {
  if (numel < 0 || (numel > 0 && (!image || !target || !dL_dimage))) return GS_ERR_ARG;
  return from_hip(launch_l1(numel, image, target, scale, dL_dimage, loss_sum, as_stream(stream)));
}

}  // extern "C"
