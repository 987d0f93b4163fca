// Internal definitions shared by the HIP kernels of the rasterizer library.
// Everything here is device-side layout and constants; the public C ABI is
// include/gs.h.
#pragma once

#include <utility>

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gs.h"

namespace gsk {

// ----------------------------------------------------------------- constants
// Rasterizer conventions (the paper's Eq. 1 plus its backbones' cutoffs).
constexpr float kAlphaMin = 1.0f / 255.0f;  // skip a Gaussian below this alpha
constexpr float kLog2AlphaMin = -7.99435343685885793771f;  // log2(1/255)
constexpr float kAlphaMax = 0.99f;          // alpha clamp
constexpr float kTMin = 1.0e-4f;            // stop a pixel before T drops below this
constexpr float kDilation = 0.3f;           // screen-space low-pass added to Sigma'
constexpr float kMip2d = 0.1f;              // the 2D mip filter's variance (Mip-Splatting)
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kExtRel = 1.0e-3f;          // widening of the footprint box (relative)
constexpr float kExtAbs = 1.0e-2f;          // and (pixels)

constexpr int kWave = 64;

// ------------------------------------------------------------ view table
// One entry per view, passed by value in kernel arguments (<= GS_MAX_VIEWS).
struct DevView {
  float R[9];
  float t[3];
  float campos[3];  // -R^T t, the camera centre in world space
  float fx, fy, cx, cy, near_plane;
  int32_t W, H, gw, gh;
  int32_t tile_base;   // global id of this view's first tile
  int32_t pad;
  int64_t pix_base;    // first pixel of this view in concatenated per-pixel arrays
};

struct Views {
  DevView v[GS_MAX_VIEWS];
  int32_t n_views;
  int32_t tile;
  int32_t total_tiles;
  int32_t mip2d;            // 1: the 2D mip filter instead of the dilation
  const float* filter3d;    // per-Gaussian 3D filter variances, or null
  const gs_camera* cam_table;  // with cam_index: view 0's camera, read when the kernel runs
  const int32_t* cam_index;
};

// View v's camera: the host-built entry, or (view 0 with a device camera
// table) the table's entry, with the camera centre -R^T t computed in double
// and rounded once, as the host does.  The entry is the same for every lane:
// its fields are moved to scalar registers so the lookup costs no VGPRs.
__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

__device__ inline DevView view_at(const Views& V, int v) {
  DevView d = V.v[v];
  if (V.cam_table) {
    const gs_camera& c = V.cam_table[__builtin_amdgcn_readfirstlane(*V.cam_index)];
#pragma unroll
    for (int k = 0; k < 9; ++k) d.R[k] = uniform_f(c.R[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) d.t[k] = uniform_f(c.t[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      d.campos[k] = uniform_f(float(-(double(c.R[k]) * c.t[0] + double(c.R[3 + k]) * c.t[1] +
                                      double(c.R[6 + k]) * c.t[2])));
    d.fx = uniform_f(c.fx);
    d.fy = uniform_f(c.fy);
    d.cx = uniform_f(c.cx);
    d.cy = uniform_f(c.cy);
    d.near_plane = uniform_f(c.near_plane);
  }
  return d;
}

// The 3D filter's opacity factor prod_i s_i / sqrt(s_i^2 + f) (1 for f = 0).
__device__ __forceinline__ float filter3d_coef(float s0, float s1, float s2, float f) {
  return (s0 * s1 * s2) / sqrtf((s0 * s0 + f) * (s1 * s1 + f) * (s2 * s2 + f));
}

// ----------------------------------------------------- projected records
// Per view, for each Gaussian g (all FP32 unless noted):
//   rec[3g+0] = (mx, my, A, B)       screen mean relative to the pixel origin of the
//                                     first tile of the footprint box (tile size of the
//                                     call); A = -a/2 log2e, B = -b log2e
//   rec[3g+1] = (C, lo, r, g)        C = -c/2 log2e; lo = log2(opacity); colour r, g
//   rec[3g+2] = (b, depth, lo, hi)   colour b; z_f32; pixel box as two u32
//                                     (x | y << 16) of its inclusive corners
//   tt[g]     u32 tiles touched (0: culled or off-screen)
//   flags[g]  u32 bit c: colour channel c was clamped at 0
// so that the exponent of G2D in base 2 is p2 = A dx^2 + B dx dy + C dy^2.

// Compact per-view raster info for the blend kernels.
constexpr int kXcds = 8;  // MI355X: workgroups are dealt to 8 XCDs round-robin

struct RViews {
  int32_t W[GS_MAX_VIEWS], H[GS_MAX_VIEWS], gw[GS_MAX_VIEWS], tile_base[GS_MAX_VIEWS];
  int64_t pix_base[GS_MAX_VIEWS];
  // Each XCD takes one contiguous share of every view's tiles (see xcd_tile),
  // walking the views in order[] (fewest tiles first: a low-resolution view's
  // tiles hold the longest lists, so they start first).  For the k-th view of
  // that order, xcd_off[x][k] = tiles XCD x takes from the views before it and
  // xcd_start[x][k] = first tile (within the view) of XCD x's share.
  int32_t order[GS_MAX_VIEWS];
  int32_t xcd_off[kXcds][GS_MAX_VIEWS + 1];
  int32_t xcd_start[kXcds][GS_MAX_VIEWS];
  int32_t n_views;
  int32_t total_tiles;
};

inline RViews make_rviews(const Views& V) {
  RViews r{};
  for (int k = 0; k < V.n_views; ++k) {
    r.W[k] = V.v[k].W;
    r.H[k] = V.v[k].H;
    r.gw[k] = V.v[k].gw;
    r.tile_base[k] = V.v[k].tile_base;
    r.pix_base[k] = V.v[k].pix_base;
  }
  r.n_views = V.n_views;
  r.total_tiles = V.total_tiles;
  // shares are tiles / 8 each; the tiles / 8 remainders of successive views are dealt
  // to the XCDs cyclically, so XCD x ends up with exactly as many tiles as blocks
  // b < total with b % 8 == x (the round-robin dispatch)
  for (int k = 0; k < V.n_views; ++k) r.order[k] = k;
  auto tiles_of = [&](int v) { return V.v[v].gw * V.v[v].gh; };
  for (int k = 1; k < V.n_views; ++k)  // stable insertion sort by tile count
    for (int j = k; j > 0 && tiles_of(r.order[j - 1]) > tiles_of(r.order[j]); --j)
      std::swap(r.order[j - 1], r.order[j]);
  int rot = 0;
  for (int x = 0; x < kXcds; ++x) r.xcd_off[x][0] = 0;
  for (int k = 0; k < V.n_views; ++k) {
    const int tiles = tiles_of(r.order[k]), q = tiles / kXcds, rem = tiles % kXcds;
    int start = 0;
    for (int x = 0; x < kXcds; ++x) {
      const int share = q + (((x - rot) & (kXcds - 1)) < rem ? 1 : 0);
      r.xcd_start[x][k] = start;
      r.xcd_off[x][k + 1] = r.xcd_off[x][k] + share;
      start += share;
    }
    rot = (rot + rem) & (kXcds - 1);
  }
  return r;
}

// ---- Adam (one element).  Shared by the standalone step and the step fused
// into the chain rule, so both produce the same bits.
struct AdamCoef {
  float b1, b2, eps, c1, c2;  // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
};

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr,
                                         const AdamCoef& A) {
  m = fmaf(A.b1, m, (1.0f - A.b1) * g);
  v = fmaf(A.b2, v, (1.0f - A.b2) * g * g);
  const float mh = m * A.c1;
  const float vh = v * A.c2;
  p -= lr * mh / (sqrtf(vh) + A.eps);
}

// bias corrections of step t = *step_dev + ahead (ahead = 1 before the count
// is advanced for this step, 0 after)
__device__ inline void adam_bias(const int32_t* step_dev, float b1, float b2, float& c1,
                                 float& c2, int ahead = 1) {
  const double t = double(*step_dev + ahead);
  c1 = float(1.0 / (1.0 - pow(double(b1), t)));
  c2 = float(1.0 / (1.0 - pow(double(b2), t)));
}

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Per view: the records, tiles touched and colour-clamp flags (written by the
// preprocess), then the index-order position of each item's first pair and,
// in view 0's copy, the pair total as int64 (both written by the binning,
// read by the backward).
struct ProjLayout {
  size_t rec, tt, flags, goff, total, stride;
  __host__ __device__ ProjLayout(int n) {
    rec = 0;
    tt = align256(size_t(n) * 48);
    flags = tt + align256(size_t(n) * 4);
    goff = flags + align256(size_t(n) * 4);
    total = goff + align256(size_t(n) * 4);
    stride = total + 256;
  }
};

__device__ inline uint32_t box_pack(int x, int y) { return uint32_t(x) | (uint32_t(y) << 16); }
__device__ inline int box_x(uint32_t b) { return int(b & 0xffffu); }
__device__ inline int box_y(uint32_t b) { return int(b >> 16); }

// ----------------------------------------------------------- launch helpers
inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Opt-in event tracing of kernel launches (abi.cpp): a scope records one event
// before and one after the launch it encloses, on the launch's stream.
extern bool g_profile_on;
void profile_begin(const char* name, hipStream_t st);
void profile_end(hipStream_t st);
struct ProfScope {
  hipStream_t st;
  bool on;
  ProfScope(const char* name, hipStream_t s) : st(s), on(g_profile_on) {
    if (on) profile_begin(name, st);
  }
  ~ProfScope() {
    if (on) profile_end(st);
  }
};
// Launch a kernel inside a tracing scope.
#define GS_LAUNCH(name, kernel, grid, block, shmem, st, ...)           \
  do {                                                                 \
    ::gsk::ProfScope gs_prof_scope_(name, st);                         \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(kernel), grid, block, shmem, st, __VA_ARGS__); \
  } while (0)

// host-side builders (abi.cpp)
bool build_views(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg, Views* out);

// kernels' host launchers (one per translation unit)
hipError_t launch_filter3d_rate(const Views& V, int n, int first, const float* means, float* nu,
                                hipStream_t st);
hipError_t launch_filter3d_var(int n, float scale, float* variance, uint32_t* scratch,
                               hipStream_t st);
hipError_t launch_preprocess(const Views& V, int n, int sh_degree, const float* means,
                             const float* log_scales, const float* quats,
                             const float* opacity_logits, const float* sh, char* proj,
                             hipStream_t st);

size_t bin_sort_ws_bytes(int n_views, int n, int64_t cap);
hipError_t launch_bin_sort(const Views& V, int n, char* proj, int64_t cap, void* ws,
                           uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                           int64_t* n_pairs_dev, hipStream_t st);
hipError_t launch_bin_sort_noalloc(const Views& V, int n, char* proj, int64_t cap,
                                   uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                                   int64_t* n_pairs_dev, hipStream_t st);
size_t bin_sort_radix_ws_bytes(int n_views, int n, int64_t cap);
hipError_t launch_bin_sort_radix(const Views& V, int n, char* proj, int64_t cap, void* ws,
                                 uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                                 int64_t* n_pairs_dev, hipStream_t st);

// One stable LSD radix pass over (key, value) u32 pairs on key bits
// [shift, shift + bits), bits <= 8 (radix_sort.hip).  n = *cnt.dev or cnt.host
// elements, at most max_n; hist holds radix_hist_words(max_n) u32,
// digit_total 256.
struct Count;
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      Count cnt, int64_t max_n, int shift, int bits, uint32_t* hist,
                      uint32_t* digit_total, hipStream_t st);
size_t radix_hist_words(int64_t max_n);

// spatial storage order (order.hip)
size_t spatial_order_ws_bytes(int n);
hipError_t launch_spatial_order(int n, const float* means, void* ws, uint32_t* perm,
                                hipStream_t st);
constexpr int kGatherMaxArrays = 16;
constexpr int kGatherMaxRow = 64;
hipError_t launch_gather_rows(int n, const uint32_t* perm, int n_arrays, const float* const* src,
                              float* const* dst, const int32_t* row_floats, hipStream_t st);

// L1 loss gradient of the backbones, dL = scale * sign(image - target) (sign(0) = 0).
__host__ __device__ __forceinline__ float l1_sign(float d, float scale) {
  return (d > 0.0f) ? scale : ((d < 0.0f) ? -scale : 0.0f);
}

// The same gradient written by the forward blend beside each image value it
// stores (the image layout); with `loss`, scale * sum |image - target| is added
// to it, one float atomic per workgroup.  target == nullptr: the forward only.
struct L1Fuse {
  const float* target;
  float* dL;
  float* loss;
  float scale;
  const int32_t* index;  // with a camera table: target += *index * stride
  int64_t stride;
};

hipError_t launch_render_fwd(const Views& V, int n, const gs_raster_cfg& cfg, const char* proj,
                             const uint32_t* ranges, const uint32_t* vals, float* image,
                             float* final_T, uint32_t* last_contrib, const L1Fuse& l1,
                             hipStream_t st);

size_t render_bwd_ws_bytes(int n_views, int n, int64_t cap);
hipError_t launch_render_bwd(const Views& V, int n, const gs_raster_cfg& cfg,
                             const float* means, const float* log_scales, const float* quats,
                             const float* opacity_logits, const float* sh, int sh_degree,
                             const char* proj, const uint32_t* ranges, const uint32_t* vals,
                             const float* final_T, const uint32_t* last_contrib,
                             const float* dL_dimage, float* d_means, float* d_log_scales,
                             float* d_quats, float* d_opacity_logits, float* d_sh,
                             float* d_mean2d_abs, int accumulate, int64_t cap, void* ws,
                             hipStream_t st);

struct FusedAdam {  // the five parameter groups' moments and learning rates
  float* m[5];
  float* v[5];
  float lr[6];  // lr[4]: SH degree-0 coefficients, lr[5]: the higher degrees
  const float* lr_dev;  // device [6] learning rates, read instead of lr when set
  float b1, b2, eps;
  int32_t* step_dev;
  int sparse;  // 1: leave Gaussians with no pair in any view untouched (sparse Adam)
};
hipError_t launch_render_bwd_adam(const Views& V, int n, const gs_raster_cfg& cfg, float* means,
                                  float* log_scales, float* quats, float* opacity_logits,
                                  float* sh, int sh_degree, const char* proj,
                                  const uint32_t* ranges, const uint32_t* vals,
                                  const float* final_T, const uint32_t* last_contrib,
                                  const float* dL_dimage, const FusedAdam& A,
                                  float* d_mean2d_abs, int64_t cap, void* ws, hipStream_t st);

hipError_t launch_step_inc(int32_t* step_dev, hipStream_t st);

// densification (densify.hip); output rows are indexed in 32 bits with the
// source index packed beside two kind bits, so n < 2^30
constexpr int32_t kDensifyMaxN = 1 << 30;
size_t densify_ws_bytes(int n);
hipError_t launch_densify_stats(int n_views, int n, const char* proj, const float* mean2d_abs,
                                float scale, float* accum, float* count, hipStream_t st);
hipError_t launch_densify_classify(int n, const float* accum, const float* count,
                                   const float* opacity_logits, float thr, float min_opacity,
                                   void* ws, int64_t* counts_out, hipStream_t st);
hipError_t launch_densify_plan(int n, int64_t k, int64_t n_cand, const float* log_scales,
                               float max_scale, void* ws, int64_t* n_new, hipStream_t st);
hipError_t launch_densify_apply(int n, const float* const* p, const float* const* m,
                                const float* const* v, const float* z, const void* ws,
                                float* const* po, float* const* mo, float* const* vo,
                                hipStream_t st);

// resolution schedule (schedule.hip)
constexpr int kDftMax = 4096;  // largest image side for the frequency map
size_t frequency_map_ws_bytes(int H, int W);
hipError_t launch_frequency_map(int n_images, int H, int W, const float* images, double* mag,
                                void* ws, hipStream_t st);
hipError_t launch_downsample(int n_planes, int H, int W, int h, int w, const float* src, float* dst,
                             hipStream_t st);
void resolution_schedule(const double* mag, int H, int W, double S, double a, int m, double r_max,
                         int per_pixel, double* r_knots, double* s_knots, double* x_knots);
hipError_t launch_adam(const gs_adam_group* groups, int n_groups, int step, float beta1,
                       float beta2, float eps, int32_t* step_dev, hipStream_t st);
hipError_t launch_l1(int64_t numel, const float* image, const float* target, float scale,
                     float* dL, float* loss_sum, hipStream_t st);

}  // namespace gsk
