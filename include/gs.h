/*
 * gs.h -- C ABI of the MI355X (gfx950) differentiable tile-based Gaussian
 * rasterizer: the per-iteration hot path of 3DGS optimisation that
 * DashGaussian's resolution and primitive schedules make cheaper.
 *
 * The paper states the rendering model (Sec. 3, Eq. 1):
 *     C(u) = sum_i T_i(u) w_i(u) c_i,   T_i(u) = prod_{j<i} (1 - w_j(u)),
 *     w_i(u) = o_i G2D_i(u),
 * evaluated once per rendered pixel, back-propagated to the Gaussian
 * parameters, followed by a primitive (Adam) update (Sec. 1, Sec. 5.2).
 * Everything else below (EWA splatting, SH colour, 1/255 cutoff, 0.99 clamp,
 * T < 1e-4 exit, 16x16 tiles) is the rasterizer convention the paper relies
 * on without restating it.
 *
 * Common rules
 * ------------
 * - Every array pointer is a DEVICE pointer unless marked "host".  Arrays are
 *   FP32 (unless typed otherwise), contiguous, row-major.  The caller owns and
 *   allocates every buffer; the library allocates no device memory.
 * - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   Every call only enqueues work on `stream` and returns; none synchronises,
 *   so all of them may be captured into a HIP graph.
 * - Argument errors are reported synchronously through the return value and
 *   nothing is enqueued.  Device-side capacity overflow is reported through
 *   *n_pairs_dev > capacity_pairs (see gs_bin_sort).  NaN inputs are not
 *   checked; they propagate.
 * - Gaussians that fail a cull (depth <= near, det <= 0, opacity < 1/255, or a
 *   footprint outside the image) are dropped silently: no pairs, zero
 *   gradients.
 * - Several views per call (n_views > 1, at most GS_MAX_VIEWS, resolutions
 *   may differ) run as ONE launch per kernel over all views: the batched form.
 *   Per-view outputs are concatenated view after view.
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_MAX_VIEWS 32
#define GS_SH_COEFFS 16 /* sh arrays always hold 16 coefficients x 3 channels */

typedef enum {
  GS_OK = 0,
  GS_ERR_ARG = 1,         /* invalid argument; nothing was enqueued          */
  GS_ERR_CAPACITY = 2,    /* a workspace or capacity is too small           */
  GS_ERR_DEVICE = 3,      /* a HIP launch failed                            */
  GS_ERR_UNSUPPORTED = 4  /* valid request the library does not implement   */
} gs_status;

/* Pinhole camera.  x_cam = R x_world + t with OpenCV axes (x right, y down,
 * z forward); R is row-major.  Pixel (px, py) has its centre at
 * (px + 0.5, py + 0.5); mean2D = (fx x/z + cx, fy y/z + cy).  width and
 * height are in [1, 16384]; near_plane > 0 (0.2 in the conventions above). */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float near_plane;
} gs_camera;

/* Raster configuration.  tile in {8, 16, 32} pixels; lds_batch in
 * {128, 256, 512} Gaussians staged in LDS per step of the blend kernels;
 * bg is the background colour added as T_final * bg.  Binning is
 * result-neutral: the image does not depend on lds_batch, and across tile
 * sizes, or between a launch of fewer than 2048 tiles (which splits lists
 * longer than 48 entries across waves) and one of more, it changes only by
 * float32 rounding.
 *
 * Mip-Splatting's filters (the backbone family with an anti-aliased primitive
 * representation that the paper equips, Sec. 5 and the supplementary):
 *   mip2d 0: Sigma' = J W Sigma W^T J^T + 0.3 I, opacity unchanged (3DGS);
 *         1: the 2D mip filter, Sigma' = J W Sigma W^T J^T + 0.1 I with the
 *            opacity scaled by sqrt(det(Sigma' - 0.1 I) / det Sigma').
 *   filter3d: NULL, or device [n] per-Gaussian 3D filter variances f
 *         (gs_filter3d_variance): Sigma becomes Sigma + f I and the opacity is
 *         scaled by prod_i s_i / sqrt(s_i^2 + f).  Read by gs_preprocess and
 *         by the chain rule of the backward calls, which differentiate
 *         through both factors (f itself is a constant).
 * The scaled opacity is the one the cull (< 1/255), the footprint and Eq. 1
 * use.  Every call of one step must get the same cfg. */
typedef struct {
  int32_t tile;
  int32_t lds_batch;
  float bg[3];
  int32_t mip2d;
  const float* filter3d;
  /* Device-side step parameters, so that one captured HIP graph of a training
   * step replays for any view and learning rate (all NULL: not used):
   *   cam_table, cam_index: device gs_camera [k] and device int32 [1]; with
   *     both set (n_views must be 1, else GS_ERR_ARG), every call takes view
   *     0's pose and intrinsics (R, t, fx, fy, cx, cy, near_plane) from
   *     cam_table[*cam_index] when it runs, and cams[0] gives only width and
   *     height (every table entry must have that size).  gs_render_fwd_l1
   *     then reads its target at target + (*cam_index) * 3 * width * height:
   *     a stack of the table's views' targets.
   *   adam_lr: device float [6]: the fused backward + Adam calls take their
   *     learning rates from it instead of their host lr array. */
  const gs_camera* cam_table;
  const int32_t* cam_index;
  const float* adam_lr;
} gs_raster_cfg;

/* ---------------------------------------------------------------------------
 * gs_preprocess: 3D -> 2D splatting of every Gaussian into every view
 * (Sec. 3: G_i is splatted to G2D_i; colour c_i from SH coefficients).
 *   means [n,3], log_scales [n,3], quats [n,4] (w,x,y,z, need not be unit;
 *   16-byte aligned), opacity_logits [n], sh [n,16,3] (coefficient-major,
 *   16-byte aligned; only the first (sh_degree+1)^2 are read), sh_degree 0..3.
 *   cams: host array [n_views]; cfg: host.
 *   proj: output, gs_proj_bytes(n_views, n) bytes, opaque per-view records
 *   (screen mean, conic, opacity, colour, depth, footprint box, tile count,
 *   clamp flags), consumed by the calls below with the same n_views, cams,
 *   cfg and n.  0 <= n < 2^31 / n_views.
 * ------------------------------------------------------------------------- */
size_t gs_proj_bytes(int32_t n_views, int32_t n);
gs_status gs_preprocess(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                        int32_t n, const float* means, const float* log_scales,
                        const float* quats, const float* opacity_logits, const float* sh,
                        int32_t sh_degree, void* proj, void* stream);

/* ---------------------------------------------------------------------------
 * gs_bin_sort: one (tile, Gaussian) pair per tile of each Gaussian's
 * footprint, keyed key = (tile_id << 32) | bits(depth_f32), sorted ascending
 * and stably (equal keys keep ascending Gaussian index), then per-tile ranges.
 * With several views tile ids run view after view (view 0's tiles first).
 *   capacity_pairs: length of keys/vals (>= 0, < 2^32).
 *   ws: workspace of gs_bin_sort_workspace_bytes(...) bytes.
 *   keys [capacity] u64: may be NULL (the blend kernels need only vals).
 *   vals [capacity] u32: Gaussian index of each sorted pair.
 *   ranges [total_tiles, 2] u32: [start, end) into vals, [0,0) when empty;
 *     total_tiles = sum over views of ceil(W/tile) * ceil(H/tile).
 *   n_pairs_dev [1] i64: number of pairs, always written.  If it exceeds
 *     capacity_pairs, keys/vals/ranges are NOT valid: grow and call again.
 *   proj: the records of gs_preprocess; the call also writes into it, for
 *     gs_render_bwd, each (view, Gaussian)'s first pair position in index
 *     order (the exclusive prefix of the tile counts) and the pair total.
 * ------------------------------------------------------------------------- */
size_t gs_bin_sort_workspace_bytes(int32_t n_views, int32_t n, int64_t capacity_pairs);
gs_status gs_bin_sort(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                      int32_t n, void* proj, int64_t capacity_pairs, void* ws,
                      size_t ws_bytes, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                      int64_t* n_pairs_dev, void* stream);

/* gs_bin_sort_noalloc: gs_bin_sort for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same keys, values, ranges and pair count as
 * gs_bin_sort, with the workspace taken from a static device array of the
 * library instead of a `ws` argument.
 *   capacity_pairs: 0 .. GS_BIN_SORT_NOALLOC_MAX_PAIRS (2^22), and
 *   n_views * n: at most GS_BIN_SORT_NOALLOC_MAX_ITEMS (2^23); larger values
 *     return GS_ERR_CAPACITY and enqueue nothing.  The array holds 12 bytes
 *     per pair of that maximum plus 4 bytes per 256 items, 64 KiB of tile
 *     counters and 256 bytes (48.2 MiB) on every GPU the library runs on,
 *     until the process ends.
 *   The call allocates nothing (no hipMalloc, no hipFree).  Its first call on
 *   a device looks up that device's copy of the array with the device
 *   current; the current device must be the one `stream` belongs to.
 *   All calls on one GPU share its one array: calls that overlap on a GPU
 *   (several streams, several host threads) race and corrupt each other's
 *   results, so serialise them.  Nothing in the array needs clearing between
 *   calls: each call writes every byte of it that it reads.
 *   The other arguments, outputs and errors are those of gs_bin_sort. */
#define GS_BIN_SORT_NOALLOC_MAX_PAIRS (1 << 22)
#define GS_BIN_SORT_NOALLOC_MAX_ITEMS (1 << 23)
gs_status gs_bin_sort_noalloc(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                              int32_t n, void* proj, int64_t capacity_pairs,
                              uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                              int64_t* n_pairs_dev, void* stream);

/* ---------------------------------------------------------------------------
 * gs_filter3d_variance: Mip-Splatting's 3D smoothing filter.  For each
 * Gaussian, nu = the highest sampling rate fx / z over the views whose image
 * rectangle [0, W] x [0, H] contains its projected centre with z > near; the
 * variance is scale / nu^2 (scale 0.2 in Mip-Splatting).  Gaussians no view
 * sees take the largest variance of the seen ones (0 when none is seen).
 *   means [n,3]; variance [n] output; scratch: device uint32 [1] (overwritten).
 *   cams: host array [n_views] (the training views), n_views >= 1 (any number:
 *   they are taken in launches of GS_MAX_VIEWS).
 * ------------------------------------------------------------------------- */
gs_status gs_filter3d_variance(int32_t n_views, const gs_camera* cams, int32_t n,
                               const float* means, float scale, float* variance,
                               uint32_t* scratch, void* stream);

/* gs_bin_sort_radix: the same keys, values, ranges and pair count as
 * gs_bin_sort, by a stable LSD radix sort with 8-bit digits (the four depth
 * digits sorted on the visible Gaussians before the pairs are expanded, then
 * the tile digits on the pairs).  Arguments and errors are those of
 * gs_bin_sort, with its own workspace size. */
size_t gs_bin_sort_radix_workspace_bytes(int32_t n_views, int32_t n, int64_t capacity_pairs);
gs_status gs_bin_sort_radix(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                            int32_t n, void* proj, int64_t capacity_pairs, void* ws,
                            size_t ws_bytes, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                            int64_t* n_pairs_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Spatial storage order.  Nothing the calls above compute depends on the order
 * in which the Gaussians are stored, except the tie-break of exactly equal
 * depths, which follows the stored index.  Stored along a space-filling
 * curve, consecutive Gaussians sit close together in space, which the binning
 * (fewer global counter atomics), sparse Adam and the preprocess (long runs
 * of Gaussians outside a view) and the blends (fewer cache lines per tile
 * list) all profit from.
 *
 * gs_spatial_order: perm [n] u32 (device, output) = the Gaussians sorted by
 *   the Morton code of their means: per axis, the cell
 *   q = min(1023, floor((m - lo) * (1024 / (hi - lo)))) in the means'
 *   bounding box [lo, hi] (each operation rounded to float32 in that order;
 *   a flat axis gives cell 0), the ten bits of q_x, q_y, q_z interleaved (x
 *   lowest); ties keep ascending index.  perm[k] is the index of the k-th
 *   Gaussian in that order.  means [n,3] device.  ws: at least
 *   gs_spatial_order_workspace_bytes(n) bytes.  n >= 0.
 * gs_gather_rows: for each of n_arrays (<= 16) device arrays of n rows of
 *   row_floats[a] (1..64) floats, dst[a] row i = src[a] row perm[i]: applies
 *   the order to the parameters (and Adam moments).  src, dst, row_floats:
 *   host arrays of n_arrays entries; dst must not overlap src.  An entry
 *   perm[i] >= n leaves row i of every dst unwritten.
 * ------------------------------------------------------------------------- */
size_t gs_spatial_order_workspace_bytes(int32_t n);
gs_status gs_spatial_order(int32_t n, const float* means, void* ws, size_t ws_bytes,
                           uint32_t* perm, void* stream);
gs_status gs_gather_rows(int32_t n, const uint32_t* perm, int32_t n_arrays,
                         const float* const* src, float* const* dst, const int32_t* row_floats,
                         void* stream);

/* Total tiles over the views for this cfg (host helper for sizing ranges). */
int64_t gs_total_tiles(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg);

/* ---------------------------------------------------------------------------
 * gs_render_fwd: front-to-back blend of Eq. 1 for every pixel of every view.
 * Per pixel, over its tile's sorted list: alpha = min(0.99, o G2D(u)),
 * Gaussians with alpha < 1/255 are skipped, and the first Gaussian that would
 * take the transmittance below 1e-4 stops the pixel without being blended.
 *   image [3,H,W] per view, final_T [H,W] per view, last_contrib [H,W] per
 *   view (number of list entries up to and including the last blended one,
 *   0 if none), all concatenated over views.
 * ------------------------------------------------------------------------- */
gs_status gs_render_fwd(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                        int32_t n, const void* proj, const uint32_t* ranges,
                        const uint32_t* vals, float* image, float* final_T,
                        uint32_t* last_contrib, void* stream);

/* gs_render_fwd_l1: gs_render_fwd that also writes the L1 loss gradient of
 * gs_l1_loss_grad beside the image, from the same float values:
 *   dL_dimage[i] = scale * sign(image[i] - target[i])  (sign(0) = 0)
 * over every pixel of every view (target and dL_dimage have the image's
 * layout, device).  If loss_sum (device, [1]) is non-NULL, scale *
 * sum|image - target| is ADDED to it, one float atomic per workgroup (its last
 * bits depend on their order; image, final_T, last_contrib and dL_dimage are
 * bit-identical to gs_render_fwd followed by gs_l1_loss_grad).  It saves that
 * call's second pass over the image.  GS_ERR_ARG for a NULL target or
 * dL_dimage, otherwise as gs_render_fwd. */
gs_status gs_render_fwd_l1(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                           int32_t n, const void* proj, const uint32_t* ranges,
                           const uint32_t* vals, float* image, float* final_T,
                           uint32_t* last_contrib, const float* target, float scale,
                           float* dL_dimage, float* loss_sum, void* stream);

/* ---------------------------------------------------------------------------
 * gs_render_bwd: back-propagation of Eq. 1 to the Gaussian parameters
 * (Sec. 3: the process is differentiable and G_i is optimised from the loss).
 * Each pixel replays its list back to front from last_contrib, recovering
 * T_i = T_{i+1} / (1 - alpha_i) from final_T, so no per-pixel history is
 * stored.  Per (tile, Gaussian) gradients land in a deterministic per-pair
 * slot of the workspace (no float atomics); they are summed per Gaussian and
 * view, then chained to the 3D parameters and summed over views.
 *   Inputs: the parameters given to gs_preprocess, its proj as the binning
 *   left it (any gs_bin_sort* call records the pair offsets there), the
 *   ranges/vals of that binning (which must not have overflowed), the forward's final_T
 *   and last_contrib, and dL_dimage (same layout as image).
 *   Outputs: d_means [n,3], d_log_scales [n,3], d_quats [n,4] (16-byte
 *   aligned), d_opacity_logits [n], d_sh [n,16,3], d_mean2d_abs [n] (nullable:
 *   sum over views of |dL/dmean2D|, the densification statistic).  With
 *   accumulate != 0 they are ACCUMULATED (+=) and SH coefficients above
 *   sh_degree are untouched; with accumulate == 0 every element is written
 *   (=), zero where nothing contributes, including those coefficients.
 *   ws: gs_render_bwd_workspace_bytes(n_views, n, capacity_pairs) bytes.
 * ------------------------------------------------------------------------- */
size_t gs_render_bwd_workspace_bytes(int32_t n_views, int32_t n, int64_t capacity_pairs);
gs_status gs_render_bwd(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                        int32_t n, const float* means, const float* log_scales,
                        const float* quats, const float* opacity_logits, const float* sh,
                        int32_t sh_degree, const void* proj, const uint32_t* ranges,
                        const uint32_t* vals, const float* final_T,
                        const uint32_t* last_contrib, const float* dL_dimage, float* d_means,
                        float* d_log_scales, float* d_quats, float* d_opacity_logits,
                        float* d_sh, float* d_mean2d_abs, int32_t accumulate,
                        int64_t capacity_pairs, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * gs_adam_step: fused Adam over several parameter groups in one launch
 * (the primitive update, Sec. 1 / Sec. 5.2):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * groups: host array [n_groups], 1 <= n_groups <= GS_MAX_ADAM_GROUPS, each
 * with device p, g, m, v of numel elements (numel >= 0); step >= 1.
 * ------------------------------------------------------------------------- */
#define GS_MAX_ADAM_GROUPS 8
typedef struct {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t numel;
  float lr;
} gs_adam_group;
gs_status gs_adam_step(const gs_adam_group* groups, int32_t n_groups, int32_t step,
                       float beta1, float beta2, float eps, void* stream);

/* gs_adam_step_device: the same update with the 1-based step read from device
 * memory (*step_dev + 1 is this step) and *step_dev incremented afterwards on
 * the stream, so one captured HIP graph replays as successive steps.
 * step_dev: device int32, initialise to 0 before the first step. */
gs_status gs_adam_step_device(const gs_adam_group* groups, int32_t n_groups, int32_t* step_dev,
                              float beta1, float beta2, float eps, void* stream);

/* ---------------------------------------------------------------------------
 * gs_render_bwd_adam: gs_render_bwd in overwrite mode (accumulate = 0)
 * followed by gs_adam_step_device over the five parameter groups (means,
 * log_scales, quats, opacity_logits, sh), fused: each Gaussian's gradient
 * goes from the chain rule straight into its Adam update (the primitive
 * update after back-propagation, Sec. 1 and Sec. 3), so gradients are never
 * written to memory and the parameters are read once.  The updated
 * parameters, moments and counter equal those of the two separate calls bit
 * for bit: the same operations run in the same order.
 *   means, log_scales, quats, opacity_logits, sh: the parameters given to
 *     gs_preprocess (same layouts and alignment), updated in place.
 *   m, v: host arrays of 5 device pointers, the Adam moments of the five
 *     groups in the parameters' layouts (m[2], v[2], m[4], v[4] 16-byte
 *     aligned), updated in place.
 *   lr: host array of 6 learning rates: the five groups, except that lr[4]
 *     applies to the SH degree-0 coefficients (values 0..2 of a Gaussian's
 *     48) and lr[5] to the higher degrees.  lr[5] = lr[4] gives the update of
 *     gs_adam_step_device with one SH group.  May be NULL when cfg->adam_lr
 *     gives them on the device.
 *   step_dev: device int32 step counter (0 before the first step).  The call
 *     advances it by one on the stream, in the first kernel it launches,
 *     before any update, and takes step t = its new value; afterwards it
 *     equals the counter gs_adam_step_device leaves.  If a later launch of
 *     the call fails (GS_ERR_DEVICE), the counter may have advanced without
 *     an update.
 *   The other arguments are those of gs_render_bwd, with the same workspace.
 * ------------------------------------------------------------------------- */
gs_status gs_render_bwd_adam(int32_t n_views, const gs_camera* cams, const gs_raster_cfg* cfg,
                             int32_t n, float* means, float* log_scales, float* quats,
                             float* opacity_logits, float* sh, int32_t sh_degree,
                             const void* proj, const uint32_t* ranges, const uint32_t* vals,
                             const float* final_T, const uint32_t* last_contrib,
                             const float* dL_dimage, float* const* m, float* const* v,
                             const float* lr, int32_t* step_dev, float beta1, float beta2,
                             float eps, float* d_mean2d_abs, int64_t capacity_pairs, void* ws,
                             size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * gs_render_bwd_sparse_adam: gs_render_bwd_adam with the sparse (lazy) Adam of
 * the Taming backbone the paper equips (its headline configuration; the
 * per-iteration primitive update, Sec. 1): a Gaussian that has no pair in any
 * of the n_views views -- culled, behind the camera or off every image --
 * keeps its parameters and both moments unchanged; every other Gaussian takes
 * exactly the update of gs_render_bwd_adam, bias-corrected with the global
 * step t (the counter's value on entry plus one), even where its gradient is
 * zero.  The counter advances once per call, as in gs_render_bwd_adam.  d_mean2d_abs, when given, is written for every
 * Gaussian (0 for the untouched ones).  Arguments, layouts, alignment and
 * errors are those of gs_render_bwd_adam.
 * ------------------------------------------------------------------------- */
gs_status gs_render_bwd_sparse_adam(int32_t n_views, const gs_camera* cams,
                                    const gs_raster_cfg* cfg, int32_t n, float* means,
                                    float* log_scales, float* quats, float* opacity_logits,
                                    float* sh, int32_t sh_degree, const void* proj,
                                    const uint32_t* ranges, const uint32_t* vals,
                                    const float* final_T, const uint32_t* last_contrib,
                                    const float* dL_dimage, float* const* m, float* const* v,
                                    const float* lr, int32_t* step_dev, float beta1, float beta2,
                                    float eps, float* d_mean2d_abs, int64_t capacity_pairs,
                                    void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * The frequency-guided resolution schedule (Sec. 4.2, Eq. 2; supplementary
 * Eq. 6-7) and the anti-aliased ground-truth downsampling (supplementary,
 * "Ground Truth Downsampling").
 *
 * gs_frequency_map: mag[H][W] (device, FP64, natural DFT order: index (ky, kx)
 *   holds frequency (ky, kx) modulo (H, W)) = (1/n) sum over the n views of
 *   ||F^n(ky, kx)||_2, F^n the unnormalised 2D DFT of view n and the norm
 *   taken over the 3 colour channels (Eq. 2 before the sum over (ky, kx)).
 *   images: device [n][3][H][W] FP32, planar.  1 <= H, W <= 4096, n >= 1.
 *   Computed in FP64; deterministic.  ws: gs_frequency_map_workspace_bytes.
 * ------------------------------------------------------------------------- */
size_t gs_frequency_map_workspace_bytes(int32_t H, int32_t W);
gs_status gs_frequency_map(int32_t n_images, int32_t H, int32_t W, const float* images,
                           double* mag, void* ws, size_t ws_bytes, void* stream);

/* gs_resolution_schedule (host code, host arrays): the knots of the
 * resolution schedule for S iterations from a frequency map copied to the
 * host.  X(F_r) = c(r) * (sum of mag over |f_y| <= H/(2r), |f_x| <= W/(2r)),
 * the spectrum of the ideal downsample by r, with c(r) = 1/r^2 (Eq. 2 with
 * unnormalised DFTs, per_pixel = 0) or c = 1/(H W) (each view's DFT
 * normalised by its pixel count, per_pixel = 1).  For natural-image spectra
 * (amplitude ~ 1/f) the first gives r_m near a^(1/3), the second near a.  r_m is the largest r in
 * [1, r_max] with X(F_r) >= X(F)/a (r_max <= 0: min(H, W)); the values
 * X_i = X(F) - (i/m)(X(F) - X(F)/a), i = 1..m-1, are solved for r_i the same
 * way (bisection), and Eq. 7 gives s_i = S ln(X_i / X_m) / ln(X(F) / X_m).
 *   r_knots, s_knots: m + 1 entries each, knot 0 = (r 1, s S), knot m =
 *   (r_m, s 0).  m >= 1, a > 1, S > 0. */
gs_status gs_resolution_schedule(const double* mag_host, int32_t H, int32_t W, double S, double a,
                                 int32_t m, double r_max, int32_t per_pixel, double* r_knots,
                                 double* s_knots);

/* gs_schedule_resolution: r at iteration k for the knots above, 1/r^2 linear
 * in k between consecutive knots, 1 from s_0 = S on, r_m before s_m = 0.
 * The render uses the integer factor floor(r). */
double gs_schedule_resolution(double k, int32_t m, const double* r_knots, const double* s_knots);

/* gs_downsample_aa: [n_planes][H][W] -> [n_planes][h][w] (device, FP32)
 * anti-aliased linear resampling: output sample i is centred at input
 * coordinate (i + 0.5) * H / h (pixel centres at +0.5) and weighs the inputs
 * with a triangle of half-width max(1, H / h) input pixels, normalised to sum
 * 1; likewise along W.  1 <= h, H, w, W <= 16384. */
gs_status gs_downsample_aa(int32_t n_planes, int32_t H, int32_t W, int32_t h, int32_t w,
                           const float* src, float* dst, void* stream);

/* ---------------------------------------------------------------------------
 * The resolution-guided primitive schedule (Sec. 4.3, Eq. 4-5; supplementary
 * "Densification of DashGaussian").
 *
 * gs_primitive_target: Eq. 4, P_i = P_init + (P_fin - P_init) / r^(2 - i/S).
 * gs_primitive_budget: Eq. 5, max(P_fin, gamma P_fin + eta P_add).
 * (host arithmetic)
 *
 * A densification step is four calls; the caller reads two device counts in
 * between and allocates the outputs:
 *   gs_densify_stats (every iteration): accum[g] += scale * d_mean2d_abs[g] and
 *     count[g] += the number of views where g has a footprint (from proj),
 *     for Gaussians seen in at least one view.  accum, count: device [n].
 *   gs_densify_classify: score = accum / count (0 if count = 0, float32);
 *     prune where sigmoid(opacity_logit) < min_opacity; candidate where not
 *     pruned, count > 0 and score >= grad_thr.  counts_dev (device int64[2])
 *     receives (pruned, candidates).
 *   gs_densify_plan: selects the min(k, candidates) candidates of highest
 *     score (ties: lowest index; k <= 0 selects none), marks a selected one
 *     for a split when its largest exp(log_scale) exceeds max_scale (else a
 *     clone) and plans the output; *n_new_dev receives the new count.
 *   gs_densify_apply: writes the new parameter and moment arrays (n_new rows
 *     each; 5 groups in the order means, log_scales, quats, opacity_logits,
 *     sh).  In index order a pruned Gaussian writes nothing, a kept one itself
 *     (moments copied), a cloned one itself then an identical copy (moments
 *     zero), a split one two children at mu + R(q) diag(exp(log_scale)) z_j,
 *     log_scale - ln 1.6, other parameters copied, moments zero.
 *     z: device [n][2][3] standard normal samples.  Outputs must not alias
 *     inputs.
 *   ws: gs_densify_workspace_bytes(n), kept between the calls of one step.
 *   0 <= n < 2^30 (GS_ERR_ARG otherwise; the workspace size is then 0).
 * ------------------------------------------------------------------------- */
double gs_primitive_target(double i, double S, double r, double p_init, double p_fin);
double gs_primitive_budget(double p_fin_prev, double p_add, double gamma, double eta);
size_t gs_densify_workspace_bytes(int32_t n);
gs_status gs_densify_stats(int32_t n_views, int32_t n, const void* proj,
                           const float* d_mean2d_abs, float scale, float* accum, float* count,
                           void* stream);
gs_status gs_densify_classify(int32_t n, const float* accum, const float* count,
                              const float* opacity_logits, float grad_thr, float min_opacity,
                              void* ws, size_t ws_bytes, int64_t* counts_dev, void* stream);
gs_status gs_densify_plan(int32_t n, int64_t k, int64_t n_candidates, const float* log_scales,
                          float max_scale, void* ws, size_t ws_bytes, int64_t* n_new_dev,
                          void* stream);
gs_status gs_densify_apply(int32_t n, const float* const* params, const float* const* m,
                           const float* const* v, const float* z, const void* ws,
                           size_t ws_bytes, float* const* params_out, float* const* m_out,
                           float* const* v_out, void* stream);

/* ---------------------------------------------------------------------------
 * gs_l1_loss_grad: L1 photometric loss of the backbones.
 *   dL_dimage[i] = scale * sign(image[i] - target[i])  (sign(0) = 0), numel
 *   elements; if loss_sum (device, [1]) is non-NULL, scale * sum|image-target|
 *   is ADDED to it (one float atomic per workgroup: the last bits of this
 *   reported value depend on their order; the gradient does not).  scale =
 *   1/numel gives the mean.
 * ------------------------------------------------------------------------- */
gs_status gs_l1_loss_grad(int64_t numel, const float* image, const float* target, float scale,
                          float* dL_dimage, float* loss_sum, void* stream);

/* ---------------------------------------------------------------------------
 * Kernel timing (tracing aid, off by default).  While enabled, every kernel the
 * library launches is bracketed by two hipEventRecord calls on the stream it
 * is launched on.  gs_profile_collect waits for the recorded events, writes
 * per-kernel aggregates (host array of at most max_entries) and clears the
 * record; it returns the number of entries written, or -1 on a HIP error.
 * Not thread-safe: enable, run and collect from one host thread.
 * ------------------------------------------------------------------------- */
typedef struct {
  char name[48];     /* kernel name without template arguments */
  int64_t launches;  /* launches recorded                      */
  double total_ms;   /* summed event-to-event duration          */
} gs_kernel_time;
void gs_profile_enable(int32_t on);
int32_t gs_profile_collect(gs_kernel_time* out, int32_t max_entries);

const char* gs_status_str(gs_status s);
int32_t gs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GS_H */
