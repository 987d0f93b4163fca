// Forward blend (Eq. 1): one workgroup per tile walks the tile's depth-sorted
// list front to back.  Batches of Gaussian records are staged in LDS by the
// whole workgroup; each 64-lane wave owns an 8x8 (or 16x16) square of the
// tile and compacts the batch to the Gaussians whose footprint box touches
// its square (ballot + popcount), so waves skip Gaussians that cannot reach
// their pixels.  (The backward runs one wave per tile instead; both share the
// float32 evaluation of alpha, so their decisions agree.)  A pixel stops at the first Gaussian that would take its
// transmittance below 1e-4; a wave leaves the list when all its pixels have
// stopped, the workgroup when all waves have.
#include "blend_common.hpp"

namespace gsk {
namespace {

template <int TILE, int BATCH>
__global__ __launch_bounds__(WaveShape<TILE>::kThreads) void k_blend_fwd(
    RViews RV, const char* __restrict__ proj, size_t stride, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ vals, float* __restrict__ image, float* __restrict__ final_T,
    uint32_t* __restrict__ last_contrib, float bg0, float bg1, float bg2) {
  using S = WaveShape<TILE>;
  constexpr int NT = S::kThreads, NW = S::kWaves, R = S::kRegion, SUB = S::kSub, P = S::kPix;
  __shared__ float4 s_r0[BATCH];
  __shared__ float4 s_r1[BATCH];
  __shared__ float s_b[BATCH];
  __shared__ uint32_t s_mask[BATCH];
  __shared__ uint16_t s_list[NW][BATCH];

  const int t = xcd_tile(blockIdx.x, RV);
  const int v = view_of_tile(RV, t);
  const int lt = t - RV.tile_base[v];
  const int gw = RV.gw[v], W = RV.W[v], H = RV.H[v];
  const int tx = lt % gw, ty = lt / gw;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wx = (NW == 1) ? 0 : (w & 1), wy = (NW == 1) ? 0 : (w >> 1);
  const int rx0 = tx * TILE + wx * R, ry0 = ty * TILE + wy * R;
  const int lx = lane & 7, ly = lane >> 3;
  const uint64_t ltmask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  float pxc[P], pyc[P], T[P], C0[P], C1[P], C2[P];
  uint32_t last[P];
  bool done[P];
#pragma unroll
  for (int j = 0; j < SUB; ++j)
#pragma unroll
    for (int i = 0; i < SUB; ++i) {
      const int p = j * SUB + i;
      const int x = rx0 + i * 8 + lx, y = ry0 + j * 8 + ly;
      pxc[p] = float(x - tx * TILE) + 0.5f;  // pixel centre in the tile's frame
      pyc[p] = float(y - ty * TILE) + 0.5f;
      T[p] = 1.0f;
      C0[p] = C1[p] = C2[p] = 0.0f;
      last[p] = 0;
      done[p] = !(x < W && y < H);
    }

  const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
  const float4* rec = reinterpret_cast<const float4*>(proj + size_t(v) * stride);

  for (uint32_t bstart = start; bstart < end; bstart += BATCH) {
    bool alive = false;
#pragma unroll
    for (int p = 0; p < P; ++p) alive |= !done[p];
    if (__syncthreads_count(alive) == 0) break;
    const int nb = int((end - bstart < uint32_t(BATCH)) ? (end - bstart) : uint32_t(BATCH));
    for (int k = tid; k < BATCH; k += NT) {
      uint32_t msk = 0;
      if (k < nb) {
        const uint32_t g = vals[bstart + k];
        const float4 r0 = rec[3 * size_t(g)];
        const float4 r1 = rec[3 * size_t(g) + 1];
        const float4 r2 = rec[3 * size_t(g) + 2];
        const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
        s_r0[k] = to_tile_frame<TILE>(r0, lo, tx, ty);
        s_r1[k] = r1;
        s_b[k] = r2.x;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
          const int x0 = tx * TILE + ((NW == 1) ? 0 : (ww & 1) * R);
          const int y0 = ty * TILE + ((NW == 1) ? 0 : (ww >> 1) * R);
          msk |= box_overlaps(lo, hi, x0, y0, x0 + R - 1, y0 + R - 1) ? (1u << ww) : 0u;
        }
      }
      s_mask[k] = msk;
    }
    __syncthreads();
    // this wave's list: the batch entries whose box touches its square, in order
    int cnt = 0;
    for (int c = 0; c < nb; c += 64) {
      const int k = c + lane;
      const bool m = (k < nb) && ((s_mask[k] >> w) & 1u);
      const uint64_t bal = __ballot(m);
      if (m) s_list[w][cnt + __popcll(bal & ltmask)] = uint16_t(k);
      cnt += __popcll(bal);
    }
    for (int q = 0; q < cnt; ++q) {
      const int k = s_list[w][q];
      const float4 r0 = s_r0[k];
      const float4 r1 = s_r1[k];
      const float cb = s_b[k];
      const uint32_t pos = bstart - start + uint32_t(k) + 1u;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        // branch-free: every lane computes, the decisions select the updates
        const Alpha e = alpha_at(r0, r1.x, r1.y, pxc[p], pyc[p]);
        const bool ok = e.ok & !done[p];
        if (__ballot(ok) == 0ull) continue;  // no pixel of this lane slot is reached
        const float Tn = T[p] * (1.0f - e.a);
        const bool stop = ok & (Tn < kTMin);
        const bool blend = ok & !stop;
        const float wgt = blend ? e.a * T[p] : 0.0f;
        C0[p] = fmaf(wgt, r1.z, C0[p]);
        C1[p] = fmaf(wgt, r1.w, C1[p]);
        C2[p] = fmaf(wgt, cb, C2[p]);
        T[p] = blend ? Tn : T[p];
        last[p] = blend ? pos : last[p];
        done[p] = done[p] | stop;
      }
      bool any = false;
#pragma unroll
      for (int p = 0; p < P; ++p) any |= !done[p];
      if (__ballot(any) == 0ull) break;
    }
    __syncthreads();
  }

  const int64_t pb = RV.pix_base[v];
  const int64_t plane = int64_t(W) * H;
#pragma unroll
  for (int j = 0; j < SUB; ++j)
#pragma unroll
    for (int i = 0; i < SUB; ++i) {
      const int p = j * SUB + i;
      const int x = rx0 + i * 8 + lx, y = ry0 + j * 8 + ly;
      if (x < W && y < H) {
        const int64_t o = int64_t(y) * W + x;
        image[3 * pb + o] = fmaf(T[p], bg0, C0[p]);
        image[3 * pb + plane + o] = fmaf(T[p], bg1, C1[p]);
        image[3 * pb + 2 * plane + o] = fmaf(T[p], bg2, C2[p]);
        final_T[pb + o] = T[p];
        last_contrib[pb + o] = last[p];
      }
    }
}

template <int TILE>
hipError_t launch_tile(int batch, const RViews& RV, const char* proj, size_t stride,
                       const uint32_t* ranges, const uint32_t* vals, float* image,
                       float* final_T, uint32_t* last_contrib, const float* bg, hipStream_t st) {
  const dim3 grid(unsigned(RV.total_tiles)), block(WaveShape<TILE>::kThreads);
  switch (batch) {
    case 128:
      GS_LAUNCH("k_blend_fwd", HIP_KERNEL_NAME(k_blend_fwd<TILE, 128>), grid, block, 0, st, RV, proj,
                         stride, ranges, vals, image, final_T, last_contrib, bg[0], bg[1], bg[2]);
      break;
    case 256:
      GS_LAUNCH("k_blend_fwd", HIP_KERNEL_NAME(k_blend_fwd<TILE, 256>), grid, block, 0, st, RV, proj,
                         stride, ranges, vals, image, final_T, last_contrib, bg[0], bg[1], bg[2]);
      break;
    default:
      GS_LAUNCH("k_blend_fwd", HIP_KERNEL_NAME(k_blend_fwd<TILE, 512>), grid, block, 0, st, RV, proj,
                         stride, ranges, vals, image, final_T, last_contrib, bg[0], bg[1], bg[2]);
      break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_render_fwd(const Views& V, int n, const gs_raster_cfg& cfg, const char* proj,
                             const uint32_t* ranges, const uint32_t* vals, float* image,
                             float* final_T, uint32_t* last_contrib, hipStream_t st) {
  if (V.total_tiles == 0) return hipSuccess;
  const RViews RV = make_rviews(V);
  const size_t stride = ProjLayout(n).stride;
  switch (cfg.tile) {
    case 8:
      return launch_tile<8>(cfg.lds_batch, RV, proj, stride, ranges, vals, image, final_T,
                            last_contrib, cfg.bg, st);
    case 16:
      return launch_tile<16>(cfg.lds_batch, RV, proj, stride, ranges, vals, image, final_T,
                             last_contrib, cfg.bg, st);
    default:
      return launch_tile<32>(cfg.lds_batch, RV, proj, stride, ranges, vals, image, final_T,
                             last_contrib, cfg.bg, st);
  }
}

}  // namespace gsk
