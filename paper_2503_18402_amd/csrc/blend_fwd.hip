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

// The L1 gradient of one pixel's three channels (elements e, e + plane,
// e + 2 plane), from the values just stored in the image; returns sum |d|.
__device__ __forceinline__ float l1_pixel(const L1Fuse& l1, int64_t e, int64_t plane, float c0,
                                          float c1, float c2) {
  const float* tgt = l1.index ? l1.target + int64_t(*l1.index) * l1.stride : l1.target;
  const float d0 = c0 - tgt[e], d1 = c1 - tgt[e + plane], d2 = c2 - tgt[e + 2 * plane];
  l1.dL[e] = l1_sign(d0, l1.scale);
  l1.dL[e + plane] = l1_sign(d1, l1.scale);
  l1.dL[e + 2 * plane] = l1_sign(d2, l1.scale);
  return (fabsf(d0) + fabsf(d1)) + fabsf(d2);
}

// scale * (the workgroup's sum of x) added to the loss with one atomic; every
// thread of the NW-wave workgroup calls it
template <int NW>
__device__ __forceinline__ void l1_block_add(const L1Fuse& l1, float x) {
  __shared__ float s_part[NW];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += s_part[w];
    atomicAdd(l1.loss, l1.scale * t);
  }
}

template <int TILE, int BATCH>
__global__ __launch_bounds__(WaveShape<TILE>::kThreads) void k_blend_fwd(
    RViews RV, const char* __restrict__ proj, size_t stride, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ vals, float* __restrict__ image, float* __restrict__ final_T,
    uint32_t* __restrict__ last_contrib, float bg0, float bg1, float bg2, int skip_long,
    L1Fuse l1) {
  using S = WaveShape<TILE>;
  constexpr int NT = S::kThreads, NW = S::kWaves, R = S::kRegion, SUB = S::kSub, P = S::kPix;
  __shared__ float4 s_r0[BATCH];
  __shared__ float4 s_r1[BATCH];
  __shared__ float s_b[BATCH];
  __shared__ uint32_t s_mask[BATCH];
  __shared__ uint16_t s_list[NW][BATCH];

  const int t = xcd_tile(blockIdx.x, RV);
  const int v = view_of_tile(RV, t);
  if (skip_long && ranges[2 * t + 1] - ranges[2 * t] > long_list_threshold<TILE>(RV, v)) return;
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
        const float aT = e.a * T[p];
        const float Tn = T[p] - aT;  // T (1 - alpha), reusing the weight's product
        const bool stop = ok & (Tn < kTMin);
        const bool blend = ok & !stop;
        const float wgt = blend ? aT : 0.0f;
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
  float l1_abs = 0.0f;
#pragma unroll
  for (int j = 0; j < SUB; ++j)
#pragma unroll
    for (int i = 0; i < SUB; ++i) {
      const int p = j * SUB + i;
      const int x = rx0 + i * 8 + lx, y = ry0 + j * 8 + ly;
      if (x < W && y < H) {
        const int64_t o = int64_t(y) * W + x;
        const float c0 = fmaf(T[p], bg0, C0[p]), c1 = fmaf(T[p], bg1, C1[p]),
                    c2 = fmaf(T[p], bg2, C2[p]);
        image[3 * pb + o] = c0;
        image[3 * pb + plane + o] = c1;
        image[3 * pb + 2 * plane + o] = c2;
        final_T[pb + o] = T[p];
        last_contrib[pb + o] = last[p];
        if (l1.target) l1_abs += l1_pixel(l1, 3 * pb + o, plane, c0, c1, c2);
      }
    }
  if (l1.loss) l1_block_add<NW>(l1, l1_abs);
}

// ---- long lists (low resolutions: few tiles, thousands of entries each): one
// block of kFWaves waves per tile, the list cut into nch <= kFMaxChunks chunks
// dealt to the waves; lane l owns pixel (l % 8, l / 8) of every 8x8 group.
// Transmittance only decreases along the list, so a pixel stops inside chunk
// k exactly when T entering k times the product of (1 - alpha) over k's
// entries falls below 1e-4:
//   A. per chunk and pixel, with no stopping: the product, the colour (T = 1
//      at the chunk start) and the last entry with alpha >= 1/255;
//   B. per pixel: the first chunk whose product takes T below 1e-4, and T and
//      colour entering it (or, if none, the final T, colour and last entry);
//   C. from that chunk on, the sequential front-to-back walk of the short
//      kernel until the pixel stops.
constexpr int kFWaves = 8;
constexpr int kFMaxChunks = 16;
constexpr uint32_t kFMinChunk = 32;
constexpr int kFBatch = 64;
constexpr int kFLongBlocks = 1024;

template <int TILE>
__device__ __forceinline__ void fwd_stage(float4* r0s, float4* r1s, float* bs, uint32_t* ms,
                                          uint32_t bstart, int nb, int lane,
                                          const uint32_t* __restrict__ vals, const float4* rec,
                                          int tx, int ty) {
  for (int k = lane; k < nb; k += 64) {
    const uint32_t g = vals[bstart + k];
    const float4 r0 = rec[3 * size_t(g)];
    const float4 r1 = rec[3 * size_t(g) + 1];
    const float4 r2 = rec[3 * size_t(g) + 2];
    const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
    r0s[k] = to_tile_frame<TILE>(r0, lo, tx, ty);
    r1s[k] = r1;
    bs[k] = r2.x;
    ms[k] = group_mask<TILE>(lo, hi, tx, ty);
  }
}

template <int TILE>
__global__ __launch_bounds__(64 * kFWaves) void k_blend_fwd_long(
    RViews RV, const char* __restrict__ proj, size_t stride, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ vals, float* __restrict__ image, float* __restrict__ final_T,
    uint32_t* __restrict__ last_contrib, float bg0, float bg1, float bg2, L1Fuse l1) {
  constexpr int GX = TileShape<TILE>::kGroupsX, Q = TileShape<TILE>::kGroups;
  __shared__ float4 s_r0[kFWaves][kFBatch];
  __shared__ float4 s_r1[kFWaves][kFBatch];
  __shared__ float s_b[kFWaves][kFBatch];
  __shared__ uint32_t s_mask[kFWaves][kFBatch];
  __shared__ float4 s_ch[kFMaxChunks][Q][64];    // A: (product, colour)
  __shared__ uint32_t s_lp[kFMaxChunks][Q][64];  // A: last entry with alpha >= 1/255
  __shared__ float4 s_st[Q][64];                 // B/C: (T, colour) of the pixel
  __shared__ uint32_t s_stop[Q][64];             // B: stop chunk + 1, 0 if none
  __shared__ uint32_t s_last[Q][64];             // B/C: last blended entry
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lx = lane & 7, ly = lane >> 3;
  const float px0 = float(lx) + 0.5f, py0 = float(ly) + 0.5f;
  float4* r0s = s_r0[wv];
  float4* r1s = s_r1[wv];
  float* bs = s_b[wv];
  uint32_t* ms = s_mask[wv];
  float l1_abs = 0.0f;  // over the block's tiles

  for (int t = blockIdx.x; t < RV.total_tiles; t += gridDim.x) {
    const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
    const int v = view_of_tile(RV, t);
    if (end - start <= long_list_threshold<TILE>(RV, v)) continue;  // block-uniform
    const int lt = t - RV.tile_base[v];
    const int gw = RV.gw[v], W = RV.W[v], H = RV.H[v];
    const int tx = lt % gw, ty = lt / gw;
    const uint32_t len = end - start;
    const uint32_t want = (len + kFMinChunk - 1) / kFMinChunk;
    const int nch = int(want < uint32_t(kFMaxChunks) ? want : uint32_t(kFMaxChunks));
    const uint32_t ch = (len + uint32_t(nch) - 1) / uint32_t(nch);
    const float4* rec = reinterpret_cast<const float4*>(proj + size_t(v) * stride);

    // A. per chunk, no stopping
    for (int c = wv; c < nch; c += kFWaves) {
      const uint32_t c0 = uint32_t(c) * ch, c1 = min(c0 + ch, len);
      float Pr[Q], C0[Q], C1[Q], C2[Q];
      uint32_t lp[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) Pr[q] = 1.0f, C0[q] = C1[q] = C2[q] = 0.0f, lp[q] = 0u;
      for (uint32_t b0 = c0; b0 < c1; b0 += kFBatch) {
        const int nb = int(min(c1 - b0, uint32_t(kFBatch)));
        fwd_stage<TILE>(r0s, r1s, bs, ms, start + b0, nb, lane, vals, rec, tx, ty);
        __builtin_amdgcn_wave_barrier();
        for (int k = 0; k < nb; ++k) {
          const uint32_t m = __builtin_amdgcn_readfirstlane(ms[k]);
          const float4 r0 = r0s[k], r1 = r1s[k];
          const float cb = bs[k];
          const uint32_t pos = b0 + uint32_t(k) + 1u;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            if (((m >> q) & 1u) == 0u) continue;  // wave-uniform: the box misses the group
            const Alpha e = alpha_at(r0, r1.x, r1.y, px0 + float((q % GX) * 8),
                                     py0 + float((q / GX) * 8));
            const float w = e.ok ? e.a * Pr[q] : 0.0f;
            C0[q] = fmaf(w, r1.z, C0[q]);
            C1[q] = fmaf(w, r1.w, C1[q]);
            C2[q] = fmaf(w, cb, C2[q]);
            Pr[q] = e.ok ? Pr[q] * (1.0f - e.a) : Pr[q];
            lp[q] = e.ok ? pos : lp[q];
          }
        }
        __builtin_amdgcn_wave_barrier();  // the staging is rewritten next
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        s_ch[c][q][lane] = make_float4(Pr[q], C0[q], C1[q], C2[q]);
        s_lp[c][q][lane] = lp[q];
      }
    }
    __syncthreads();
    // B. wave q handles pixel group q
    if (wv < Q) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (q != wv) continue;
        float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
        uint32_t last = 0u, stop = 0u;
        for (int c = 0; c < nch; ++c) {
          const float4 pc = s_ch[c][q][lane];
          if (T * pc.x < kTMin) {
            stop = uint32_t(c) + 1u;
            break;
          }
          C0 = fmaf(T, pc.y, C0);
          C1 = fmaf(T, pc.z, C1);
          C2 = fmaf(T, pc.w, C2);
          T *= pc.x;
          const uint32_t l = s_lp[c][q][lane];
          last = l ? l : last;
        }
        s_st[q][lane] = make_float4(T, C0, C1, C2);
        s_stop[q][lane] = stop;
        s_last[q][lane] = last;
      }
    }
    __syncthreads();
    // C. sequential walk from each pixel's stop chunk until it stops
    for (int c = wv; c < nch; c += kFWaves) {
      float T[Q], C0[Q], C1[Q], C2[Q];
      uint32_t last[Q];
      bool done[Q], mine[Q];
      bool any = false;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        mine[q] = s_stop[q][lane] == uint32_t(c) + 1u;
        const float4 st = s_st[q][lane];
        T[q] = st.x, C0[q] = st.y, C1[q] = st.z, C2[q] = st.w;
        last[q] = s_last[q][lane];
        done[q] = !mine[q];
        any |= mine[q];
      }
      if (__ballot(any) == 0ull) continue;
      for (uint32_t b0 = uint32_t(c) * ch; b0 < len; b0 += kFBatch) {
        bool alive = false;
#pragma unroll
        for (int q = 0; q < Q; ++q) alive |= !done[q];
        if (__ballot(alive) == 0ull) break;
        const int nb = int(min(len - b0, uint32_t(kFBatch)));
        fwd_stage<TILE>(r0s, r1s, bs, ms, start + b0, nb, lane, vals, rec, tx, ty);
        __builtin_amdgcn_wave_barrier();
        for (int k = 0; k < nb; ++k) {
          const uint32_t m = __builtin_amdgcn_readfirstlane(ms[k]);
          const float4 r0 = r0s[k], r1 = r1s[k];
          const float cb = bs[k];
          const uint32_t pos = b0 + uint32_t(k) + 1u;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            if (((m >> q) & 1u) == 0u) continue;
            const Alpha e = alpha_at(r0, r1.x, r1.y, px0 + float((q % GX) * 8),
                                     py0 + float((q / GX) * 8));
            const bool ok = e.ok & !done[q];
            const float aT = e.a * T[q];
            const float Tn = T[q] - aT;
            const bool stop = ok & (Tn < kTMin);
            const bool blend = ok & !stop;
            const float wgt = blend ? aT : 0.0f;
            C0[q] = fmaf(wgt, r1.z, C0[q]);
            C1[q] = fmaf(wgt, r1.w, C1[q]);
            C2[q] = fmaf(wgt, cb, C2[q]);
            T[q] = blend ? Tn : T[q];
            last[q] = blend ? pos : last[q];
            done[q] = done[q] | stop;
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (mine[q]) {
          s_st[q][lane] = make_float4(T[q], C0[q], C1[q], C2[q]);
          s_last[q][lane] = last[q];
        }
      }
    }
    __syncthreads();
    // outputs: wave q writes pixel group q
    if (wv < Q) {
      const int64_t pb = RV.pix_base[v];
      const int64_t plane = int64_t(W) * H;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (q != wv) continue;
        const int x = tx * TILE + (q % GX) * 8 + lx, y = ty * TILE + (q / GX) * 8 + ly;
        if (x < W && y < H) {
          const float4 st = s_st[q][lane];
          const int64_t o = int64_t(y) * W + x;
          const float c0 = fmaf(st.x, bg0, st.y), c1 = fmaf(st.x, bg1, st.z),
                      c2 = fmaf(st.x, bg2, st.w);
          image[3 * pb + o] = c0;
          image[3 * pb + plane + o] = c1;
          image[3 * pb + 2 * plane + o] = c2;
          final_T[pb + o] = st.x;
          last_contrib[pb + o] = s_last[q][lane];
          if (l1.target) l1_abs += l1_pixel(l1, 3 * pb + o, plane, c0, c1, c2);
        }
      }
    }
    __syncthreads();  // the block's next tile rewrites the LDS
  }
  if (l1.loss) l1_block_add<kFWaves>(l1, l1_abs);
}

template <int TILE>
hipError_t launch_tile(int batch, const RViews& RV, const char* proj, size_t stride,
                       const uint32_t* ranges, const uint32_t* vals, float* image,
                       float* final_T, uint32_t* last_contrib, const float* bg, const L1Fuse& l1,
                       hipStream_t st) {
  const dim3 grid(unsigned(RV.total_tiles)), block(WaveShape<TILE>::kThreads);
  // launches with few tiles hand long lists to the list-parallel kernel
  const int skip_long = split_long_lists(RV, TILE) ? 1 : 0;
  if (skip_long) {
    const unsigned nb = unsigned(RV.total_tiles < kFLongBlocks ? RV.total_tiles : kFLongBlocks);
    GS_LAUNCH("k_blend_fwd_long", HIP_KERNEL_NAME(k_blend_fwd_long<TILE <= 16 ? TILE : 16>),
              dim3(nb), dim3(64 * kFWaves), 0, st, RV, proj, stride, ranges, vals, image, final_T,
              last_contrib, bg[0], bg[1], bg[2], l1);
  }
  switch (batch) {
    case 128:
      GS_LAUNCH("k_blend_fwd", HIP_KERNEL_NAME(k_blend_fwd<TILE, 128>), grid, block, 0, st, RV, proj,
                         stride, ranges, vals, image, final_T, last_contrib, bg[0], bg[1], bg[2],
                         skip_long, l1);
      break;
    case 256:
      GS_LAUNCH("k_blend_fwd", HIP_KERNEL_NAME(k_blend_fwd<TILE, 256>), grid, block, 0, st, RV, proj,
                         stride, ranges, vals, image, final_T, last_contrib, bg[0], bg[1], bg[2],
                         skip_long, l1);
      break;
    default:
      GS_LAUNCH("k_blend_fwd", HIP_KERNEL_NAME(k_blend_fwd<TILE, 512>), grid, block, 0, st, RV, proj,
                         stride, ranges, vals, image, final_T, last_contrib, bg[0], bg[1], bg[2],
                         skip_long, l1);
      break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_render_fwd(const Views& V, int n, const gs_raster_cfg& cfg, const char* proj,
                             const uint32_t* ranges, const uint32_t* vals, float* image,
                             float* final_T, uint32_t* last_contrib, const L1Fuse& l1,
                             hipStream_t st) {
  if (V.total_tiles == 0) return hipSuccess;
  const RViews RV = make_rviews(V);
  const size_t stride = ProjLayout(n).stride;
  switch (cfg.tile) {
    case 8:
      return launch_tile<8>(cfg.lds_batch, RV, proj, stride, ranges, vals, image, final_T,
                            last_contrib, cfg.bg, l1, st);
    case 16:
      return launch_tile<16>(cfg.lds_batch, RV, proj, stride, ranges, vals, image, final_T,
                             last_contrib, cfg.bg, l1, st);
    default:
      return launch_tile<32>(cfg.lds_batch, RV, proj, stride, ranges, vals, image, final_T,
                             last_contrib, cfg.bg, l1, st);
  }
}

}  // namespace gsk
