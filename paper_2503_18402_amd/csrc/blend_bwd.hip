// Backward of Eq. 1 and the chain rule to the Gaussian parameters.
//
// k_blend_bwd: one workgroup per tile replays the tile's list back to front
// in LDS-staged batches.  Each pixel starts at its own last contributor with
// T = final_T and recovers T_i = T_{i+1} / (1 - alpha_i); the colour behind a
// Gaussian is carried as its dot product with dL/dC.  Per (tile, Gaussian) nine
// 2D terms (the two offset sums sum dL/dpower * (dx, dy), whose product with
// the conic is the mean2D gradient, then conic a/b/c, opacity, rgb) are summed
// over the tile's pixels in a fixed order (wave butterfly, then waves in order)
// and written to that pair's own slot: the pair slots of a Gaussian are
// contiguous (ordered by Gaussian index, then by tile inside its footprint),
// so no float atomics are needed and gradients are bit-reproducible.
//
// k_chain: one thread per Gaussian sums its pair slots per view and chains the
// 2D gradients through the EWA projection, the covariance, the quaternion,
// the sigmoid and the SH colour back to the parameters, accumulating over
// views in registers before one read-modify-write of the outputs.
#include "blend_common.hpp"

namespace gsk {
namespace {

constexpr int kG = 9;  // 2D gradient components per (tile, Gaussian)

// ---- wave-wide sums of the nine gradient components, registers only.
// Halving transposes: a 32-lane swap (v_permlane32_swap) pairs each value with
// its partner half-wave, a 16-lane swap (v_permlane16_swap) pairs rows, and a
// DPP prefix over each 16-lane row finishes.  Afterwards lane 16 r + 15 of
// q[0] holds component kRow0[r], of q[1] component kRow1[r], of q[2] (rows 0, 1)
// component 8.  About 30 VALU instructions for all nine sums, in a fixed order.
template <int N>
__device__ __forceinline__ float row_shr(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + N, 0xF, 0xF,
                                                    true));
}
__device__ __forceinline__ float row_sum16(float x) {
  x += row_shr<1>(x);
  x += row_shr<2>(x);
  x += row_shr<4>(x);
  x += row_shr<8>(x);
  return x;
}
__device__ __forceinline__ float swap32_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ void wave_sum9(const float* v, float* q) {
  const float r01 = swap32_add(v[0], v[1]);  // lanes 0-31: v0, 32-63: v1 (pair sums)
  const float r23 = swap32_add(v[2], v[3]);
  const float r45 = swap32_add(v[4], v[5]);
  const float r67 = swap32_add(v[6], v[7]);
  const float r8 = swap32_add(v[8], 0.0f);   // lanes 0-31: v8, 32-63: 0
  q[0] = row_sum16(swap16_add(r01, r23));     // rows: v0, v2, v1, v3
  q[1] = row_sum16(swap16_add(r45, r67));     // rows: v4, v6, v5, v7
  q[2] = row_sum16(swap16_add(r8, r8));       // rows: v8, v8, 0, 0
}

// ---- one wave's walk over a tile's list, shared by the short- and the
// long-list kernels.  The wave's 64 lanes own the tile's pixels (lane l: pixel
// (l % 8, l / 8) of every 8x8 group); per pixel it carries T, dL/dC and the
// colour behind the current entry dotted with dL/dC.
template <int TILE>
struct BwdPix {
  static constexpr int Q = TileShape<TILE>::kGroups;
  float T[Q], g0[Q], g1[Q], g2[Q], SdL[Q];
  uint32_t last[Q];
  uint32_t glast[Q];  // per group: the largest last contributor (wave-uniform)
  uint32_t mylast;    // over the tile (wave-uniform)
};

// load final_T, last_contrib and dL/dC of the tile's pixels; SdL starts at
// T_final * (bg . dL/dC)
template <int TILE>
__device__ __forceinline__ void bwd_load_pixels(BwdPix<TILE>& P, const RViews& RV, int v, int tx,
                                                int ty, int lane, const float* __restrict__ final_T,
                                                const uint32_t* __restrict__ last_contrib,
                                                const float* __restrict__ dL_dimage, float bg0,
                                                float bg1, float bg2) {
  constexpr int GX = TileShape<TILE>::kGroupsX, Q = TileShape<TILE>::kGroups;
  const int lx = lane & 7, ly = lane >> 3;
  const int W = RV.W[v], H = RV.H[v];
  const int64_t pb = RV.pix_base[v];
  const int64_t plane = int64_t(W) * H;
  P.mylast = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int x = tx * TILE + (q % GX) * 8 + lx, y = ty * TILE + (q / GX) * 8 + ly;
    // pixels past the image edge load pixel 0 and are neutralised by selects
    // (conditional stores into the arrays would keep them in scratch memory)
    const bool in = (x < W) & (y < H);
    const int64_t o = in ? int64_t(y) * W + x : 0;
    const float ft = final_T[pb + o];
    const uint32_t lc = last_contrib[pb + o];
    const float d0 = dL_dimage[3 * pb + o], d1 = dL_dimage[3 * pb + plane + o],
                d2 = dL_dimage[3 * pb + 2 * plane + o];
    P.T[q] = in ? ft : 1.0f;
    P.last[q] = in ? lc : 0u;
    P.g0[q] = in ? d0 : 0.0f;
    P.g1[q] = in ? d1 : 0.0f;
    P.g2[q] = in ? d2 : 0.0f;
    P.SdL[q] = P.T[q] * fmaf(bg0, P.g0[q], fmaf(bg1, P.g1[q], bg2 * P.g2[q]));
    uint32_t mx = P.last[q];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mx = max(mx, uint32_t(__shfl_xor(int(mx), d, 64)));
    P.glast[q] = __builtin_amdgcn_readfirstlane(mx);
    P.mylast = max(P.mylast, P.glast[q]);
  }
}

// one wave's LDS staging of list entries: record in the tile frame, box mask,
// and the entry's per-pair gradient slot
struct BwdStage {
  float4* r0;
  float4* r1;
  float* b;
  uint32_t* mask;
  uint32_t* pidx;
};

template <int TILE>
__device__ __forceinline__ void bwd_stage(const BwdStage& S, uint32_t bstart, int nb, int lane,
                                          const uint32_t* __restrict__ vals, const float4* rec,
                                          const uint32_t* goff, int tx, int ty) {
  for (int k = lane; k < nb; k += 64) {
    const uint32_t g = vals[bstart + k];
    const float4 r0 = rec[3 * size_t(g)];
    const float4 r1 = rec[3 * size_t(g) + 1];
    const float4 r2 = rec[3 * size_t(g) + 2];
    const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
    S.r0[k] = to_tile_frame<TILE>(r0, lo, tx, ty);
    S.r1[k] = r1;
    S.b[k] = r2.x;
    S.mask[k] = group_mask<TILE>(lo, hi, tx, ty);
    const int tx0 = box_x(lo) / TILE, ty0 = box_y(lo) / TILE, tx1 = box_x(hi) / TILE;
    S.pidx[k] = goff[g] + uint32_t((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0));
  }
}

// The backward step of staged entry k at list position pos (1-based) for every
// pixel of the wave: recover T_i, accumulate the nine 2D gradients, reduce
// them over the wave and write the pair's slot.
template <int TILE>
__device__ __forceinline__ void bwd_step(BwdPix<TILE>& P, const BwdStage& S, int k, uint32_t pos,
                                         int lane, float px0, float py0,
                                         float* __restrict__ pair_grad, int64_t cap) {
  constexpr int GX = TileShape<TILE>::kGroupsX, Q = TileShape<TILE>::kGroups;
  uint32_t m = __builtin_amdgcn_readfirstlane(S.mask[k]);
#pragma unroll
  for (int q = 0; q < Q; ++q)
    if (pos > P.glast[q]) m &= ~(1u << q);
  if (m == 0u) return;
  const float4 r0 = S.r0[k];
  const float4 r1 = S.r1[k];
  const float cb = S.b[k];
  const float lo = r1.y;  // log2 of the blending opacity
  // -0 is the identity of float addition (+0 is not: +0 + -0 = +0), so the
  // first group's products need no add
  float acc[kG];
#pragma unroll
  for (int c = 0; c < kG; ++c) acc[c] = -0.0f;
  bool hit = false;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if ((m >> q) & 1u) {
      // branch-free: every lane computes, the decisions select the updates
      const float px = px0 + float((q % GX) * 8), py = py0 + float((q / GX) * 8);
      const Alpha e = alpha_at(r0, r1.x, lo, px, py);
      const bool ok = e.ok & (pos <= P.last[q]);
      // footprint boxes are conservative: often no pixel of the group is reached
      if (__ballot(ok) == 0ull) continue;
      const bool grad = ok & (e.raw <= kAlphaMax);  // the 0.99 clamp passes no gradient
      hit = true;
      const float inv = __builtin_amdgcn_rcpf(1.0f - e.a);
      const float Ti = P.T[q] * inv;
      const float wgt = ok ? e.a * Ti : 0.0f;
      const float cg = fmaf(r1.z, P.g0[q], fmaf(r1.w, P.g1[q], cb * P.g2[q]));
      const float dLda = grad ? fmaf(P.T[q], cg, -P.SdL[q]) * inv : 0.0f;  // (T cg - SdL) / (1 - a)
      P.SdL[q] = fmaf(wgt, cg, P.SdL[q]);
      P.T[q] = ok ? Ti : P.T[q];
      acc[6] = fmaf(wgt, P.g0[q], acc[6]);
      acc[7] = fmaf(wgt, P.g1[q], acc[7]);
      acc[8] = fmaf(wgt, P.g2[q], acc[8]);
      const float dpow = dLda * e.raw;
      acc[5] += dpow;  // dL/do times o: the chain rule divides by the opacity
      const float dpx = dpow * e.dx, dpy = dpow * e.dy;
      acc[2] = fmaf(dpx, e.dx, acc[2]);
      acc[3] = fmaf(dpx, e.dy, acc[3]);
      acc[4] = fmaf(dpy, e.dy, acc[4]);
      // the offsets weighted by dpow; the mean gradient is these two sums
      // times the Gaussian's conic, applied once in the chain rule
      acc[0] += dpx;
      acc[1] += dpy;
    }
  }
  if (hit) {  // wave-uniform
    float qv[3];
    wave_sum9(acc, qv);
    const uint32_t idx = S.pidx[k];
    if ((lane & 15) == 15 && int64_t(idx) < cap) {
      // natural-unit conic gradients from the base-2 accumulators; the offset
      // sums (0, 1) are stored as they are
      // scales of components (0..3) and (4..7): 1, 1, -1/2, -1 and -1/2, 1, 1, 1
      const int row = lane >> 4;
      const int c0 = ((row & 1) << 1) | (row >> 1);  // 0, 2, 1, 3
      const float s0 = c0 < 2 ? 1.0f : (c0 == 2 ? -0.5f : -1.0f);
      const float s1 = c0 == 0 ? -0.5f : 1.0f;
      float* dst = pair_grad + size_t(idx) * kG;
      dst[c0] = s0 * qv[0];
      dst[c0 + 4] = s1 * qv[1];
      if (row == 0) dst[8] = qv[2];
    }
  }
}



// One 64-lane wave per tile walks the list back to front in LDS-staged batches.
// With `skip_long`, tiles whose list is longer than their view's threshold are
// left to k_blend_bwd_long.
template <int TILE, int BATCH>
__global__ __launch_bounds__(64) void k_blend_bwd(
    RViews RV, int n, const char* __restrict__ proj, size_t stride,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float* __restrict__ final_T, const uint32_t* __restrict__ last_contrib,
    const float* __restrict__ dL_dimage, size_t goff_off,
    float* __restrict__ pair_grad, int64_t cap, float bg0, float bg1, float bg2, int skip_long,
    const uint32_t* __restrict__ order) {
  __shared__ float4 s_r0[BATCH];
  __shared__ float4 s_r1[BATCH];
  __shared__ float s_b[BATCH];
  __shared__ uint32_t s_mask[BATCH];
  __shared__ uint32_t s_pidx[BATCH];
  const BwdStage S{s_r0, s_r1, s_b, s_mask, s_pidx};

  const int t = order ? int(order[blockIdx.x]) : xcd_tile(blockIdx.x, RV);
  const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
  const int v = view_of_tile(RV, t);
  if (skip_long && end - start > long_list_threshold<TILE>(RV, v)) return;
  const int lt = t - RV.tile_base[v];
  const int gw = RV.gw[v];
  const int tx = lt % gw, ty = lt / gw;
  const int lane = threadIdx.x;
  BwdPix<TILE> P;
  bwd_load_pixels<TILE>(P, RV, v, tx, ty, lane, final_T, last_contrib, dL_dimage, bg0, bg1, bg2);
  const uint32_t stop = min(start + P.mylast, end);
  const float4* rec = reinterpret_cast<const float4*>(proj + size_t(v) * stride);
  const uint32_t* goff = reinterpret_cast<const uint32_t*>(proj + size_t(v) * stride + goff_off);
  const float px0 = float(lane & 7) + 0.5f, py0 = float(lane >> 3) + 0.5f;

  for (uint32_t bend = stop; bend > start;) {
    const uint32_t bstart = (bend - start > uint32_t(BATCH)) ? bend - BATCH : start;
    const int nb = int(bend - bstart);
    __syncthreads();  // the previous batch is consumed
    bwd_stage<TILE>(S, bstart, nb, lane, vals, rec, goff, tx, ty);
    __syncthreads();
    for (int k = nb - 1; k >= 0; --k)
      bwd_step<TILE>(P, S, k, bstart - start + uint32_t(k) + 1u, lane, px0, py0, pair_grad, cap);
    bend = bstart;
  }
}

// ---- long lists (low resolutions: few tiles, thousands of entries each): one
// block of kLongWaves waves per tile, the list cut into nch <= kMaxChunks
// chunks dealt to the waves.  Which entries a pixel blends is fixed by the
// forward's last_contrib and the alpha test alone, so the chunks are
// independent:
//   A. each chunk's transmittance product and colour (front to back, T = 1 at
//      its start) per pixel;
//   B. per pixel, the transmittance after each chunk (prefix of the products)
//      and the colour behind it dotted with dL/dC (suffix of the chunk
//      colours, weighted by their incoming T, plus T_final (bg . dL/dC));
//   C. each chunk's backward walk from that state, as in k_blend_bwd.
// The T recovery by division therefore runs over at most one chunk.
constexpr int kLongWaves = 8;
constexpr int kMaxChunks = 16;
constexpr uint32_t kMinChunk = 32;
constexpr int kLongBatch = 64;
constexpr int kLongBlocks = 1024;

template <int TILE>
__global__ __launch_bounds__(64 * kLongWaves) void k_blend_bwd_long(
    RViews RV, int n, const char* __restrict__ proj, size_t stride,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const float* __restrict__ final_T, const uint32_t* __restrict__ last_contrib,
    const float* __restrict__ dL_dimage, size_t goff_off,
    float* __restrict__ pair_grad, int64_t cap, float bg0, float bg1, float bg2) {
  constexpr int GX = TileShape<TILE>::kGroupsX, Q = TileShape<TILE>::kGroups;
  __shared__ float4 s_r0[kLongWaves][kLongBatch];
  __shared__ float4 s_r1[kLongWaves][kLongBatch];
  __shared__ float s_b[kLongWaves][kLongBatch];
  __shared__ uint32_t s_mask[kLongWaves][kLongBatch];
  __shared__ uint32_t s_pidx[kLongWaves][kLongBatch];
  // per chunk and pixel: (product, colour) after pass A, (T after, SdL after) after B
  __shared__ float4 s_ch[kMaxChunks][Q][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const BwdStage S{s_r0[wv], s_r1[wv], s_b[wv], s_mask[wv], s_pidx[wv]};
  const float px0 = float(lane & 7) + 0.5f, py0 = float(lane >> 3) + 0.5f;

  for (int t = blockIdx.x; t < RV.total_tiles; t += gridDim.x) {
    const uint32_t start = ranges[2 * t], end = ranges[2 * t + 1];
    const int v = view_of_tile(RV, t);
    if (end - start <= long_list_threshold<TILE>(RV, v)) continue;  // block-uniform
    const int lt = t - RV.tile_base[v];
    const int gw = RV.gw[v];
    const int tx = lt % gw, ty = lt / gw;
    BwdPix<TILE> P;
    bwd_load_pixels<TILE>(P, RV, v, tx, ty, lane, final_T, last_contrib, dL_dimage, bg0, bg1,
                          bg2);
    const uint32_t len = min(P.mylast, end - start);  // entries anyone blends
    const uint32_t want = (len + kMinChunk - 1) / kMinChunk;
    const int nch = int(want < uint32_t(kMaxChunks) ? want : uint32_t(kMaxChunks));
    const uint32_t ch = nch > 0 ? (len + uint32_t(nch) - 1) / uint32_t(nch) : 0u;
    const float4* rec = reinterpret_cast<const float4*>(proj + size_t(v) * stride);
    const uint32_t* goff =
        reinterpret_cast<const uint32_t*>(proj + size_t(v) * stride + goff_off);

    // A. per chunk: product of (1 - alpha) and colour over the blended entries
    for (int c = wv; c < nch; c += kLongWaves) {
      const uint32_t c0 = uint32_t(c) * ch, c1 = min(c0 + ch, len);
      float Pr[Q], C0[Q], C1[Q], C2[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) Pr[q] = 1.0f, C0[q] = C1[q] = C2[q] = 0.0f;
      for (uint32_t b0 = c0; b0 < c1; b0 += kLongBatch) {
        const int nb = int(min(c1 - b0, uint32_t(kLongBatch)));
        bwd_stage<TILE>(S, start + b0, nb, lane, vals, rec, goff, tx, ty);
        __builtin_amdgcn_wave_barrier();
        for (int k = 0; k < nb; ++k) {
          const uint32_t pos = b0 + uint32_t(k) + 1u;
          const uint32_t m = __builtin_amdgcn_readfirstlane(S.mask[k]);
          const float4 r0 = S.r0[k], r1 = S.r1[k];
          const float cb = S.b[k];
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            if (((m >> q) & 1u) == 0u || pos > P.glast[q]) continue;  // wave-uniform
            const float px = px0 + float((q % GX) * 8), py = py0 + float((q / GX) * 8);
            const Alpha e = alpha_at(r0, r1.x, r1.y, px, py);
            const bool ok = e.ok & (pos <= P.last[q]);
            const float w = ok ? e.a * Pr[q] : 0.0f;
            C0[q] = fmaf(w, r1.z, C0[q]);
            C1[q] = fmaf(w, r1.w, C1[q]);
            C2[q] = fmaf(w, cb, C2[q]);
            Pr[q] = ok ? Pr[q] * (1.0f - e.a) : Pr[q];
          }
        }
        __builtin_amdgcn_wave_barrier();  // the staging is rewritten next
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) s_ch[c][q][lane] = make_float4(Pr[q], C0[q], C1[q], C2[q]);
    }
    __syncthreads();
    // B. wave q handles pixel group q: T after each chunk and the colour behind it
    if (wv < Q) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (q != wv) continue;
        // prefix: the transmittance entering each chunk replaces its product
        float T = 1.0f;
        for (int c = 0; c < nch; ++c) {
          const float pr = s_ch[c][q][lane].x;
          s_ch[c][q][lane].x = T;
          T *= pr;
        }
        // suffix: P.SdL holds T_final (bg . dL/dC); the forward's T_final is the
        // transmittance after the last chunk
        float behind = P.SdL[q];
        float Tafter = P.T[q];
        for (int c = nch - 1; c >= 0; --c) {
          const float4 pc = s_ch[c][q][lane];  // (T entering, colour)
          s_ch[c][q][lane] = make_float4(Tafter, behind, 0.0f, 0.0f);
          const float cg = fmaf(pc.y, P.g0[q], fmaf(pc.z, P.g1[q], pc.w * P.g2[q]));
          behind = fmaf(pc.x, cg, behind);
          Tafter = pc.x;
        }
      }
    }
    __syncthreads();
    // C. backward walk of each chunk from its end state
    for (int c = wv; c < nch; c += kLongWaves) {
      const uint32_t c0 = uint32_t(c) * ch, c1 = min(c0 + ch, len);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const float4 st = s_ch[c][q][lane];
        P.T[q] = st.x;
        P.SdL[q] = st.y;
      }
      for (uint32_t bend = c1; bend > c0;) {
        const uint32_t bstart = (bend - c0 > uint32_t(kLongBatch)) ? bend - kLongBatch : c0;
        const int nb = int(bend - bstart);
        bwd_stage<TILE>(S, start + bstart, nb, lane, vals, rec, goff, tx, ty);
        __builtin_amdgcn_wave_barrier();
        for (int k = nb - 1; k >= 0; --k)
          bwd_step<TILE>(P, S, k, bstart + uint32_t(k) + 1u, lane, px0, py0, pair_grad, cap);
        __builtin_amdgcn_wave_barrier();
        bend = bstart;
      }
    }
    __syncthreads();  // s_ch is rewritten for the block's next tile
  }
}

// -------------------------------------------------------------- chain rule
constexpr float SH0 = 0.28209479177387814f;
constexpr float SH1 = 0.48860251190291992f;
constexpr float SH2a = 1.0925484305920792f;
constexpr float SH2b = 0.31539156525252005f;
constexpr float SH2c = 0.54627421529603959f;
constexpr float SH3a = 0.59004358992664352f;
constexpr float SH3b = 2.8906114426405538f;
constexpr float SH3c = 0.45704579946446572f;
constexpr float SH3d = 0.37317633259011540f;
constexpr float SH3e = 1.4453057213202769f;

__device__ inline void sh_basis_b(float x, float y, float z, int deg, float* Y) {
  Y[0] = SH0;
  if (deg < 1) return;
  Y[1] = -SH1 * y;
  Y[2] = SH1 * z;
  Y[3] = -SH1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = SH2a * (x * y);
  Y[5] = -SH2a * (y * z);
  Y[6] = SH2b * (2.0f * zz - xx - yy);
  Y[7] = -SH2a * (x * z);
  Y[8] = SH2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -SH3a * y * (3.0f * xx - yy);
  Y[10] = SH3b * (x * y) * z;
  Y[11] = -SH3c * y * (4.0f * zz - xx - yy);
  Y[12] = SH3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  Y[13] = -SH3c * x * (4.0f * zz - xx - yy);
  Y[14] = SH3e * z * (xx - yy);
  Y[15] = -SH3a * x * (xx - 3.0f * yy);
}

// sum_k wk dY_k/d(x,y,z) for the polynomial form of the basis
__device__ inline void sh_dir_grad(float x, float y, float z, int deg, const float* wk,
                                   float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if (deg < 1) return;
  gy -= SH1 * wk[1];
  gz += SH1 * wk[2];
  gx -= SH1 * wk[3];
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx += SH2a * y * wk[4];          gy += SH2a * x * wk[4];
  gy -= SH2a * z * wk[5];          gz -= SH2a * y * wk[5];
  gx -= 2.0f * SH2b * x * wk[6];   gy -= 2.0f * SH2b * y * wk[6];   gz += 4.0f * SH2b * z * wk[6];
  gx -= SH2a * z * wk[7];          gz -= SH2a * x * wk[7];
  gx += 2.0f * SH2c * x * wk[8];   gy -= 2.0f * SH2c * y * wk[8];
  if (deg < 3) return;
  gx -= SH3a * 6.0f * x * y * wk[9];
  gy -= SH3a * (3.0f * xx - 3.0f * yy) * wk[9];
  gx += SH3b * y * z * wk[10];     gy += SH3b * x * z * wk[10];     gz += SH3b * x * y * wk[10];
  gx += SH3c * 2.0f * x * y * wk[11];
  gy -= SH3c * (4.0f * zz - xx - 3.0f * yy) * wk[11];
  gz -= SH3c * 8.0f * y * z * wk[11];
  gx -= SH3d * 6.0f * x * z * wk[12];
  gy -= SH3d * 6.0f * y * z * wk[12];
  gz += SH3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * wk[12];
  gx -= SH3c * (4.0f * zz - 3.0f * xx - yy) * wk[13];
  gy += SH3c * 2.0f * x * y * wk[13];
  gz -= SH3c * 8.0f * x * z * wk[13];
  gx += SH3e * 2.0f * x * z * wk[14];
  gy -= SH3e * 2.0f * y * z * wk[14];
  gz += SH3e * (xx - yy) * wk[14];
  gx -= SH3a * (3.0f * xx - 3.0f * yy) * wk[15];
  gy += SH3a * 6.0f * x * y * wk[15];
}

// One lane per (view, Gaussian) item: sum the item's pair slots (contiguous,
// tiles_touched of them, in index order) into nine planes g2d[c][item],
// written coalesced.  A lane adds up to kCoopSlots slots itself, in ascending
// order; an item with more (a footprint of many tiles) is summed by the whole
// wave: lane-strided coalesced loads, then the fixed-order register reduction,
// so the wave never waits on one lane's long serial loop.
constexpr int kCoopSlots = 32;

// U consecutive slots from slot k of an item with tt slots added to s in
// order (a slot past the last reloads slot k); returns the next slot
template <int U>
__device__ __forceinline__ uint32_t sum_slots(const float* __restrict__ pg, uint32_t k,
                                              uint32_t tt, float* s) {
  float x[U][kG];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const float* q = pg + size_t(k + u < tt ? k + u : k) * kG;
#pragma unroll
    for (int c = 0; c < kG; ++c) x[u][c] = q[c];
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (k + u < tt)
#pragma unroll
      for (int c = 0; c < kG; ++c) s[c] += x[u][c];
  return k + U;
}

__global__ __launch_bounds__(256) void k_pair_sum(const char* __restrict__ proj, size_t stride,
                                                  size_t tt_off, int n, int64_t M,
                                                  size_t goff_off,
                                                  const float* __restrict__ pair_grad,
                                                  int64_t cap, float* __restrict__ g2d) {
  const int lane = threadIdx.x & 63;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  uint32_t tt = 0u, off = 0u;
  if (i < M) {
    const int64_t v = i / n, g = i - v * n;
    tt = reinterpret_cast<const uint32_t*>(proj + v * stride + tt_off)[g];
    off = reinterpret_cast<const uint32_t*>(proj + v * stride + goff_off)[g];
    if (int64_t(off) + tt > cap) tt = 0u;  // pairs past the capacity have no slots
  }
  float s[kG];
#pragma unroll
  for (int c = 0; c < kG; ++c) s[c] = 0.0f;
  const bool coop = tt > uint32_t(kCoopSlots);
  if (!coop) {
    // several slots' loads in flight per step (a lane past its last slot
    // reloads slot k, which exists); the sums still add slot after slot in
    // order.  A lane with more than four slots left loads eight, else four:
    // 32 us at 1M Gaussians, 1600x1064, and 17 us at 200x133 (tile 8), against
    // 34 / 18 us with four per step and 31 / 20 us with eight (whose unused
    // loads and registers cost where items have one or two slots)
    const float* pg = pair_grad + size_t(off) * kG;
    for (uint32_t k = 0; k < tt;) {
      if (tt - k > 4u)
        k = sum_slots<8>(pg, k, tt, s);
      else
        k = sum_slots<4>(pg, k, tt, s);
    }
  }
  // the wave's long items, one after the other (all lanes take part)
  for (uint64_t bm = __ballot(coop); bm != 0ull; bm &= bm - 1ull) {
    const int src = __builtin_ctzll(bm);
    const uint32_t o = uint32_t(__shfl(int(off), src, 64));
    const uint32_t m = uint32_t(__shfl(int(tt), src, 64));
    float acc[kG];
#pragma unroll
    for (int c = 0; c < kG; ++c) acc[c] = 0.0f;
    const float* pg = pair_grad + size_t(o) * kG;
    for (uint32_t k = uint32_t(lane); k < m; k += 64u)
#pragma unroll
      for (int c = 0; c < kG; ++c) acc[c] += pg[size_t(k) * kG + c];
    float qv[3];
    wave_sum9(acc, qv);
    // lane 16 r + 15 holds components c0(r) (qv[0]) and c0(r) + 4 (qv[1]); lane 15 also 8
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c0 = ((r & 1) << 1) | (r >> 1);
      const float a = __shfl(qv[0], 16 * r + 15, 64), b = __shfl(qv[1], 16 * r + 15, 64);
      if (lane == src) {
        s[c0] = a;
        s[c0 + 4] = b;
      }
    }
    const float c8 = __shfl(qv[2], 15, 64);
    if (lane == src) s[8] = c8;
  }
  if (i < M) {
#pragma unroll
    for (int c = 0; c < kG; ++c) g2d[c * M + i] = s[c];
  }
}

// Inputs of the chain rule: the parameters, the projected records and the
// per-view 2D gradient planes.
struct ChainIn {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* sh;
  const char* proj;
  const float* g2d;
  int n, sh_degree;
};

// One Gaussian's parameter gradients, summed over the views of the call.
struct ChainOut {
  float dm[3], dls[3];
  float4 dq;
  float dlogit, m2abs;
  float dsh[GS_SH_COEFFS * 3];  // zero above the SH degree
};

// Chains Gaussian g's 2D gradients of every view to its parameters.  Returns
// false, leaving O untouched, when no view has a pair of g.  sh_row: g's 48
// SH coefficients (in LDS), or nullptr to read them from I.sh.
__device__ __forceinline__ bool chain_grad(const Views& V, const ChainIn& I, int g, ChainOut& O,
                                           const float* sh_row = nullptr) {
  const ProjLayout L(I.n);
  const int64_t M = int64_t(V.n_views) * I.n;
  const int K = (I.sh_degree + 1) * (I.sh_degree + 1);

  // does any view have gradient slots for this Gaussian?
  bool any = false;
  for (int v = 0; v < V.n_views; ++v)
    any |= reinterpret_cast<const uint32_t*>(I.proj + size_t(v) * L.stride + L.tt)[g] > 0u;
  if (!any) return false;

  const float mx = I.means[3 * g + 0], my = I.means[3 * g + 1], mz = I.means[3 * g + 2];
  const float s0 = expf(I.log_scales[3 * g + 0]);
  const float s1 = expf(I.log_scales[3 * g + 1]);
  const float s2 = expf(I.log_scales[3 * g + 2]);
  const float4 q4 = reinterpret_cast<const float4*>(I.quats)[g];
  const float qn2 = q4.x * q4.x + q4.y * q4.y + q4.z * q4.z + q4.w * q4.w;
  const float qlen = sqrtf(qn2);
  const float qinv = 1.0f / qlen;
  const float qw = q4.x * qinv, qx = q4.y * qinv, qy = q4.z * qinv, qz = q4.w * qinv;
  float Rq[9];
  Rq[0] = 1.0f - 2.0f * (qy * qy + qz * qz);
  Rq[1] = 2.0f * (qx * qy - qw * qz);
  Rq[2] = 2.0f * (qx * qz + qw * qy);
  Rq[3] = 2.0f * (qx * qy + qw * qz);
  Rq[4] = 1.0f - 2.0f * (qx * qx + qz * qz);
  Rq[5] = 2.0f * (qy * qz - qw * qx);
  Rq[6] = 2.0f * (qx * qz - qw * qy);
  Rq[7] = 2.0f * (qy * qz + qw * qx);
  Rq[8] = 1.0f - 2.0f * (qx * qx + qy * qy);
  const float sc[3] = {s0, s1, s2};
  float M3[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M3[3 * i + j] = Rq[3 * i + j] * sc[j];
  float Sg[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Sg[3 * i + j] =
          M3[3 * i] * M3[3 * j] + M3[3 * i + 1] * M3[3 * j + 1] + M3[3 * i + 2] * M3[3 * j + 2];
  // Mip-Splatting's 3D filter: Sigma + f I, opacity times c3 = prod s_i / sqrt(s_i^2 + f)
  const float f3 = V.filter3d ? V.filter3d[g] : 0.0f;
  Sg[0] += f3;
  Sg[4] += f3;
  Sg[8] += f3;
  const float c3 = V.filter3d ? filter3d_coef(s0, s1, s2, f3) : 1.0f;
  const float o = 1.0f / (1.0f + expf(-I.opacity_logits[g]));
  const float low = V.mip2d ? kMip2d : kDilation;
  const float* shg = sh_row ? sh_row : I.sh + size_t(g) * GS_SH_COEFFS * 3;

  float dm[3] = {0, 0, 0}, dS[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  float dop = 0.0f, m2abs = 0.0f;
  float* dshacc = O.dsh;  // coefficients above the degree stay zero
#pragma unroll
  for (int k = 0; k < GS_SH_COEFFS * 3; ++k) dshacc[k] = 0.0f;

  for (int v = 0; v < V.n_views; ++v) {
    const char* base = I.proj + size_t(v) * L.stride;
    const uint32_t tt = reinterpret_cast<const uint32_t*>(base + L.tt)[g];
    if (tt == 0u) continue;
    float gr[kG];
#pragma unroll
    for (int c = 0; c < kG; ++c) gr[c] = I.g2d[c * M + int64_t(v) * I.n + g];
    const uint32_t flags = reinterpret_cast<const uint32_t*>(base + L.flags)[g];
    const DevView cv = view_at(V, v);

    // ---- recompute the projection of this view
    const float xc = fmaf(cv.R[0], mx, fmaf(cv.R[1], my, fmaf(cv.R[2], mz, cv.t[0])));
    const float yc = fmaf(cv.R[3], mx, fmaf(cv.R[4], my, fmaf(cv.R[5], mz, cv.t[1])));
    const float zc = __fadd_rn(
        __fadd_rn(__fadd_rn(__fmul_rn(cv.R[6], mx), __fmul_rn(cv.R[7], my)),
                  __fmul_rn(cv.R[8], mz)),
        cv.t[2]);
    const float iz = 1.0f / zc, iz2 = iz * iz;
    const float j00 = cv.fx * iz, j11 = cv.fy * iz;
    const float j02 = -cv.fx * xc * iz2, j12 = -cv.fy * yc * iz2;
    float Tm[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Tm[k] = j00 * cv.R[k] + j02 * cv.R[6 + k];
      Tm[3 + k] = j11 * cv.R[3 + k] + j12 * cv.R[6 + k];
    }
    float U[6];  // U = T Sigma
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        U[3 * a + j] = Tm[3 * a] * Sg[j] + Tm[3 * a + 1] * Sg[3 + j] + Tm[3 * a + 2] * Sg[6 + j];
    const float r00 = U[0] * Tm[0] + U[1] * Tm[1] + U[2] * Tm[2];
    const float r01 = U[0] * Tm[3] + U[1] * Tm[4] + U[2] * Tm[5];
    const float r11 = U[3] * Tm[3] + U[4] * Tm[4] + U[5] * Tm[5];
    const float c00 = r00 + low, c01 = r01, c11 = r11 + low;
    const float idet = 1.0f / (c00 * c11 - c01 * c01);
    const float ca = c11 * idet, cb = -c01 * idet, cc = c00 * idet;

    // ---- conic -> Sigma': G' = -Q GQ Q with GQ = [[ga, gb/2], [gb/2, gc]]
    const float ga = gr[2], gbh = 0.5f * gr[3], gc = gr[4];
    const float X00 = ga * ca + gbh * cb, X01 = ga * cb + gbh * cc;
    const float X10 = gbh * ca + gc * cb, X11 = gbh * cb + gc * cc;
    float G00 = -(ca * X00 + cb * X10);
    float G01 = -0.5f * ((ca * X01 + cb * X11) + (cb * X00 + cc * X10));
    float G11 = -(cb * X01 + cc * X11);
    // the 2D mip filter's opacity factor c2 = sqrt(D1 / D2), D1 = det of the
    // unfiltered covariance, D2 = det Sigma' = 1 / idet: its gradient joins G'
    float c2 = 1.0f, id1 = 0.0f;
    if (V.mip2d) {
      const float d1 = r00 * r11 - r01 * r01;
      c2 = d1 > 0.0f ? sqrtf(d1 * idet) : 0.0f;
      id1 = d1 > 0.0f ? 1.0f / d1 : 0.0f;
    }
    // the blend summed o_b dL/do_b over the pixels (o_b = o c3 c2, the opacity
    // it blended with): divide by o_b once here
    const float ob = o * c3 * c2;
    const float gop = ob > 0.0f ? gr[5] / ob : 0.0f;  // dL/do_b
    if (V.mip2d && c2 > 0.0f) {
      const float gc2 = gop * o * c3;  // dL/dc2
      G00 += gc2 * (0.5f * c2 * (r11 * id1 - c11 * idet));
      G01 += gc2 * (0.5f * c2 * r01 * (idet - id1));
      G11 += gc2 * (0.5f * c2 * (r00 * id1 - c00 * idet));
    }
    // Sigma' = T Sigma T^T: dSigma += T^T G' T ; dT = 2 G' U
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float a0 = G00 * Tm[j] + G01 * Tm[3 + j];
        const float a1 = G01 * Tm[j] + G11 * Tm[3 + j];
        dS[3 * i + j] += Tm[i] * a0 + Tm[3 + i] * a1;
      }
    float dT[6];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      dT[j] = 2.0f * (G00 * U[j] + G01 * U[3 + j]);
      dT[3 + j] = 2.0f * (G01 * U[j] + G11 * U[3 + j]);
    }
    // T = J W: dJ = dT W^T (only J00, J02, J11, J12 vary)
    const float dJ00 = dT[0] * cv.R[0] + dT[1] * cv.R[1] + dT[2] * cv.R[2];
    const float dJ02 = dT[0] * cv.R[6] + dT[1] * cv.R[7] + dT[2] * cv.R[8];
    const float dJ11 = dT[3] * cv.R[3] + dT[4] * cv.R[4] + dT[5] * cv.R[5];
    const float dJ12 = dT[3] * cv.R[6] + dT[4] * cv.R[7] + dT[5] * cv.R[8];
    // dL/dmean2D = Q (sum dpow dx, sum dpow dy) with Q the conic (a, b; b, c):
    // d p2 / d mean = -(2A dx + B dy, B dx + 2C dy) in base 2, and -ln2 (2A, B, 2C)
    // = (a, b, c)
    const float gmx = ca * gr[0] + cb * gr[1], gmy = cb * gr[0] + cc * gr[1];
    const float iz3 = iz2 * iz;
    const float gxc = gmx * cv.fx * iz - dJ02 * cv.fx * iz2;
    const float gyc = gmy * cv.fy * iz - dJ12 * cv.fy * iz2;
    const float gzc = -gmx * cv.fx * xc * iz2 - gmy * cv.fy * yc * iz2 - dJ00 * cv.fx * iz2 +
                      dJ02 * 2.0f * cv.fx * xc * iz3 - dJ11 * cv.fy * iz2 +
                      dJ12 * 2.0f * cv.fy * yc * iz3;
#pragma unroll
    for (int k = 0; k < 3; ++k) dm[k] += cv.R[k] * gxc + cv.R[3 + k] * gyc + cv.R[6 + k] * gzc;

    // ---- colour
    float dx = mx - cv.campos[0], dy = my - cv.campos[1], dz = mz - cv.campos[2];
    const float dlen = sqrtf(dx * dx + dy * dy + dz * dz);
    const float dn = 1.0f / dlen;
    dx *= dn; dy *= dn; dz *= dn;
    float Y[GS_SH_COEFFS];
#pragma unroll
    for (int k = 0; k < GS_SH_COEFFS; ++k) Y[k] = 0.0f;
    sh_basis_b(dx, dy, dz, I.sh_degree, Y);
    const float grgb[3] = {(flags & 1u) ? 0.0f : gr[6], (flags & 2u) ? 0.0f : gr[7],
                           (flags & 4u) ? 0.0f : gr[8]};
    float wk[GS_SH_COEFFS];
#pragma unroll
    for (int k = 0; k < GS_SH_COEFFS; ++k) {
      wk[k] = 0.0f;
      if (k < K) {
        wk[k] = grgb[0] * shg[3 * k] + grgb[1] * shg[3 * k + 1] + grgb[2] * shg[3 * k + 2];
#pragma unroll
        for (int c = 0; c < 3; ++c) dshacc[3 * k + c] += grgb[c] * Y[k];
      }
    }
    float gdx, gdy, gdz;
    sh_dir_grad(dx, dy, dz, I.sh_degree, wk, gdx, gdy, gdz);
    const float dd = dx * gdx + dy * gdy + dz * gdz;
    dm[0] += (gdx - dx * dd) * dn;
    dm[1] += (gdy - dy * dd) * dn;
    dm[2] += (gdz - dz * dd) * dn;

    dop += V.mip2d ? gop * c2 : gop;  // w.r.t. the opacity before the 2D factor
    m2abs += sqrtf(gmx * gmx + gmy * gmy);
  }

  // ---- Sigma = M M^T -> scales and rotation
  float dMm[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      dMm[3 * i + j] = 2.0f * (dS[3 * i] * M3[j] + dS[3 * i + 1] * M3[3 + j] + dS[3 * i + 2] * M3[6 + j]);
  float dls[3], dR[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    dls[j] = (dMm[j] * Rq[j] + dMm[3 + j] * Rq[3 + j] + dMm[6 + j] * Rq[6 + j]) * sc[j];
#pragma unroll
    for (int i = 0; i < 3; ++i) dR[3 * i + j] = dMm[3 * i + j] * sc[j];
  }
  if (V.filter3d) {  // d c3 / d log s_j = c3 f / (s_j^2 + f)
    const float gc3 = dop * o * c3;
#pragma unroll
    for (int j = 0; j < 3; ++j) dls[j] += gc3 * f3 / (sc[j] * sc[j] + f3);
  }
  const float gw = -2.0f * qz * dR[1] + 2.0f * qy * dR[2] + 2.0f * qz * dR[3] -
                   2.0f * qx * dR[5] - 2.0f * qy * dR[6] + 2.0f * qx * dR[7];
  const float gx = 2.0f * qy * dR[1] + 2.0f * qz * dR[2] + 2.0f * qy * dR[3] - 4.0f * qx * dR[4] -
                   2.0f * qw * dR[5] + 2.0f * qz * dR[6] + 2.0f * qw * dR[7] - 4.0f * qx * dR[8];
  const float gy = -4.0f * qy * dR[0] + 2.0f * qx * dR[1] + 2.0f * qw * dR[2] +
                   2.0f * qx * dR[3] + 2.0f * qz * dR[5] - 2.0f * qw * dR[6] +
                   2.0f * qz * dR[7] - 4.0f * qy * dR[8];
  const float gz = -4.0f * qz * dR[0] - 2.0f * qw * dR[1] + 2.0f * qx * dR[2] +
                   2.0f * qw * dR[3] - 4.0f * qz * dR[4] + 2.0f * qy * dR[5] +
                   2.0f * qx * dR[6] + 2.0f * qy * dR[7];
  const float qd = qw * gw + qx * gx + qy * gy + qz * gz;
  float4 dq4 = make_float4((gw - qw * qd) * qinv, (gx - qx * qd) * qinv, (gy - qy * qd) * qinv,
                           (gz - qz * qd) * qinv);
  const float dlogit = (V.filter3d ? dop * c3 : dop) * o * (1.0f - o);
  O.dlogit = dlogit;
  O.dq = dq4;
  O.m2abs = m2abs;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    O.dm[k] = dm[k];
    O.dls[k] = dls[k];
  }
  return true;
}

// The block's SH rows staged in LDS with coalesced 16-byte loads (rows of an
// odd stride, conflict-free), only for the Gaussians with a pair in some view:
// the others leave the chain rule at once and never read their row (in the
// spatial storage order whole blocks of them skip the load).  Every thread of
// the block must call it; it ends with a barrier.
template <int T>
__device__ inline void stage_sh_needed(const Views& V, const ChainIn& I, int g0, float* s_buf,
                                       int* s_need) {
  constexpr int F = GS_SH_COEFFS * 3, kRow = F + 1;
  const int g = g0 + int(threadIdx.x);
  bool any = false;
  if (g < I.n) {
    const ProjLayout L(I.n);
    for (int v = 0; v < V.n_views; ++v)
      any |= reinterpret_cast<const uint32_t*>(I.proj + size_t(v) * L.stride + L.tt)[g] > 0u;
  }
  s_need[threadIdx.x] = any ? 1 : 0;
  __syncthreads();
  const int rows = (I.n - g0 < T) ? I.n - g0 : T;
  const float4* src = reinterpret_cast<const float4*>(I.sh + size_t(g0) * F);
  // a thread's float4s are i = t + u * T, u < 12 (rows <= T): every load is
  // issued before the first LDS write, so their latencies overlap
  constexpr int U = F / 4;
  float4 q[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = int(threadIdx.x) + u * T;
    if (i < rows * U && s_need[(4 * i) / F]) q[u] = src[i];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = int(threadIdx.x) + u * T;
    const int f = 4 * i, row = f / F, k = f - row * F;
    if (i < rows * U && s_need[row]) {
      float* d = s_buf + row * kRow + k;
      d[0] = q[u].x;
      d[1] = q[u].y;
      d[2] = q[u].z;
      d[3] = q[u].w;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(128) void k_chain(Views V, ChainIn I, int accumulate,
                                               float* __restrict__ d_means,
                                               float* __restrict__ d_log_scales,
                                               float* __restrict__ d_quats,
                                               float* __restrict__ d_opacity_logits,
                                               float* __restrict__ d_sh,
                                               float* __restrict__ d_mean2d_abs) {
  // the block's SH coefficients staged in LDS as in k_chain_adam
  constexpr int F = GS_SH_COEFFS * 3, kRow = F + 1;
  __shared__ float s_sh[128 * kRow];
  __shared__ int s_need[128];
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  stage_sh_needed<128>(V, I, blockIdx.x * blockDim.x, s_sh, s_need);
  if (g >= I.n) return;
  ChainOut O;
  float* dshg = d_sh + size_t(g) * GS_SH_COEFFS * 3;
  if (!chain_grad(V, I, g, O, s_sh + threadIdx.x * kRow)) {
    if (!accumulate) {
      for (int k = 0; k < 3; ++k) d_means[3 * g + k] = d_log_scales[3 * g + k] = 0.0f;
      reinterpret_cast<float4*>(d_quats)[g] = make_float4(0.f, 0.f, 0.f, 0.f);
      d_opacity_logits[g] = 0.0f;
      for (int k = 0; k < GS_SH_COEFFS * 3; ++k) dshg[k] = 0.0f;
      if (d_mean2d_abs) d_mean2d_abs[g] = 0.0f;
    }
    return;
  }
  float4 dq4 = O.dq;
  if (accumulate) {
    const float4 p4 = reinterpret_cast<float4*>(d_quats)[g];
    dq4.x += p4.x; dq4.y += p4.y; dq4.z += p4.z; dq4.w += p4.w;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      O.dm[k] += d_means[3 * g + k];
      O.dls[k] += d_log_scales[3 * g + k];
    }
    d_opacity_logits[g] += O.dlogit;
    const int K3 = 3 * (I.sh_degree + 1) * (I.sh_degree + 1);
#pragma unroll
    for (int k = 0; k < GS_SH_COEFFS * 3; ++k)
      if (k < K3) dshg[k] += O.dsh[k];
    if (d_mean2d_abs) d_mean2d_abs[g] += O.m2abs;
  } else {
    d_opacity_logits[g] = O.dlogit;
#pragma unroll
    for (int k = 0; k < GS_SH_COEFFS * 3; ++k) dshg[k] = O.dsh[k];
    if (d_mean2d_abs) d_mean2d_abs[g] = O.m2abs;
  }
  reinterpret_cast<float4*>(d_quats)[g] = dq4;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d_means[3 * g + k] = O.dm[k];
    d_log_scales[3 * g + k] = O.dls[k];
  }
}

// The chain rule fused with the Adam step of all five parameter groups: each
// thread chains its Gaussian and updates its means, scales, rotation and
// opacity straight from registers; the block's SH gradients go through LDS so
// that the SH update (48 of the 59 values per Gaussian) streams p, m and v
// with coalesced float4 accesses.  Gaussians without pairs get a zero
// gradient, as in the unfused step.  Each Gaussian's parameters are read (by
// chain_grad) before any of them is updated, and only its own block updates
// them, so the in-place update is safe.
constexpr int kCA = 128;

// Adam's moments are read and written once per step and not touched again
// until the next step's update.  Non-temporal accesses keep them from pushing
// the parameters out of the caches, which the next step's preprocess reads
// right after (1M Gaussians, 1600x1064: preprocess 58 -> 42 us in the step,
// chain + Adam 267 -> 257 us).  Only the groups whose accesses are coalesced
// per instruction use them: a wave's three loads of a three-float group
// (means, log-scales) share cache lines, which a non-temporal load does not
// keep (chain + Adam 267 -> 275 us with those included).
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_nt(const float4* p) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void store_nt(float4* p, float4 a) {
  const f32x4 v = {a.x, a.y, a.z, a.w};
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p));
}
__device__ __forceinline__ float load_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void store_nt(float* p, float a) { __builtin_nontemporal_store(a, p); }

struct AdamGroups {
  float* p[5];
  float* m[5];
  float* v[5];
  float lr[6];  // the five groups; lr[4] for the SH degree-0 terms, lr[5] for the rest
  const float* lr_dev;  // device copy of lr, read instead when set
  float b1, b2, eps;
  const int32_t* step_dev;
  int sparse;  // 1: Gaussians with no pair in any view keep p, m and v unchanged
};

// memory-bound: at most 168 VGPRs, so three waves fit per SIMD
__global__ __launch_bounds__(kCA) __attribute__((amdgpu_waves_per_eu(3))) void k_chain_adam(
    Views V, ChainIn I, AdamGroups A, float* __restrict__ d_mean2d_abs) {
  // the block's SH coefficients arrive in LDS (stage_sh_needed) for the chain
  // rule's direction term; the same LDS then holds the SH gradients for the
  // Adam loop
  constexpr int F = GS_SH_COEFFS * 3, kRow = F + 1;
  __shared__ __align__(16) float s_buf[kCA * kRow];
  float4* s_g = reinterpret_cast<float4*>(s_buf);
  __shared__ float s_c[2];
  __shared__ int s_upd[kCA];
  // the count was advanced for this step by k_zero_pairs, earlier in the same call;
  // the learning rates come from the device when lr_dev is set
  __shared__ float lr[6];
  if (threadIdx.x == 0) adam_bias(A.step_dev, A.b1, A.b2, s_c[0], s_c[1], 0);
  if (threadIdx.x < 6) lr[threadIdx.x] = A.lr_dev ? A.lr_dev[threadIdx.x] : A.lr[threadIdx.x];
  const int g = blockIdx.x * kCA + threadIdx.x;
  stage_sh_needed<kCA>(V, I, blockIdx.x * kCA, s_buf, s_upd);
  ChainOut O;
  bool have = false;
  if (g < I.n) have = chain_grad(V, I, g, O, s_buf + threadIdx.x * kRow);
  __syncthreads();  // every row is read before the gradients overwrite the LDS
  const bool upd = have || !A.sparse;
  s_upd[threadIdx.x] = upd ? 1 : 0;
  if (!have) {
#pragma unroll
    for (int k = 0; k < 3; ++k) O.dm[k] = O.dls[k] = 0.0f;
    O.dq = make_float4(0.f, 0.f, 0.f, 0.f);
    O.dlogit = O.m2abs = 0.0f;
#pragma unroll
    for (int k = 0; k < GS_SH_COEFFS * 3; ++k) O.dsh[k] = 0.0f;
  }
#pragma unroll
  for (int q = 0; q < GS_SH_COEFFS * 3 / 4; ++q)
    s_g[threadIdx.x * (GS_SH_COEFFS * 3 / 4) + q] =
        make_float4(O.dsh[4 * q], O.dsh[4 * q + 1], O.dsh[4 * q + 2], O.dsh[4 * q + 3]);
  __syncthreads();
  const AdamCoef C{A.b1, A.b2, A.eps, s_c[0], s_c[1]};
  if (g < I.n && d_mean2d_abs) d_mean2d_abs[g] = O.m2abs;
  if (g < I.n && upd) {
    // every value is loaded before the first store (the groups are distinct
    // arrays), so the loads' latencies overlap
    float pm[3], mm[3], vm[3], ps[3], ms[3], vs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int j = 3 * g + k;
      pm[k] = A.p[0][j];
      mm[k] = A.m[0][j];
      vm[k] = A.v[0][j];
      ps[k] = A.p[1][j];
      ms[k] = A.m[1][j];
      vs[k] = A.v[1][j];
    }
    float4 p4 = reinterpret_cast<float4*>(A.p[2])[g];
    float4 m4 = load_nt(reinterpret_cast<float4*>(A.m[2]) + g);
    float4 v4 = load_nt(reinterpret_cast<float4*>(A.v[2]) + g);
    float po = A.p[3][g], mo = load_nt(A.m[3] + g), vo = load_nt(A.v[3] + g);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      adam_one(pm[k], O.dm[k], mm[k], vm[k], lr[0], C);
      adam_one(ps[k], O.dls[k], ms[k], vs[k], lr[1], C);
    }
    adam_one(p4.x, O.dq.x, m4.x, v4.x, lr[2], C);
    adam_one(p4.y, O.dq.y, m4.y, v4.y, lr[2], C);
    adam_one(p4.z, O.dq.z, m4.z, v4.z, lr[2], C);
    adam_one(p4.w, O.dq.w, m4.w, v4.w, lr[2], C);
    adam_one(po, O.dlogit, mo, vo, lr[3], C);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int j = 3 * g + k;
      A.p[0][j] = pm[k];
      A.m[0][j] = mm[k];
      A.v[0][j] = vm[k];
      A.p[1][j] = ps[k];
      A.m[1][j] = ms[k];
      A.v[1][j] = vs[k];
    }
    reinterpret_cast<float4*>(A.p[2])[g] = p4;
    store_nt(reinterpret_cast<float4*>(A.m[2]) + g, m4);
    store_nt(reinterpret_cast<float4*>(A.v[2]) + g, v4);
    A.p[3][g] = po;
    store_nt(A.m[3] + g, mo);
    store_nt(A.v[3] + g, vo);
  }
  // SH: the block's contiguous slab of 48 values per Gaussian, float4 per lane
  const int g0 = blockIdx.x * kCA;
  const int n4 = ((I.n - g0 < kCA) ? I.n - g0 : kCA) * (GS_SH_COEFFS * 3 / 4);
  float4* __restrict__ P = reinterpret_cast<float4*>(A.p[4] + size_t(g0) * GS_SH_COEFFS * 3);
  float4* __restrict__ Mm = reinterpret_cast<float4*>(A.m[4] + size_t(g0) * GS_SH_COEFFS * 3);
  float4* __restrict__ Vv = reinterpret_cast<float4*>(A.v[4] + size_t(g0) * GS_SH_COEFFS * 3);
#pragma unroll 4
  for (int j = threadIdx.x; j < n4; j += kCA) {
    if (!s_upd[j / (GS_SH_COEFFS * 3 / 4)]) continue;
    float4 p = P[j], m = load_nt(Mm + j), v = load_nt(Vv + j);
    const float4 gg = s_g[j];
    // values 0..2 of a Gaussian's 48 are its degree-0 coefficients
    const int e = (4 * j) % (GS_SH_COEFFS * 3);
    adam_one(p.x, gg.x, m.x, v.x, e + 0 < 3 ? lr[4] : lr[5], C);
    adam_one(p.y, gg.y, m.y, v.y, e + 1 < 3 ? lr[4] : lr[5], C);
    adam_one(p.z, gg.z, m.z, v.z, e + 2 < 3 ? lr[4] : lr[5], C);
    adam_one(p.w, gg.w, m.w, v.w, lr[5], C);
    P[j] = p;
    store_nt(Mm + j, m);
    store_nt(Vv + j, v);
  }
}


struct BwdWs {
  size_t g2d, pairs, bytes;
  BwdWs(int64_t M, int64_t cap) {
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align256(b); return r; };
    g2d = take(4 * kG * M);
    pairs = take(size_t(cap) * kG * 4);
    bytes = o;
  }
};

// ---- static balancing of the one-wave-per-tile backward.  All of its waves
// are resident at once, so a SIMD's time is the sum of its waves' work, and
// tiles dealt out in index order leave the busiest SIMD about 1.2x the mean.
// Block 0 of k_zero_pairs ranks each XCD's share of the tiles by list length
// (256 buckets, longest first) and deals the ranks to that XCD's blocks with
// order_block (rounds of 32 of its blocks, every other round reversed), so
// that blocks b and b + 256 pair a heavy tile with a light one while every
// XCD keeps the contiguous share of each view that xcd_tile gives it (the
// Gaussians of neighbouring tiles then meet in one L2).  Which block takes
// which tile changes no result.

// The balanced order of XCD x's share: its n_x tiles (the ones xcd_tile gives
// blocks x, x + 8, ...) ranked into 256 buckets of list length, heaviest first
// (bucket width from the share's longest list), and dealt by order_block.  One
// 1024-thread block per XCD share; every thread of the block calls it.
__device__ void tile_order_xcd(const RViews& RV, const uint32_t* __restrict__ ranges,
                               uint32_t* __restrict__ order, int x) {
  const int n_x = RV.xcd_off[x][RV.n_views];  // tiles (and blocks) of XCD x
  auto tile = [&](int idx) { return xcd_tile(idx * kXcds + x, RV); };
  auto cost = [&](int t) { return ranges[2 * t + 1] - ranges[2 * t]; };
  __shared__ uint32_t s_hist[256], s_off[256], s_max;
  const int tid = threadIdx.x;
  if (tid < 256) s_hist[tid] = 0u;
  if (tid == 0) s_max = 0u;
  __syncthreads();
  uint32_t mx = 0;
  for (int idx = tid; idx < n_x; idx += 1024) mx = max(mx, cost(tile(idx)));
  atomicMax(&s_max, mx);
  __syncthreads();
  const uint64_t top = uint64_t(s_max) + 1u;
  auto bucket = [&](uint32_t c) { return 255u - uint32_t(uint64_t(c) * 256u / top); };
  for (int idx = tid; idx < n_x; idx += 1024) atomicAdd(&s_hist[bucket(cost(tile(idx)))], 1u);
  __syncthreads();
  // exclusive scan of the 256 bucket counts by the first wave, four per lane
  if (tid < 64) {
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = s_hist[4 * tid + k];
      sum += v[k];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d, 64);
      if (tid >= d) inc += y;
    }
    uint32_t ex = inc - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s_off[4 * tid + k] = ex;
      ex += v[k];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < n_x; idx += 1024) {
    const int t = tile(idx);
    const int r = int(atomicAdd(&s_off[bucket(cost(t))], 1u));  // rank, heaviest first
    order[order_block(r, n_x) * kXcds + x] = uint32_t(t);
  }
}

// Blocks kXcds.. clear the pair slots [0, min(total, cap)); blocks 0..kXcds-1
// meanwhile write the backward's tile order when `order` is set (block x the
// order of XCD x's share) and block 0, for the backward fused with Adam,
// advances the device step count (`step_dev`) once.
constexpr int kZeroBlocks = 512;
__global__ __launch_bounds__(1024) void k_zero_pairs(float* __restrict__ p,
                                                     const int64_t* __restrict__ total,
                                                     int64_t cap, RViews RV,
                                                     const uint32_t* __restrict__ ranges,
                                                     uint32_t* __restrict__ order,
                                                     int32_t* __restrict__ step_dev) {
  if (blockIdx.x < unsigned(kXcds)) {
    if (blockIdx.x == 0 && step_dev && threadIdx.x == 0) *step_dev += 1;
    if (order) tile_order_xcd(RV, ranges, order, int(blockIdx.x));
    return;
  }
  const int64_t tot = total ? *total : 0;
  const int64_t np = (tot < cap) ? tot : cap;
  const int64_t m = np * kG;
  for (int64_t i = int64_t(blockIdx.x - kXcds) * blockDim.x + threadIdx.x; i < m;
       i += int64_t(gridDim.x - kXcds) * blockDim.x)
    p[i] = 0.0f;
}

template <int TILE>
void launch_bwd_tile(int batch, dim3 grid, const RViews& RV, int n, const char* proj,
                     size_t stride, const uint32_t* ranges, const uint32_t* vals,
                     const float* final_T, const uint32_t* last_contrib, const float* dL,
                     size_t goff, float* pairs, int64_t cap, const float* bg,
                     const uint32_t* order, hipStream_t st) {
  const dim3 block(64);
  // launches with few tiles hand long lists to the list-parallel kernel
  const int split = split_long_lists(RV, TILE) ? 1 : 0;
#define GS_BWD_LAUNCH(B)                                                                       \
  GS_LAUNCH("k_blend_bwd", HIP_KERNEL_NAME(k_blend_bwd<TILE, B>), grid, block, 0, st, RV, n, proj,   \
                     stride, ranges, vals, final_T, last_contrib, dL, goff, pairs, cap, bg[0], \
                     bg[1], bg[2], split, split ? nullptr : order)
  switch (batch) {
    case 128: GS_BWD_LAUNCH(128); break;
    case 256: GS_BWD_LAUNCH(256); break;
    default: GS_BWD_LAUNCH(512); break;
  }
#undef GS_BWD_LAUNCH
  if (split) {
    const unsigned nb = unsigned(RV.total_tiles < kLongBlocks ? RV.total_tiles : kLongBlocks);
    GS_LAUNCH("k_blend_bwd_long", HIP_KERNEL_NAME(k_blend_bwd_long<TILE <= 16 ? TILE : 16>),
              dim3(nb), dim3(64 * kLongWaves), 0, st, RV, n, proj, stride, ranges, vals, final_T,
              last_contrib, dL, goff, pairs, cap, bg[0], bg[1], bg[2]);
  }
}

}  // namespace

size_t render_bwd_ws_bytes(int n_views, int n, int64_t cap) {
  return BwdWs(int64_t(n_views) * n, cap).bytes;
}

namespace {

// Everything before the chain rule: the backward blend into the per-pair
// slots and their sums into the per-view 2D gradient planes.
hipError_t bwd_to_planes(const Views& V, int n, const gs_raster_cfg& cfg, const char* proj,
                         const uint32_t* ranges, const uint32_t* vals, const float* final_T,
                         const uint32_t* last_contrib, const float* dL_dimage, int64_t cap,
                         char* ws, float** g2d_out, int32_t* step_dev, hipStream_t st) {
  const int64_t M = int64_t(V.n_views) * n;
  const BwdWs B(M, cap);
  float* pairs = reinterpret_cast<float*>(ws + B.pairs);
  const ProjLayout L(n);
  // the items' pair offsets and the pair total, recorded in proj by the binning
  const size_t goff = L.goff;
  const int64_t* total = proj ? reinterpret_cast<const int64_t*>(proj + L.total) : nullptr;
  // the balanced tile order (launches without list-parallel tiles), kept in the
  // 2D-gradient planes, which k_pair_sum writes only after the blend
  const RViews RV = make_rviews(V);
  const size_t T = size_t(V.total_tiles);
  uint32_t* order = nullptr;
  if (T > 0 && !split_long_lists(RV, cfg.tile) && size_t(4) * kG * size_t(M) >= 4 * T)
    order = reinterpret_cast<uint32_t*>(ws + B.g2d);
  GS_LAUNCH("k_zero_pairs", k_zero_pairs, dim3(kXcds + kZeroBlocks), dim3(1024), 0, st, pairs,
            total, cap, RV, ranges, order, step_dev);
  if (V.total_tiles > 0) {
    const dim3 grid(unsigned(V.total_tiles));
    switch (cfg.tile) {
      case 8:
        launch_bwd_tile<8>(cfg.lds_batch, grid, RV, n, proj, L.stride, ranges, vals, final_T,
                           last_contrib, dL_dimage, goff, pairs, cap, cfg.bg, order, st);
        break;
      case 16:
        launch_bwd_tile<16>(cfg.lds_batch, grid, RV, n, proj, L.stride, ranges, vals, final_T,
                            last_contrib, dL_dimage, goff, pairs, cap, cfg.bg, order, st);
        break;
      default:
        launch_bwd_tile<32>(cfg.lds_batch, grid, RV, n, proj, L.stride, ranges, vals, final_T,
                            last_contrib, dL_dimage, goff, pairs, cap, cfg.bg, order, st);
        break;
    }
  }
  float* g2d = reinterpret_cast<float*>(ws + B.g2d);
  if (M > 0)
    GS_LAUNCH("k_pair_sum", k_pair_sum, dim3(unsigned((M + 255) / 256)), dim3(256), 0, st, proj,
              L.stride, L.tt, n, M, goff, pairs, cap, g2d);
  *g2d_out = g2d;
  return hipSuccess;
}

}  // namespace

hipError_t launch_render_bwd(const Views& V, int n, const gs_raster_cfg& cfg,
                             const float* means, const float* log_scales, const float* quats,
                             const float* opacity_logits, const float* sh, int sh_degree,
                             const char* proj, const uint32_t* ranges, const uint32_t* vals,
                             const float* final_T, const uint32_t* last_contrib,
                             const float* dL_dimage, float* d_means, float* d_log_scales,
                             float* d_quats, float* d_opacity_logits, float* d_sh,
                             float* d_mean2d_abs, int accumulate, int64_t cap, void* ws,
                             hipStream_t st) {
  if (int64_t(V.n_views) * n == 0) return hipSuccess;
  float* g2d = nullptr;
  hipError_t e = bwd_to_planes(V, n, cfg, proj, ranges, vals, final_T, last_contrib, dL_dimage,
                               cap, static_cast<char*>(ws), &g2d, nullptr, st);
  if (e != hipSuccess) return e;
  const ChainIn I{means, log_scales, quats, opacity_logits, sh, proj, g2d, n, sh_degree};
  GS_LAUNCH("k_chain", k_chain, dim3(unsigned((n + 127) / 128)), dim3(128), 0, st, V, I,
            accumulate, d_means, d_log_scales, d_quats, d_opacity_logits, d_sh, d_mean2d_abs);
  return hipGetLastError();
}

hipError_t launch_render_bwd_adam(const Views& V, int n, const gs_raster_cfg& cfg, float* means,
                                  float* log_scales, float* quats, float* opacity_logits,
                                  float* sh, int sh_degree, const char* proj,
                                  const uint32_t* ranges, const uint32_t* vals,
                                  const float* final_T, const uint32_t* last_contrib,
                                  const float* dL_dimage, const FusedAdam& A,
                                  float* d_mean2d_abs, int64_t cap, void* ws, hipStream_t st) {
  if (n > 0) {
    float* g2d = nullptr;
    hipError_t e = bwd_to_planes(V, n, cfg, proj, ranges, vals, final_T, last_contrib,
                                 dL_dimage, cap, static_cast<char*>(ws), &g2d, A.step_dev, st);
    if (e != hipSuccess) return e;
    const ChainIn I{means, log_scales, quats, opacity_logits, sh, proj, g2d, n, sh_degree};
    AdamGroups G{};
    float* P[5] = {means, log_scales, quats, opacity_logits, sh};
    for (int k = 0; k < 5; ++k) {
      G.p[k] = P[k];
      G.m[k] = A.m[k];
      G.v[k] = A.v[k];
    }
    for (int k = 0; k < 6; ++k) G.lr[k] = A.lr[k];
    G.lr_dev = A.lr_dev;
    G.b1 = A.b1;
    G.b2 = A.b2;
    G.eps = A.eps;
    G.step_dev = A.step_dev;
    G.sparse = A.sparse;
    GS_LAUNCH("k_chain_adam", k_chain_adam, dim3(unsigned((n + kCA - 1) / kCA)), dim3(kCA), 0,
              st, V, I, G, d_mean2d_abs);
    return hipGetLastError();  // k_zero_pairs advanced the step count
  }
  return launch_step_inc(A.step_dev, st);
}

}  // namespace gsk
