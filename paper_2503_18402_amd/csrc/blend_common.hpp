// Pieces shared by the forward and backward blend kernels.  The alpha of a
// (pixel, Gaussian) evaluation is computed by ONE inline function so that the
// backward replays exactly the forward's float32 decisions (cutoff, clamp,
// early exit); the library is built without floating-point contraction and
// every fused multiply-add here is explicit.
#pragma once

#include "gs_internal.hpp"

namespace gsk {

// One 64-lane wave per tile.  The tile is cut into 8x8 groups; lane l owns the
// pixel (l % 8, l / 8) of every group, so a lane holds kGroups pixels and a
// Gaussian's footprint box selects whole groups with a wave-uniform mask.
template <int TILE>
struct TileShape {
  static constexpr int kGroupsX = TILE / 8;
  static constexpr int kGroups = kGroupsX * kGroupsX;
};

// Forward layout: several waves per tile, each owning an R x R square (R = 8 for
// 8x8 and 16x16 tiles, 16 for 32x32 tiles); lane l sits at (l % 8, l / 8) of every
// 8x8 sub-square of its wave, so a lane owns kSub x kSub pixels.
template <int TILE>
struct WaveShape {
  static constexpr int kThreads = (TILE == 8) ? 64 : 256;
  static constexpr int kWaves = kThreads / 64;
  static constexpr int kRegion = (TILE == 8) ? 8 : TILE / 2;
  static constexpr int kSub = kRegion / 8;
  static constexpr int kPix = kSub * kSub;
};

__device__ __forceinline__ bool box_overlaps(uint32_t lo, uint32_t hi, int x0, int y0, int x1,
                                             int y1) {
  return box_x(lo) <= x1 && box_x(hi) >= x0 && box_y(lo) <= y1 && box_y(hi) >= y0;
}

// alpha of a record at pixel centre (px, py): the record holds the base-2
// conic (A, B, C) and lo = log2 of the opacity, so o G2D = 2^(p2 + lo) with
// p2 = A dx^2 + B dx dy + C dy^2.  The pixel takes the Gaussian iff `ok`:
// p2 <= 0 and o G2D >= 1/255, decided on the exponent, so callers that branch
// on `ok` before using `a` evaluate the exponential only where it is used.
struct Alpha {
  float dx, dy, raw, a;
  bool ok;
};
__device__ __forceinline__ Alpha alpha_at(const float4 r0, const float C, const float lo,
                                          const float px, const float py) {
  Alpha r;
  r.dx = px - r0.x;
  r.dy = py - r0.y;
  const float t0 = r0.w * r.dy;
  const float t1 = fmaf(r0.z, r.dx, t0);
  const float t2 = C * r.dy;
  const float t3 = t2 * r.dy;
  const float p2 = fmaf(r.dx, t1, t3);
  const float q = p2 + lo;
  r.ok = (p2 <= 0.0f) & (q >= kLog2AlphaMin);
  r.raw = __builtin_amdgcn_exp2f(q);
  r.a = fminf(kAlphaMax, r.raw);
  return r;
}

// Workgroups are dealt to the XCDs round-robin (block b runs on XCD b % 8), and each
// XCD has its own L2.  Neighbouring tiles share most of their Gaussians, so every
// XCD walks one contiguous eighth of each view's tiles, views in RV.order (fewest
// tiles first): block b is the (b / 8)-th tile of XCD b % 8 in that walk.  This
// keeps L2 locality, balances mixed-resolution batches across XCDs, and starts the
// long lists of low-resolution views first.  A bijection on [0, total tiles).
__host__ __device__ __forceinline__ int xcd_tile(int b, const RViews& RV) {
  const int x = b % kXcds, idx = b / kXcds;
  int k = 0;
  for (int j = 1; j < RV.n_views; ++j) k = (RV.xcd_off[x][j] <= idx) ? j : k;
  return RV.tile_base[RV.order[k]] + RV.xcd_start[x][k] + (idx - RV.xcd_off[x][k]);
}

// The inverse of xcd_tile: the XCD whose share holds global tile t and the
// tile's index in that XCD's walk (block = index * 8 + XCD).
__host__ __device__ __forceinline__ int xcd_of_tile(int t, const RViews& RV, int& idx) {
  int v = 0;
  for (int k = 1; k < RV.n_views; ++k) v = (RV.tile_base[k] <= t) ? k : v;
  int pos = 0;
  for (int k = 0; k < RV.n_views; ++k) pos = (RV.order[k] == v) ? k : pos;
  const int l = t - RV.tile_base[v];
  // a view's shares are contiguous in XCD order; the last one starting at or
  // before l holds it (an empty share starts where the next one does, and the
  // last XCD's share starts before the view's end only when it is not empty)
  int x = 0;
  for (int j = 1; j < kXcds; ++j) x = (RV.xcd_start[j][pos] <= l) ? j : x;
  idx = RV.xcd_off[x][pos] + (l - RV.xcd_start[x][pos]);
  return x;
}

// The backward's balanced tile order.  Within each XCD's share (the tiles
// xcd_tile gives it, so neighbouring tiles still meet in one L2), tiles
// ranked by list length (rank 0 the heaviest) are dealt to the XCD's blocks
// in rounds of kOrderRound / 8, every other complete round reversed, so that
// blocks b and b + kOrderRound (which the round-robin dispatch places on the
// same SIMDs) pair a heavy tile with a light one.  Index in the XCD's walk of
// rank r among its n tiles; a bijection on [0, n).
constexpr int kOrderRound = 256;
constexpr int kXcdRound = kOrderRound / kXcds;

__host__ __device__ __forceinline__ int order_block(int r, int n, int round_len = kXcdRound) {
  const int full = n / round_len;  // complete rounds
  const int round = r / round_len, j = r - round * round_len;
  return (round < full && (round & 1)) ? round * round_len + (round_len - 1 - j) : r;
}

// List-parallel blending, for launches with few tiles: when the whole launch
// has fewer than kFewTiles tiles (a low-resolution view on its own), lists
// longer than kLongList go to the list-parallel kernels (tiles of 8 and 16
// pixels; the forward and the backward use the same rule, so both take the
// same path for a tile).  A wave walking a list alone on its SIMD costs about
// 0.4 us per entry, and with few tiles nothing else runs meanwhile.  A launch
// with more tiles (a full-resolution view, or a batch of views) fills the chip
// with tiles alone; its longest lists start first (views are walked fewest
// tiles first), and splitting them only adds the list-parallel passes' extra
// work, so such launches skip the long-list kernels altogether.
constexpr uint32_t kLongList = 48;
constexpr int kFewTiles = 2048;

__host__ __device__ inline bool split_long_lists(const RViews& RV, int tile) {
  return tile <= 16 && RV.total_tiles < kFewTiles;
}

template <int TILE>
__device__ __forceinline__ uint32_t long_list_threshold(const RViews&, int) {
  return kLongList;
}

// global tile id -> view (views are few; the loop runs on the scalar unit)
__device__ __forceinline__ int view_of_tile(const RViews& RV, int t) {
  int v = 0;
  for (int k = 1; k < RV.n_views; ++k) v = (RV.tile_base[k] <= t) ? k : v;
  return v;
}

// The record's mean is relative to the origin of the footprint's first tile;
// move it to the frame of tile (tx, ty) so pixel offsets stay small numbers.
template <int TILE>
__device__ __forceinline__ float4 to_tile_frame(float4 r0, uint32_t lo, int tx, int ty) {
  r0.x += float((box_x(lo) / TILE - tx) * TILE);
  r0.y += float((box_y(lo) / TILE - ty) * TILE);
  return r0;
}

// Bit g set when the footprint box [lo, hi] touches 8x8 group g of tile (tx, ty).
template <int TILE>
__device__ __forceinline__ uint32_t group_mask(uint32_t lo, uint32_t hi, int tx, int ty) {
  constexpr int GX = TILE / 8;
  // box in group units relative to the tile, clamped to the tile's groups
  const int gx0 = max((box_x(lo) - tx * TILE) >> 3, 0);
  const int gx1 = min((box_x(hi) - tx * TILE) >> 3, GX - 1);
  const int gy0 = max((box_y(lo) - ty * TILE) >> 3, 0);
  const int gy1 = min((box_y(hi) - ty * TILE) >> 3, GX - 1);
  if (gx0 > gx1 || gy0 > gy1) return 0u;
  const uint32_t row = ((1u << (gx1 + 1)) - 1u) & ~((1u << gx0) - 1u);
  uint32_t m = 0u;
#pragma unroll
  for (int gy = 0; gy < GX; ++gy)
    if (gy >= gy0 && gy <= gy1) m |= row << (gy * GX);
  return m;
}

}  // namespace gsk
