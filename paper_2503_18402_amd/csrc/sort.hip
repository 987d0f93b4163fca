// Binning: one (tile, Gaussian) pair per tile of every visible footprint,
// grouped by tile, ordered within a tile by (depth, Gaussian index), plus the
// per-tile ranges.
//
// That order is the one of the stable ascending sort of
// key = (tile_id << 32) | bits(depth_f32) over pairs emitted in Gaussian index
// order.  Because the index breaks every tie, the order is unique, so any
// correct sort produces it.  Instead of sorting all pairs globally on every key
// digit, the pairs are bucketed by tile and each tile's (short) list is sorted
// on chip:
//   0. offsets: each pair's position in index order (Gaussian by Gaussian,
//              tiles row-major in its box) from a scan of the tile counts;
//   1. count:  one atomic increment per pair on its tile's counter; the
//              value it returns is the pair's rank in its tile, kept at the
//              pair's index-order position;
//   2. scan:   one block scans the counters into each tile's first slot and
//              checks the pair total against the capacity;
//   3. bucket: every pair stores the 64-bit sort key
//              (bits(depth_f32) << 32) | Gaussian index at its tile's first
//              slot plus its rank: no atomics;
//   4. sort:   each tile's keys are sorted by a bitonic network and the
//              values written (and the keys when asked for): lists of up to
//              512 keys by one wave in registers, up to 2048 by a 256-thread
//              block in registers with LDS exchanges for the strides that
//              cross waves, longer ones by a 1024-thread block in LDS (lists
//              longer than one LDS chunk also run the network's long strides
//              through global memory).
// The slot order after step 3 depends on atomic timing; after step 4 it does
// not.  A block whose pairs fall on at most 2048 tiles it can index (all tiles
// of its views at low resolutions, where every tile collects thousands of
// pairs; or the bounding rectangle of its footprints' tiles, when its
// Gaussians sit close together in space) counts in LDS first and reserves one
// slot range per touched tile in step 3 instead, through a cursor that starts
// after the tile's ranked pairs.  The counters, cursors and first slots live in
// the caller's ranges array (during steps 1-3: ranges[2t] = ranked count, then
// first slot; ranges[2t+1] = LDS-counted count, then cursor, then end), so the
// workspace holds the bucketed keys, the ranks, the offsets' block sums and
// four counts.
//
// The pair expansion spreads each wave's pairs evenly over its 64 lanes, so a
// Gaussian with a footprint of thousands of tiles does not serialise on one lane.
#include <algorithm>
#include <mutex>

#include "scan.hpp"

namespace gsk {
namespace {

struct TileInfo {  // per view: first global tile, one past its last tile, grid width
  int32_t tile_base[GS_MAX_VIEWS];
  int32_t tile_end[GS_MAX_VIEWS];
  int32_t gw[GS_MAX_VIEWS];
};

struct Items {  // the (view, Gaussian) items of a preprocess output
  TileInfo TI;
  const char* proj;
  size_t stride, tt_off;
  char* goff_proj;  // non-null: record each item's first pair position (at goff_off)
  size_t goff_off;
  int64_t m;  // n_views * n
  int n, tile;
};

constexpr int kXT = 256;        // threads per expansion block
constexpr int kAggBins = 2048;  // most tiles a block aggregates in LDS
constexpr int kAggRounds = 8;   // items per aggregating block: at most kXT * kAggRounds
// but no fewer blocks than this while items allow: each block walks its rounds
// one after the other (load, scan, LDS bins), so 2048 blocks (8 per CU) hide
// that latency; at 1M Gaussians on views of a few hundred tiles, 512 blocks
// took 1.8-2.3x as long when the Gaussians are stored in spatial order (blocks
// touch few tiles), while in index order (every block touches most tiles) the
// 4x more reservation atomics cost 1.4x
constexpr int kAggBlocks = 2048;

// Calls f(global tile id, sort key, index-order position, tile x | tile y << 16
// in its view's grid) once for every pair of the items [first, first + kXT),
// whose first pair sits at index-order position pbase.  Every thread of the
// block must call it.  Returns the items' pair count.
template <class F>
__device__ inline uint32_t for_each_pair(const Items& S, int64_t first, uint32_t pbase, F&& f) {
  __shared__ uint32_t s_end[kXT];   // inclusive prefix of pair counts within the wave
  __shared__ uint32_t s_wtot[kXT / 64];
  __shared__ uint32_t s_base[kXT];  // global id of the footprint's first tile
  __shared__ uint32_t s_w[kXT];     // footprint width in tiles
  __shared__ uint32_t s_gw[kXT];    // tile-grid width of the item's view
  __shared__ uint64_t s_key[kXT];   // bits(depth) << 32 | Gaussian index
  __shared__ uint32_t s_xy[kXT];    // footprint's first tile: x | y << 16
  const int lane = threadIdx.x & 63, w0 = threadIdx.x & ~63;
  const int64_t i = first + threadIdx.x;
  uint32_t cnt = 0, base = 0, w = 1, gw = 1, xy = 0;
  uint64_t key = 0;
  if (i < S.m) {
    const int64_t v = i / S.n, g = i - v * S.n;
    const char* pv = S.proj + size_t(v) * S.stride;
    if (reinterpret_cast<const uint32_t*>(pv + S.tt_off)[g] > 0u) {
      const float4 r2 = reinterpret_cast<const float4*>(pv)[3 * g + 2];
      const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
      const int tx0 = box_x(lo) / S.tile, ty0 = box_y(lo) / S.tile;
      const int tx1 = box_x(hi) / S.tile, ty1 = box_y(hi) / S.tile;
      w = uint32_t(tx1 - tx0 + 1);
      cnt = w * uint32_t(ty1 - ty0 + 1);
      gw = uint32_t(S.TI.gw[v]);
      base = uint32_t(S.TI.tile_base[v]) + uint32_t(ty0) * gw + uint32_t(tx0);
      xy = uint32_t(tx0) | (uint32_t(ty0) << 16);
      key = (uint64_t(__float_as_uint(r2.y)) << 32) | uint64_t(g);
    }
  }
  const uint32_t inc = wave_incl_scan(cnt);
  if (lane == 63) s_wtot[threadIdx.x >> 6] = inc;
  s_end[threadIdx.x] = inc;
  s_base[threadIdx.x] = base;
  s_w[threadIdx.x] = w;
  s_gw[threadIdx.x] = gw;
  s_key[threadIdx.x] = key;
  s_xy[threadIdx.x] = xy;
  __syncthreads();
  const uint32_t total = __shfl(inc, 63, 64);
  uint32_t wbase = pbase, all = 0;
#pragma unroll
  for (int w = 0; w < kXT / 64; ++w) {
    const uint32_t t = s_wtot[w];
    wbase += (w < (threadIdx.x >> 6)) ? t : 0u;
    all += t;
  }
  if (S.goff_proj && i < S.m) {
    const int64_t v = i / S.n, g = i - v * S.n;
    reinterpret_cast<uint32_t*>(S.goff_proj + size_t(v) * S.stride + S.goff_off)[g] =
        wbase + (inc - cnt);
  }
  for (uint32_t j = uint32_t(lane); j < total; j += 64) {
    // the item owning the wave's j-th pair: the first k with s_end[k] > j
    int k = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
      if (s_end[w0 + k + step - 1] <= j) k += step;
    const uint32_t local = j - (k > 0 ? s_end[w0 + k - 1] : 0u);
    const uint32_t wk = s_w[w0 + k];
    const uint32_t ty = local / wk, tx = local - ty * wk;
    f(s_base[w0 + k] + ty * s_gw[w0 + k] + tx, s_key[w0 + k], wbase + j,
      s_xy[w0 + k] + tx + (ty << 16));
  }
  __syncthreads();  // the arrays are rewritten by the next call
  return all;
}

// Pair count of each block's items (the block decomposition of k_tile_count
// and k_bucket); k_scan_spine then turns them into each block's first
// index-order position.
__global__ __launch_bounds__(kXT) void k_tile_reduce(Items S, int rounds,
                                                     uint32_t* __restrict__ block_pairs) {
  __shared__ uint32_t s_w[kXT / 64];
  const int64_t i0 = int64_t(blockIdx.x) * kXT * rounds;
  uint32_t acc = 0;
  for (int r = 0; r < rounds; ++r) {
    const int64_t i = i0 + int64_t(r) * kXT + threadIdx.x;
    if (i < S.m) {
      const int64_t v = i / S.n, g = i - v * S.n;
      acc += reinterpret_cast<const uint32_t*>(S.proj + size_t(v) * S.stride + S.tt_off)[g];
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc += uint32_t(__shfl_xor(int(acc), d, 64));
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kXT / 64; ++w) t += s_w[w];
    block_pairs[blockIdx.x] = t;
  }
}

// A block takes kXT * rounds consecutive items.  It counts its pairs per tile
// in LDS first and issues one global atomic per touched tile when its pairs
// fall on at most agg_bins tiles that it can index:
//   - all tiles of the views its items belong to (low resolutions, where
//     every tile collects thousands of pairs and same-counter atomics
//     serialise), bin = tile - first tile of those views; or
//   - for items of one view, the bounding rectangle of their footprints'
//     tiles (Gaussians stored close together in space, as the spatial order
//     stores them, cover few tiles), bin = row-major cell of that rectangle.
// Otherwise every pair goes to the global counters and ranks itself there.
struct BlockSpan {
  int64_t i0, i1;    // items
  int32_t mode;      // 0: global counters, 1: the views' tiles, 2: the rectangle
  int32_t t_lo;      // mode 1: first tile of the block's views
  int32_t bx0, by0, bw, gw, base;  // mode 2: rectangle origin and width; view grid
  int32_t span;      // bins in use
  __device__ int bin(uint32_t t, uint32_t xy) const {
    return mode == 1 ? int(t) - t_lo
                     : (int(xy >> 16) - by0) * bw + (int(xy & 0xffffu) - bx0);
  }
  __device__ uint32_t tile_of(int b) const {
    if (mode == 1) return uint32_t(t_lo + b);
    const int y = b / bw, x = b - y * bw;
    return uint32_t(base + (by0 + y) * gw + bx0 + x);
  }
};

// every thread of the block must call it
__device__ inline BlockSpan block_span(const Items& S, int rounds, int agg_bins) {
  BlockSpan b{};
  b.i0 = int64_t(blockIdx.x) * kXT * rounds;
  b.i1 = (b.i0 + int64_t(kXT) * rounds < S.m) ? b.i0 + int64_t(kXT) * rounds : S.m;
  const int v0 = int(b.i0 / S.n), v1 = int((b.i1 - 1) / S.n);
  b.t_lo = S.TI.tile_base[v0];
  b.span = S.TI.tile_end[v1] - b.t_lo;
  b.mode = b.span <= agg_bins ? 1 : 0;
  if (b.mode == 1 || v0 != v1 || agg_bins == 0) return b;  // block-uniform
  // the tile rectangle of the block's footprints
  int x0 = 1 << 30, y0 = 1 << 30, x1 = -1, y1 = -1;
  const char* pv = S.proj + size_t(v0) * S.stride;
  for (int64_t i = b.i0 + threadIdx.x; i < b.i1; i += kXT) {
    const int64_t g = i - int64_t(v0) * S.n;
    if (reinterpret_cast<const uint32_t*>(pv + S.tt_off)[g] > 0u) {
      const float4 r2 = reinterpret_cast<const float4*>(pv)[3 * g + 2];
      const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
      x0 = min(x0, box_x(lo) / S.tile);
      y0 = min(y0, box_y(lo) / S.tile);
      x1 = max(x1, box_x(hi) / S.tile);
      y1 = max(y1, box_y(hi) / S.tile);
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    x0 = min(x0, __shfl_xor(x0, d, 64));
    y0 = min(y0, __shfl_xor(y0, d, 64));
    x1 = max(x1, __shfl_xor(x1, d, 64));
    y1 = max(y1, __shfl_xor(y1, d, 64));
  }
  __shared__ int s_r[4][kXT / 64];
  if ((threadIdx.x & 63) == 0) {
    s_r[0][threadIdx.x >> 6] = x0;
    s_r[1][threadIdx.x >> 6] = y0;
    s_r[2][threadIdx.x >> 6] = x1;
    s_r[3][threadIdx.x >> 6] = y1;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kXT / 64; ++w) {
    x0 = min(x0, s_r[0][w]);
    y0 = min(y0, s_r[1][w]);
    x1 = max(x1, s_r[2][w]);
    y1 = max(y1, s_r[3][w]);
  }
  __syncthreads();  // s_r is rewritten by the next call
  if (x1 >= x0 && int64_t(x1 - x0 + 1) * (y1 - y0 + 1) <= agg_bins) {
    b.mode = 2;
    b.bx0 = x0;
    b.by0 = y0;
    b.bw = x1 - x0 + 1;
    b.gw = S.TI.gw[v0];
    b.base = S.TI.tile_base[v0];
    b.span = b.bw * (y1 - y0 + 1);
  }
  return b;
}

// The counter an LDS-counting block reserves through for global tile t: with
// `copies` (launches of at most kAggBins tiles, where the same few hundred
// counters receive one atomic from nearly every block) one of kXcds copies,
// chosen by the block, so each copy sees an eighth of those atomics; else the
// tile's ranges[2t + 1].
__device__ __forceinline__ uint32_t* agg_counter(uint32_t* ranges, uint32_t* copies, uint32_t t) {
  return copies ? copies + (blockIdx.x % kXcds) * kAggBins + t : ranges + 2 * size_t(t) + 1;
}

__global__ __launch_bounds__(kXT) void k_tile_count(Items S, int rounds, int agg_bins,
                                                    const uint32_t* __restrict__ block_pos,
                                                    int64_t cap, uint32_t* __restrict__ ranges,
                                                    uint32_t* __restrict__ rank,
                                                    uint32_t* __restrict__ copies) {
  extern __shared__ uint32_t s_bins[];
  const BlockSpan B = block_span(S, rounds, agg_bins);
  if (B.mode) {
    for (int b = threadIdx.x; b < B.span; b += kXT) s_bins[b] = 0u;
    __syncthreads();
    uint32_t pos = block_pos[blockIdx.x];  // for the items' pair offsets
    for (int64_t c = B.i0; c < B.i1; c += kXT)
      pos += for_each_pair(S, c, pos, [&](uint32_t t, uint64_t, uint32_t, uint32_t xy) {
        atomicAdd(&s_bins[B.bin(t, xy)], 1u);
      });
    for (int b = threadIdx.x; b < B.span; b += kXT)
      if (s_bins[b]) atomicAdd(agg_counter(ranges, copies, B.tile_of(b)), s_bins[b]);
  } else {
    // the returned count is the pair's rank among its tile's ranked pairs
    uint32_t pos = block_pos[blockIdx.x];
    for (int64_t c = B.i0; c < B.i1; c += kXT)
      pos += for_each_pair(S, c, pos, [&](uint32_t t, uint64_t, uint32_t p, uint32_t) {
        const uint32_t r = atomicAdd(&ranges[2 * size_t(t)], 1u);
        if (int64_t(p) < cap) rank[p] = r;
      });
  }
}

// Places every pair's key in its tile's bucket: a ranked pair at the tile's
// first slot plus its rank; with LDS bins the block first reserves one
// contiguous slot range per touched tile from the tile's cursor (which starts
// after the ranked pairs), then ranks its pairs inside it with LDS atomics.
__global__ __launch_bounds__(kXT) void k_bucket(Items S, int rounds, int agg_bins,
                                                const int64_t* __restrict__ n_eff,
                                                const uint32_t* __restrict__ block_pos,
                                                const uint32_t* __restrict__ rank,
                                                uint32_t* __restrict__ ranges,
                                                uint32_t* __restrict__ copies,
                                                uint64_t* __restrict__ bucket) {
  extern __shared__ uint32_t s_bins[];
  if (*n_eff == 0) return;  // capacity overflow (or no pairs): nothing to place
  const BlockSpan B = block_span(S, rounds, agg_bins);
  if (B.mode) {
    for (int b = threadIdx.x; b < B.span; b += kXT) s_bins[b] = 0u;
    __syncthreads();
    for (int64_t c = B.i0; c < B.i1; c += kXT)
      for_each_pair(S, c, 0u, [&](uint32_t t, uint64_t, uint32_t, uint32_t xy) {
        atomicAdd(&s_bins[B.bin(t, xy)], 1u);
      });
    // a thread's bins are b = t + u kXT, u < kAggBins / kXT: all their
    // reservation atomics are issued before the first result is used, so the
    // returns' latencies overlap
    constexpr int kU = kAggBins / kXT;
    uint32_t got[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = int(threadIdx.x) + u * kXT;
      const uint32_t k = b < B.span ? s_bins[b] : 0u;
      got[u] = k ? atomicAdd(agg_counter(ranges, copies, B.tile_of(b)), k) : 0u;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = int(threadIdx.x) + u * kXT;
      if (b < B.span && s_bins[b]) s_bins[b] = got[u];
    }
    __syncthreads();
    for (int64_t c = B.i0; c < B.i1; c += kXT)
      for_each_pair(S, c, 0u, [&](uint32_t t, uint64_t key, uint32_t, uint32_t xy) {
        bucket[atomicAdd(&s_bins[B.bin(t, xy)], 1u)] = key;
      });
  } else {
    uint32_t pos = block_pos[blockIdx.x];
    for (int64_t c = B.i0; c < B.i1; c += kXT)
      pos += for_each_pair(S, c, pos, [&](uint32_t t, uint64_t key, uint32_t p, uint32_t) {
        bucket[ranges[2 * size_t(t)] + rank[p]] = key;
      });
  }
}

// One block: with c_t = ranges[2t] (ranked pairs) + the pairs of LDS-counting
// blocks (ranges[2t+1], or the sum of the tile's kXcds counter copies),
// ranges[2t] = exclusive prefix of c (the tile's first slot) and ranges[2t+1]
// = that prefix plus the ranked pairs (where the LDS-counting blocks' cursor
// starts; with copies, copy x's cursor starts after copies 0..x-1's pairs);
// the pair total, and whether it fits the capacity.  Sums are 64-bit, so an
// overflowing total is always detected.
constexpr int kTS = 1024;
constexpr int kTSItems = 8;

__device__ inline uint64_t wave_incl_scan64(uint64_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

__global__ __launch_bounds__(kTS) void k_tile_scan(uint32_t* __restrict__ ranges,
                                                   uint32_t* __restrict__ copies, int n_tiles,
                                                   int64_t* __restrict__ proj_total,
                                                   int64_t cap, int64_t* __restrict__ n_tot,
                                                   int64_t* __restrict__ n_eff,
                                                   int64_t* __restrict__ n_long,
                                                   int64_t* __restrict__ n_mid,
                                                   int64_t* __restrict__ n_pairs_user) {
  __shared__ uint64_t s_w[kTS / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t carry = 0;
  for (int base = 0; base < n_tiles; base += kTS * kTSItems) {
    const int i0 = base + threadIdx.x * kTSItems;
    uint32_t c[kTSItems], cr[kTSItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kTSItems; ++k) {
      cr[k] = (i0 + k < n_tiles) ? ranges[2 * size_t(i0 + k)] : 0u;
      uint32_t agg = 0u;
      if (i0 + k < n_tiles) {
        if (copies) {
#pragma unroll
          for (int x = 0; x < kXcds; ++x) agg += copies[x * kAggBins + i0 + k];
        } else {
          agg = ranges[2 * size_t(i0 + k) + 1];
        }
      }
      c[k] = cr[k] + agg;
      s += c[k];
    }
    const uint64_t inc = wave_incl_scan64(s);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint64_t before = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kTS / 64; ++q) {
      const uint64_t t = s_w[q];
      before += (q < wv) ? t : 0u;
      tot += t;
    }
    __syncthreads();
    uint64_t ex = carry + before + inc - s;
#pragma unroll
    for (int k = 0; k < kTSItems; ++k) {
      if (i0 + k < n_tiles) {
        ranges[2 * size_t(i0 + k)] = uint32_t(ex);
        ranges[2 * size_t(i0 + k) + 1] = uint32_t(ex + cr[k]);
        if (copies) {
          uint32_t cur = uint32_t(ex + cr[k]);
#pragma unroll
          for (int x = 0; x < kXcds; ++x) {
            const uint32_t a = copies[x * kAggBins + i0 + k];
            copies[x * kAggBins + i0 + k] = cur;
            cur += a;
          }
        }
      }
      ex += c[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    const int64_t t = int64_t(carry);
    *n_tot = t;
    if (proj_total) *proj_total = t;
    *n_eff = (t <= cap) ? t : 0;
    *n_pairs_user = t;
    *n_long = 0;  // set by the wave sort for lists it leaves to the larger tiers
    *n_mid = 0;
  }
}

// ---- bitonic network without directions: every step puts the smaller key at
// the lower index.  A merge of block size 2h starts with a mirror step
// (i, i ^ (2h - 1)) and continues with plain steps (i, i + d), d = h/2 .. 1.
// Keys at indices >= n act as +infinity: every step with a partner >= n would
// leave it in place, so they are neither stored nor compared.
__device__ inline void step_pair(uint32_t c, uint32_t h, bool mirror, uint32_t& i, uint32_t& l) {
  i = ((c & ~(h - 1)) << 1) | (c & (h - 1));
  l = mirror ? ((i | (2 * h - 1)) - (c & (h - 1))) : (i + h);
}

template <int THREADS>
__device__ inline void net_step(uint64_t* a, uint32_t n, uint32_t half_len, uint32_t h,
                                bool mirror) {
  for (uint32_t c = threadIdx.x; c < half_len; c += THREADS) {
    uint32_t i, l;
    step_pair(c, h, mirror, i, l);
    if (l < n) {
      const uint64_t x = a[i], y = a[l];
      if (y < x) {
        a[i] = y;
        a[l] = x;
      }
    }
  }
  __syncthreads();
}

// full sort of a[0, n) (n <= len, len a power of two) in LDS
template <int THREADS>
__device__ inline void lds_sort(uint64_t* a, uint32_t n, uint32_t len) {
  for (uint32_t h = 1; h < len; h <<= 1) {
    net_step<THREADS>(a, n, len / 2, h, true);
    for (uint32_t d = h >> 1; d > 0; d >>= 1) net_step<THREADS>(a, n, len / 2, d, false);
  }
}

__device__ inline uint32_t pow2_ceil(uint32_t x) {
  return x <= 1u ? 1u : (1u << (32 - __builtin_clz(x - 1u)));
}

template <int THREADS>
__device__ inline void write_sorted(const uint64_t* a, uint32_t n, uint32_t start, uint32_t t,
                                    uint32_t* __restrict__ vals, uint64_t* __restrict__ keys) {
  for (uint32_t i = threadIdx.x; i < n; i += THREADS) {
    const uint64_t k = a[i];
    vals[start + i] = uint32_t(k);
    if (keys) keys[start + i] = (uint64_t(t) << 32) | (k >> 32);
  }
}

// ---- lists of at most kWaveKeys keys: one wave per tile, 8 keys per lane in
// registers (element 8 lane + r in k[r]), padded with +infinity to a power of
// two; the same direction-free network with in-lane steps for strides below 8
// and lane shuffles above, so no LDS and no barriers.
constexpr int kWaveKeys = 512;
constexpr int kSmall = 2048;

__device__ __forceinline__ void cx(uint64_t& a, uint64_t& b) {
  const uint64_t x = a < b ? a : b, y = a < b ? b : a;
  a = x;
  b = y;
}

// lane l reads lane l ^ M.  Within a row of 16 lanes the exchange runs on the
// DPP path of the VALU (xor 1, 2, 3: quad permutes; 7, 15: half-row and row
// mirrors), within 32 lanes as a swizzle (xor 4, 8, 16, 31), otherwise as a
// permute through the LDS crossbar
template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t x) {
  const int v = int(x);
  if constexpr (M == 1) return uint32_t(__builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true));
  else if constexpr (M == 2) return uint32_t(__builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true));
  else if constexpr (M == 3) return uint32_t(__builtin_amdgcn_update_dpp(0, v, 0x1B, 0xF, 0xF, true));
  else if constexpr (M == 7) return uint32_t(__builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true));
  else if constexpr (M == 15) return uint32_t(__builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true));
  else if constexpr (M < 32) return uint32_t(__builtin_amdgcn_ds_swizzle(v, (M << 10) | 0x1F));
  else return uint32_t(__shfl_xor(v, M, 64));
}

template <int M>
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t x) {
  const uint32_t lo = xor_lane<M>(uint32_t(x));
  const uint32_t hi = xor_lane<M>(uint32_t(x >> 32));
  return (uint64_t(hi) << 32) | lo;
}

// lanes whose stride bit is clear hold the lower element and keep the minimum
template <int M>
__device__ __forceinline__ void cross_step_m(uint64_t (&k)[8], bool lower, bool mirror) {
  uint64_t p[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) p[r] = shfl_xor64<M>(k[mirror ? 7 - r : r]);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const bool lt = p[r] < k[r];
    k[r] = (lower == lt) ? p[r] : k[r];
  }
}

// the same step with a runtime mask, every exchange through the LDS crossbar
// (the block-wide network below measured faster with it than with the
// dispatch over exchange paths)
__device__ __forceinline__ void cross_step_perm(uint64_t (&k)[8], int mask, bool lower,
                                                bool mirror) {
  uint64_t p[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint64_t x = k[mirror ? 7 - r : r];
    const uint32_t lo = uint32_t(__shfl_xor(int(uint32_t(x)), mask, 64));
    const uint32_t hi = uint32_t(__shfl_xor(int(uint32_t(x >> 32)), mask, 64));
    p[r] = (uint64_t(hi) << 32) | lo;
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const bool lt = p[r] < k[r];
    k[r] = (lower == lt) ? p[r] : k[r];
  }
}

// the lane masks the networks use: 2^j for plain steps, 2^j - 1 for mirrors
__device__ __forceinline__ void cross_step(uint64_t (&k)[8], int mask, bool lower, bool mirror) {
  switch (mask) {  // wave-uniform
    case 1: cross_step_m<1>(k, lower, mirror); break;
    case 2: cross_step_m<2>(k, lower, mirror); break;
    case 3: cross_step_m<3>(k, lower, mirror); break;
    case 4: cross_step_m<4>(k, lower, mirror); break;
    case 7: cross_step_m<7>(k, lower, mirror); break;
    case 8: cross_step_m<8>(k, lower, mirror); break;
    case 15: cross_step_m<15>(k, lower, mirror); break;
    case 16: cross_step_m<16>(k, lower, mirror); break;
    case 31: cross_step_m<31>(k, lower, mirror); break;
    case 32: cross_step_m<32>(k, lower, mirror); break;
    default: cross_step_m<63>(k, lower, mirror); break;
  }
}

__device__ inline void wave_sort(uint64_t (&k)[8], uint32_t len) {
  const int lane = threadIdx.x & 63;
  for (uint32_t h = 1; h < len; h <<= 1) {
    if (h == 1) {
      cx(k[0], k[1]); cx(k[2], k[3]); cx(k[4], k[5]); cx(k[6], k[7]);
    } else if (h == 2) {
      cx(k[0], k[3]); cx(k[1], k[2]); cx(k[4], k[7]); cx(k[5], k[6]);
    } else if (h == 4) {
      cx(k[0], k[7]); cx(k[1], k[6]); cx(k[2], k[5]); cx(k[3], k[4]);
    } else {
      cross_step(k, int(2 * h / 8 - 1), (lane & int(h / 8)) == 0, true);
    }
    for (uint32_t d = h >> 1; d > 0; d >>= 1) {
      if (d >= 8) {
        cross_step(k, int(d / 8), (lane & int(d / 8)) == 0, false);
      } else if (d == 4) {
        cx(k[0], k[4]); cx(k[1], k[5]); cx(k[2], k[6]); cx(k[3], k[7]);
      } else if (d == 2) {
        cx(k[0], k[2]); cx(k[1], k[3]); cx(k[4], k[6]); cx(k[5], k[7]);
      } else {
        cx(k[0], k[1]); cx(k[2], k[3]); cx(k[4], k[5]); cx(k[6], k[7]);
      }
    }
  }
}

// The same network over W waves of a block, 8 keys per lane: element
// e = 512 w + 8 lane + r of the block's 512 W keys.  Strides below 8 run
// in-lane and strides below 512 by lane shuffles, as in wave_sort; longer
// ones exchange through LDS (s holds 512 W keys), two barriers each.  Every
// thread of the block must call it with the same len (a power of two, at most
// 512 W); keys at e >= len must be +infinity.
template <int W>
__device__ inline void block_reg_sort(uint64_t (&k)[8], uint32_t len, uint64_t* s) {
  const int lane = threadIdx.x & 63;
  const uint32_t e0 = 512u * uint32_t(threadIdx.x >> 6) + 8u * uint32_t(lane);
  // a wave whose keys all sit at e >= len holds only +infinity, which every
  // step leaves in place (partners of such keys are such keys): it only
  // keeps the barriers
  const bool idle = 512u * uint32_t(threadIdx.x >> 6) >= len;
  // partner e ^ m; the element whose bit hb is clear keeps the minimum
  auto lds_step = [&](uint32_t m, uint32_t hb) {
    if (!idle) {
#pragma unroll
      for (int r = 0; r < 8; ++r) s[e0 + r] = k[r];
    }
    __syncthreads();
    if (!idle) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const uint32_t e = e0 + uint32_t(r);
        const uint64_t p = s[e ^ m];
        const bool lower = (e & hb) == 0u;
        const bool lt = p < k[r];
        k[r] = (lower == lt) ? p : k[r];
      }
    }
    __syncthreads();
  };
  for (uint32_t h = 1; h < len; h <<= 1) {
    if (h >= 512u) {
      lds_step(2 * h - 1, h);
    } else if (!idle) {
      if (h == 1) {
        cx(k[0], k[1]); cx(k[2], k[3]); cx(k[4], k[5]); cx(k[6], k[7]);
      } else if (h == 2) {
        cx(k[0], k[3]); cx(k[1], k[2]); cx(k[4], k[7]); cx(k[5], k[6]);
      } else if (h == 4) {
        cx(k[0], k[7]); cx(k[1], k[6]); cx(k[2], k[5]); cx(k[3], k[4]);
      } else {
        cross_step_perm(k, int(2 * h / 8 - 1), (lane & int(h / 8)) == 0, true);
      }
    }
    for (uint32_t d = h >> 1; d > 0; d >>= 1) {
      if (d >= 512u) {
        lds_step(d, d);
      } else if (idle) {
      } else if (d >= 8u) {
        cross_step_perm(k, int(d / 8), (lane & int(d / 8)) == 0, false);
      } else if (d == 4) {
        cx(k[0], k[4]); cx(k[1], k[5]); cx(k[2], k[6]); cx(k[3], k[7]);
      } else if (d == 2) {
        cx(k[0], k[2]); cx(k[1], k[3]); cx(k[4], k[6]); cx(k[5], k[7]);
      } else {
        cx(k[0], k[1]); cx(k[2], k[3]); cx(k[4], k[5]); cx(k[6], k[7]);
      }
    }
  }
}

// A tile's list of n <= 512 W keys sorted by block_reg_sort and written out.
template <int W>
__device__ inline void sort_list_regs(const uint64_t* __restrict__ bucket, uint32_t start,
                                      uint32_t n, uint32_t t, uint64_t* s,
                                      uint32_t* __restrict__ vals, uint64_t* __restrict__ keys) {
  const uint32_t e0 = 512u * uint32_t(threadIdx.x >> 6) + 8u * uint32_t(threadIdx.x & 63);
  uint64_t k[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t e = e0 + uint32_t(r);
    k[r] = (e < n) ? bucket[start + e] : ~uint64_t(0);
  }
  block_reg_sort<W>(k, pow2_ceil(n), s);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t e = e0 + uint32_t(r);
    if (e < n) {
      vals[start + e] = uint32_t(k[r]);
      if (keys) keys[start + e] = (uint64_t(t) << 32) | (k[r] >> 32);
    }
  }
}

// One wave per tile, four tiles per block.  Also writes every tile's range end
// (or [0,0) everywhere after a capacity overflow) and flags the presence of
// lists for the two larger tiers.
__global__ __launch_bounds__(256) void k_tile_sort_wave(
    int n_tiles, const int64_t* __restrict__ n_tot, const int64_t* __restrict__ n_eff,
    int64_t* __restrict__ n_mid, int64_t* __restrict__ n_long,
    const uint64_t* __restrict__ bucket, uint32_t* __restrict__ vals,
    uint64_t* __restrict__ keys, uint32_t* __restrict__ ranges) {
  const int lane = threadIdx.x & 63;
  const uint32_t t = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (t >= uint32_t(n_tiles)) return;  // wave-uniform; no block barrier below
  if (*n_eff == 0) {
    if (lane == 0) {
      ranges[2 * size_t(t)] = 0u;
      ranges[2 * size_t(t) + 1] = 0u;
    }
    return;
  }
  // each wave writes only its own range end (the cursor has counted down to the
  // first slot); the next tile's first slot stays
  const uint32_t start = ranges[2 * size_t(t)];
  const uint32_t end = (t + 1 < uint32_t(n_tiles)) ? ranges[2 * size_t(t) + 2] : uint32_t(*n_tot);
  if (lane == 0) ranges[2 * size_t(t) + 1] = end;
  const uint32_t n = end - start;
  if (n > uint32_t(kWaveKeys)) {
    if (lane == 0) *(n > uint32_t(kSmall) ? n_long : n_mid) = 1;
    return;
  }
  if (n == 0) return;
  uint64_t k[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t i = 8u * lane + r;
    k[r] = (i < n) ? bucket[start + i] : ~uint64_t(0);
  }
  wave_sort(k, n <= 8u ? 8u : pow2_ceil(n));
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const uint32_t i = 8u * lane + r;
    if (i < n) {
      vals[start + i] = uint32_t(k[r]);
      if (keys) keys[start + i] = (uint64_t(t) << 32) | (k[r] >> 32);
    }
  }
}

// Lists of kWaveKeys+1 .. kSmall keys: 256-thread blocks striding over the
// tiles, 8 keys per lane in registers (block_reg_sort: LDS only for the
// strides that cross waves; 0.046 -> 0.029 ms against the network in LDS at
// 1M Gaussians, 200x133, tile 8).  Up to 2048 blocks: at 400x266 (1700 tiles)
// every tile then has its own block (binning 161 -> 153 us against 1024 blocks).
constexpr int kMidThreads = 256;
constexpr int kMidBlocks = 2048;

__global__ __launch_bounds__(kMidThreads) void k_tile_sort_mid(
    int n_tiles, const int64_t* __restrict__ n_eff, const int64_t* __restrict__ n_mid,
    const uint64_t* __restrict__ bucket, uint32_t* __restrict__ vals,
    uint64_t* __restrict__ keys, const uint32_t* __restrict__ ranges) {
  __shared__ uint64_t s[kSmall];
  if (*n_eff == 0 || *n_mid == 0) return;
  for (uint32_t t = blockIdx.x; t < uint32_t(n_tiles); t += gridDim.x) {
    const uint32_t start = ranges[2 * size_t(t)];
    const uint32_t n = ranges[2 * size_t(t) + 1] - start;
    if (n <= uint32_t(kWaveKeys) || n > uint32_t(kSmall)) continue;  // block-uniform
    sort_list_regs<kMidThreads / 64>(bucket, start, n, t, s, vals, keys);
  }
}

// Longer lists: 1024-thread blocks, each striding over the tiles (a block
// needs much of a CU's LDS, so one block per tile would serialise on empty
// tiles), with LDS chunks of kChunk keys.  A list of at most kChunk keys is
// sorted in LDS (block_reg_sort over the block's 16 waves measured slower
// here: 0.070 against 0.058 ms at 1M Gaussians, 200x133, tile 8).  A longer one is sorted in place in the bucket: each chunk is
// sorted in LDS, then for every further merge size the strides >= kChunk run on
// global memory and the shorter ones per chunk in LDS.  (All waves of a block
// share one CU, whose L1 keeps the block's global writes coherent across the
// barriers.)  The 64 KB chunk lets two blocks share a CU, so 512 blocks take
// all of a low-resolution view's long lists at once; with 16384-key chunks one
// block held a CU, and the 425 lists of 1M Gaussians at 200x133 (tile 8) took
// two rounds of 256 blocks (sorts 96 -> 80 us, the same keys).
constexpr int kChunk = 8192;
constexpr int kBigThreads = 1024;
constexpr int kBigBlocks = 512;

__device__ inline void sort_long(uint64_t* s, uint64_t* a, uint32_t n) {
  const uint32_t len = pow2_ceil(n);
  auto load = [&](uint32_t c0, uint32_t m) {
    for (uint32_t i = threadIdx.x; i < m; i += kBigThreads) s[i] = a[c0 + i];
    __syncthreads();
  };
  auto store = [&](uint32_t c0, uint32_t m) {
    for (uint32_t i = threadIdx.x; i < m; i += kBigThreads) a[c0 + i] = s[i];
    __syncthreads();
  };
  // every chunk sorted on its own (chunks are aligned blocks of the network)
  for (uint32_t c0 = 0; c0 < n; c0 += kChunk) {
    const uint32_t m = (n - c0 < uint32_t(kChunk)) ? n - c0 : uint32_t(kChunk);
    load(c0, m);
    lds_sort<kBigThreads>(s, m, kChunk);
    store(c0, m);
  }
  for (uint32_t h = kChunk; h < len; h <<= 1) {
    net_step<kBigThreads>(a, n, len / 2, h, true);
    for (uint32_t d = h >> 1; d >= uint32_t(kChunk); d >>= 1)
      net_step<kBigThreads>(a, n, len / 2, d, false);
    for (uint32_t c0 = 0; c0 < n; c0 += kChunk) {
      const uint32_t m = (n - c0 < uint32_t(kChunk)) ? n - c0 : uint32_t(kChunk);
      load(c0, m);
      for (uint32_t d = kChunk / 2; d > 0; d >>= 1)
        net_step<kBigThreads>(s, m, kChunk / 2, d, false);
      store(c0, m);
    }
  }
}

__global__ __launch_bounds__(kBigThreads) void k_tile_sort_big(
    int n_tiles, const int64_t* __restrict__ n_eff, const int64_t* __restrict__ n_long,
    uint64_t* __restrict__ bucket,
    uint32_t* __restrict__ vals, uint64_t* __restrict__ keys,
    uint32_t* __restrict__ ranges) {
  __shared__ uint64_t s[kChunk];
  // empty tiles read [0, 0): the wave tier leaves them at [p, p) because a
  // tile's end is its neighbour's start, which must stay until every wave has
  // read it.  Here every range is final, and the long-list loop below reads
  // non-empty tiles only.
  for (uint32_t t = blockIdx.x * kBigThreads + threadIdx.x; t < uint32_t(n_tiles);
       t += gridDim.x * kBigThreads)
    if (ranges[2 * size_t(t)] == ranges[2 * size_t(t) + 1])
      ranges[2 * size_t(t)] = ranges[2 * size_t(t) + 1] = 0u;
  if (*n_eff == 0 || *n_long == 0) return;
  for (uint32_t t = blockIdx.x; t < uint32_t(n_tiles); t += gridDim.x) {
    const uint32_t start = ranges[2 * size_t(t)], end = ranges[2 * size_t(t) + 1];
    const uint32_t n = end - start;
    if (n <= uint32_t(kSmall)) continue;  // block-uniform
    if (n <= uint32_t(kChunk)) {
      for (uint32_t i = threadIdx.x; i < n; i += kBigThreads) s[i] = bucket[start + i];
      __syncthreads();
      lds_sort<kBigThreads>(s, n, pow2_ceil(n));
      write_sorted<kBigThreads>(s, n, start, t, vals, keys);
    } else {
      sort_long(s, bucket + start, n);
      write_sorted<kBigThreads>(bucket + start, n, start, t, vals, keys);
    }
    __syncthreads();  // s is reused by the block's next tile
  }
}

// value into p[0, count) and q[0, count_q)
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t count,
                                                  uint32_t value, uint32_t* __restrict__ q,
                                                  int64_t count_q) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = value;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count_q;
       i += int64_t(gridDim.x) * blockDim.x)
    q[i] = value;
}

struct WsLayout {
  size_t cnt, copies, bucket, rank, bpos, total;
  WsLayout(int64_t m, int64_t cap) {
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    cnt = take(8 * 4);
    copies = take(4 * size_t(kXcds) * kAggBins);
    bucket = take(8 * size_t(cap));
    rank = take(4 * size_t(cap));
    bpos = take(4 * (size_t((m + kXT - 1) / kXT) + 1));  // per expansion block
    total = o;
  }
};

// ---- the no-allocation form (gs_bin_sort_noalloc): the workspace of a call
// of at most GS_BIN_SORT_NOALLOC_MAX_PAIRS pairs of capacity lives in this
// file-scope device array, one copy per GPU.  Host code never passes the
// array's name to a kernel (on the host it only names the symbol): the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t align256c(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kNoAllocBytes =
    256 + align256c(4 * size_t(kXcds) * kAggBins) + align256c(8 * size_t(GS_BIN_SORT_NOALLOC_MAX_PAIRS)) +
    align256c(4 * size_t(GS_BIN_SORT_NOALLOC_MAX_PAIRS)) +
    align256c(4 * (size_t(GS_BIN_SORT_NOALLOC_MAX_ITEMS + kXT - 1) / kXT + 1));
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on the first call on that
// device (with it current) and kept until the process ends.
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

size_t bin_sort_ws_bytes(int n_views, int n, int64_t cap) {
  return WsLayout(int64_t(n_views) * n, cap).total;
}

hipError_t launch_bin_sort_noalloc(const Views& V, int n, char* proj, int64_t cap,
                                   uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                                   int64_t* n_pairs_dev, hipStream_t st) {
  const int64_t m = int64_t(V.n_views) * n;
  if (cap < 0 || cap > GS_BIN_SORT_NOALLOC_MAX_PAIRS || m > GS_BIN_SORT_NOALLOC_MAX_ITEMS ||
      WsLayout(m, cap).total > kNoAllocBytes)
    return hipErrorInvalidValue;  // the caller rejects this first
  void* ws = nullptr;
  const hipError_t e = scratch_address(&ws);
  if (e != hipSuccess) return e;
  // every call writes each scratch byte it reads before reading it (the counts
  // in the tile scan, the block offsets in the reduce pass, the ranks in the
  // count pass, the bucket slots [0, pairs) in the bucket pass), so nothing is
  // cleared
  return launch_bin_sort(V, n, proj, cap, ws, keys, vals, ranges, n_pairs_dev, st);
}

hipError_t launch_bin_sort(const Views& V, int n, char* proj, int64_t cap, void* ws_,
                           uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                           int64_t* n_pairs_dev, hipStream_t st) {
  const WsLayout W(int64_t(V.n_views) * n, cap);
  char* ws = static_cast<char*>(ws_);
  int64_t* counts = reinterpret_cast<int64_t*>(ws + W.cnt);
  int64_t* n_tot = counts + 0;
  int64_t* n_eff = counts + 1;
  int64_t* n_long = counts + 2;
  int64_t* n_mid = counts + 3;
  uint64_t* bucket = reinterpret_cast<uint64_t*>(ws + W.bucket);
  uint32_t* rank = reinterpret_cast<uint32_t*>(ws + W.rank);
  uint32_t* bpos = reinterpret_cast<uint32_t*>(ws + W.bpos);
  uint32_t* copies_ws = reinterpret_cast<uint32_t*>(ws + W.copies);
  const ProjLayout L(n);
  Items S{};
  int min_view_tiles = 1 << 30;
  for (int v = 0; v < V.n_views; ++v) {
    S.TI.tile_base[v] = V.v[v].tile_base;
    S.TI.tile_end[v] = V.v[v].tile_base + V.v[v].gw * V.v[v].gh;
    S.TI.gw[v] = V.v[v].gw;
    min_view_tiles = std::min(min_view_tiles, V.v[v].gw * V.v[v].gh);
  }
  S.proj = proj;
  S.stride = L.stride;
  S.tt_off = L.tt;
  S.goff_proj = proj;  // the count pass records the items' pair offsets
  S.goff_off = L.goff;
  S.m = int64_t(V.n_views) * n;
  S.n = n;
  S.tile = V.tile;
  const int T = V.total_tiles;
  const int64_t nr = 2 * int64_t(T);
  // LDS aggregation pays where views have few tiles; blocks then take more
  // items (fewer global atomics), as long as the grid still fills the chip:
  // a small scene keeps one round per block
  const bool any_agg = min_view_tiles <= kAggBins;
  int rounds = 1;
  if (any_agg) {
    const int64_t want = (S.m + int64_t(kXT) * kAggBlocks - 1) / (int64_t(kXT) * kAggBlocks);
    rounds = int(std::min<int64_t>(std::max<int64_t>(want, 1), kAggRounds));
  }
  // every launch may aggregate: whole views of few tiles, or the tile rectangle
  // of a block of Gaussians that sit close together
  const size_t agg_lds = sizeof(uint32_t) * kAggBins;
  const int agg_bins = kAggBins;
  const unsigned xb = unsigned((S.m + int64_t(kXT) * rounds - 1) / (int64_t(kXT) * rounds));

  // launches of at most kAggBins tiles spread the LDS-counting blocks'
  // reservation atomics over kXcds counter copies
  uint32_t* copies = (T <= kAggBins) ? copies_ws : nullptr;
  const int64_t nc = copies ? int64_t(kXcds) * kAggBins : 0;
  GS_LAUNCH("k_fill_u32", k_fill_u32, dim3(unsigned(nr / 256 + 1 < 4096 ? nr / 256 + 1 : 4096)),
            dim3(256), 0, st, ranges, nr, 0u, copies, nc);
  if (xb > 0) {
    // index-order positions of each block's first pair: ranked pairs store
    // their ranks there, and every item's pair offset (recorded in proj for
    // the backward) follows from them
    GS_LAUNCH("k_tile_reduce", k_tile_reduce, dim3(xb), dim3(kXT), 0, st, S, rounds, bpos);
    GS_LAUNCH("k_scan_spine", k_scan_spine, dim3(1), dim3(kScanThreads), 0, st, bpos,
              Count{nullptr, int64_t(xb) * kScanTile}, nullptr, nullptr);
    GS_LAUNCH("k_tile_count", k_tile_count, dim3(xb), dim3(kXT), agg_lds, st, S, rounds, agg_bins,
              bpos, cap, ranges, rank, copies);
  }
  int64_t* proj_total = proj ? reinterpret_cast<int64_t*>(proj + L.total) : nullptr;
  GS_LAUNCH("k_tile_scan", k_tile_scan, dim3(1), dim3(kTS), 0, st, ranges, copies, T, proj_total,
            cap, n_tot, n_eff, n_long, n_mid, n_pairs_dev);
  Items Sb = S;
  Sb.goff_proj = nullptr;
  if (xb > 0)
    GS_LAUNCH("k_bucket", k_bucket, dim3(xb), dim3(kXT), agg_lds, st, Sb, rounds, agg_bins, n_eff,
              bpos, rank, ranges, copies, bucket);
  GS_LAUNCH("k_tile_sort_wave", k_tile_sort_wave, dim3(unsigned((T + 3) / 4)), dim3(256), 0, st,
            T, n_tot, n_eff, n_mid, n_long, bucket, vals, keys, ranges);
  GS_LAUNCH("k_tile_sort_mid", k_tile_sort_mid, dim3(unsigned(T < kMidBlocks ? T : kMidBlocks)),
            dim3(kMidThreads), 0, st, T, n_eff, n_mid, bucket, vals, keys, ranges);
  GS_LAUNCH("k_tile_sort_big", k_tile_sort_big, dim3(unsigned(T < kBigBlocks ? T : kBigBlocks)),
            dim3(kBigThreads), 0, st, T, n_eff, n_long, bucket, vals, keys, ranges);
  return hipGetLastError();
}

}  // namespace gsk
