// Binning by a stable LSD radix sort of the (tile | depth) keys, beside the
// bucket-then-tile-sort of sort.hip: the same result (the stable sort of the
// 64-bit keys is unique, ties keep the ascending Gaussian index), by the
// classic route.
//
// The 64-bit key is key = (tile_id << 32) | bits(depth_f32) and the sort takes
// 8-bit digits.  An LSD sort handles the least significant digits first, and
// every pair of one Gaussian carries the same depth bits, so the four depth
// digits are sorted on the visible Gaussians themselves (about one item per
// Gaussian) before the pairs are expanded; the expansion keeps that order and
// the remaining tile digits are then sorted on the pairs.  The result is
// exactly the stable sort of the full 64-bit keys (items enter in index
// order), at a fraction of the traffic of sorting every pair on every digit.
//
// Each radix pass is reduce-then-scan (histogram, per-digit row scan, stable
// scatter), with no inter-block waiting.  The stable in-block rank uses
// wavefront ballots: the lanes holding the same digit are found with one
// ballot per digit bit, and ranked with a popcount of the lanes below.
#include "scan.hpp"

namespace gsk {
namespace {

constexpr int kRT = 256;          // threads per radix block
constexpr int kRIPT = 16;         // items per thread
constexpr int kRTile = kRT * kRIPT;
constexpr int kRWaveItems = kRTile / 4;

__device__ inline int64_t cnt_blocks(int64_t n) { return (n + kRTile - 1) / kRTile; }

__global__ __launch_bounds__(kRT) void k_radix_hist(const uint32_t* __restrict__ keys, Count cnt,
                                                    int shift, int bits,
                                                    uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_cnt[4][256];
  const int64_t n = cnt.get();
  const int64_t nb = cnt_blocks(n);
  if (int64_t(blockIdx.x) >= nb) return;
  for (int i = threadIdx.x; i < 4 * 256; i += kRT) (&s_cnt[0][0])[i] = 0;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  const int w = threadIdx.x >> 6;
  const int64_t base = int64_t(blockIdx.x) * kRTile;
#pragma unroll 4
  for (int k = 0; k < kRIPT; ++k) {
    const int64_t i = base + int64_t(k) * kRT + threadIdx.x;
    if (i < n) atomicAdd(&s_cnt[w][(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d <= int(mask); d += kRT)
    hist[int64_t(d) * nb + blockIdx.x] = s_cnt[0][d] + s_cnt[1][d] + s_cnt[2][d] + s_cnt[3][d];
}

// one block per digit: exclusive scan of that digit's per-block counts
__global__ __launch_bounds__(kRT) void k_radix_rowscan(uint32_t* __restrict__ hist, Count cnt,
                                                       uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t s_tmp[4];
  const int64_t nb = cnt_blocks(cnt.get());
  uint32_t* row = hist + int64_t(blockIdx.x) * nb;
  uint32_t carry = 0;
  for (int64_t c = 0; c < nb; c += kRT) {
    const int64_t i = c + threadIdx.x;
    const uint32_t x = (i < nb) ? row[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(x, tot, s_tmp);
    if (i < nb) row[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kRT) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, Count cnt, int shift, int bits,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t s_wcnt[4][256];
  __shared__ uint32_t s_key[kRTile];
  __shared__ uint32_t s_val[kRTile];
  __shared__ uint32_t s_boff[256];
  __shared__ uint32_t s_gbase[256];
  __shared__ uint32_t s_tmp[4];
  const int64_t n = cnt.get();
  const int64_t nb = cnt_blocks(n);
  const int64_t b = blockIdx.x;
  if (b >= nb) return;
  const uint32_t mask = (1u << bits) - 1u;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < 4 * 256; i += kRT) (&s_wcnt[0][0])[i] = 0;
  __syncthreads();

  const int64_t base = b * kRTile;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t key[kRIPT], val[kRIPT], dig[kRIPT], rank[kRIPT];
#pragma unroll
  for (int r = 0; r < kRIPT; ++r) {
    const int64_t i = base + int64_t(w) * kRWaveItems + r * 64 + lane;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const uint32_t v = valid ? vin[i] : 0u;
    const uint32_t d = (k >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int bb = 0; bb < bits; ++bb) {
      const bool bit = (d >> bb) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t c = s_wcnt[w][d];
    rank[r] = c + uint32_t(__popcll(peers & lt));
    // the highest lane of each digit group advances that digit's counter
    if (valid && (peers >> lane) == 1ull) s_wcnt[w][d] = c + uint32_t(__popcll(peers));
    key[r] = k;
    val[r] = v;
    dig[r] = valid ? d : 0xffffffffu;
  }
  __syncthreads();
  // per digit: prefix over waves, block total, block-local and global offsets
  {
    const int d = tid;
    const uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
    const uint32_t tot = c0 + c1 + c2 + c3;
    uint32_t btot;
    const uint32_t boff = block_excl_scan256(d <= int(mask) ? tot : 0u, btot, s_tmp);
    const uint32_t dt = (d <= int(mask)) ? digit_total[d] : 0u;
    uint32_t gtot;
    const uint32_t gex = block_excl_scan256(dt, gtot, s_tmp);
    s_wcnt[0][d] = 0;
    s_wcnt[1][d] = c0;
    s_wcnt[2][d] = c0 + c1;
    s_wcnt[3][d] = c0 + c1 + c2;
    s_boff[d] = boff;
    if (d <= int(mask)) s_gbase[d] = gex + hist[int64_t(d) * nb + b];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRIPT; ++r) {
    const uint32_t d = dig[r];
    if (d != 0xffffffffu) {
      const uint32_t pos = s_boff[d] + s_wcnt[w][d] + rank[r];
      s_key[pos] = key[r];
      s_val[pos] = val[r];
    }
  }
  __syncthreads();
  const int64_t m = (n - base < kRTile) ? (n - base) : kRTile;
  for (int j = tid; j < m; j += kRT) {
    const uint32_t k = s_key[j];
    const uint32_t d = (k >> shift) & mask;
    const uint32_t out = s_gbase[d] + (uint32_t(j) - s_boff[d]);
    kout[out] = k;
    vout[out] = s_val[j];
  }
}

}  // namespace

// One LSD pass on (key, value) u32 pairs: bits [shift, shift+bits), bits <= 8.
hipError_t radix_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      Count cnt, int64_t max_n, int shift, int bits, uint32_t* hist,
                      uint32_t* digit_total, hipStream_t st) {
  const int64_t nb = (max_n + kRTile - 1) / kRTile;
  if (nb == 0) return hipSuccess;
  GS_LAUNCH("k_radix_hist", k_radix_hist, dim3(unsigned(nb)), dim3(kRT), 0, st, kin, cnt, shift, bits,
                     hist);
  GS_LAUNCH("k_radix_rowscan", k_radix_rowscan, dim3(1u << bits), dim3(kRT), 0, st, hist, cnt,
                     digit_total);
  GS_LAUNCH("k_radix_scatter", k_radix_scatter, dim3(unsigned(nb)), dim3(kRT), 0, st, kin, vin, kout, vout,
                     cnt, shift, bits, hist, digit_total);
  return hipGetLastError();
}

size_t radix_hist_words(int64_t max_n) { return 256 * size_t((max_n + kRTile - 1) / kRTile); }

namespace {

// ---------------------------------------------------------------- functors
struct VisSrc {  // 1 for every (view, Gaussian) item with a non-empty footprint
  const char* proj;
  size_t stride, tt_off;
  int n;
  __device__ uint32_t operator()(int64_t i) const {
    const int64_t v = i / n, g = i - v * n;
    const uint32_t* tt = reinterpret_cast<const uint32_t*>(proj + v * stride + tt_off);
    return tt[g] > 0u ? 1u : 0u;
  }
};
struct VisDst {  // compact: depth bits as the key, item id as the value
  const char* proj;
  size_t stride;
  int n;
  uint32_t* key;
  uint32_t* val;
  __device__ void operator()(int64_t i, uint32_t pos, uint32_t flag) const {
    if (!flag) return;
    const int64_t v = i / n, g = i - v * n;
    const float4* rec = reinterpret_cast<const float4*>(proj + v * stride);
    key[pos] = __float_as_uint(rec[3 * g + 2].y);
    val[pos] = uint32_t(i);
  }
};
struct SortedTTSrc {  // tiles touched of the i-th depth-sorted item
  const char* proj;
  size_t stride, tt_off;
  int n;
  const uint32_t* items;
  __device__ uint32_t operator()(int64_t i) const {
    const uint32_t it = items[i];
    const uint32_t v = it / uint32_t(n), g = it - v * uint32_t(n);
    return reinterpret_cast<const uint32_t*>(proj + size_t(v) * stride + tt_off)[g];
  }
};
struct OffDst {
  uint32_t* off;
  __device__ void operator()(int64_t i, uint32_t pos, uint32_t) const { off[i] = pos; }
};
struct TTSrcItems {  // tiles touched of item i (index order)
  const char* proj;
  size_t stride, tt_off;
  int n;
  __device__ uint32_t operator()(int64_t i) const {
    const int64_t v = i / n, g = i - v * n;
    return reinterpret_cast<const uint32_t*>(proj + v * stride + tt_off)[g];
  }
};
struct ProjGoffDst {  // item i's first pair position, into proj for the backward
  char* proj;
  size_t stride, goff_off;
  int n;
  __device__ void operator()(int64_t i, uint32_t pos, uint32_t) const {
    const int64_t v = i / n, g = i - v * n;
    reinterpret_cast<uint32_t*>(proj + v * stride + goff_off)[g] = pos;
  }
};

struct TileInfo {  // per view: first global tile and grid width
  int32_t tile_base[GS_MAX_VIEWS];
  int32_t gw[GS_MAX_VIEWS];
};

__global__ __launch_bounds__(256) void k_finalize_count(const int64_t* __restrict__ total,
                                                        int64_t cap, int64_t* __restrict__ n_eff,
                                                        int64_t* __restrict__ n_pairs_user) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t t = *total;
    *n_eff = (t <= cap) ? t : 0;
    *n_pairs_user = t;
  }
}

// one thread per depth-sorted visible item: write its (tile, Gaussian) pairs
__global__ __launch_bounds__(256) void k_emit(TileInfo TI, int tile, int n, const char* proj,
                                              size_t stride, const uint32_t* __restrict__ items,
                                              const uint32_t* __restrict__ offs,
                                              const int64_t* __restrict__ n_vis,
                                              const int64_t* __restrict__ n_eff,
                                              uint32_t* __restrict__ pair_tile,
                                              uint32_t* __restrict__ pair_val) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= *n_vis || *n_eff == 0) return;
  const uint32_t it = items[i];
  const uint32_t v = it / uint32_t(n), g = it - v * uint32_t(n);
  const float4 r2 = reinterpret_cast<const float4*>(proj + size_t(v) * stride)[3 * size_t(g) + 2];
  const uint32_t lo = __float_as_uint(r2.z), hi = __float_as_uint(r2.w);
  const int tx0 = box_x(lo) / tile, ty0 = box_y(lo) / tile;
  const int tx1 = box_x(hi) / tile, ty1 = box_y(hi) / tile;
  const int gw = TI.gw[v];
  const uint32_t tb = uint32_t(TI.tile_base[v]);
  uint32_t o = offs[i];
  for (int ty = ty0; ty <= ty1; ++ty) {
    const uint32_t row = tb + uint32_t(ty * gw);
    for (int tx = tx0; tx <= tx1; ++tx) {
      pair_tile[o] = row + uint32_t(tx);
      pair_val[o] = g;
      ++o;
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t count,
                                                  uint32_t value) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = value;
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tiles,
                                                const int64_t* __restrict__ n_eff,
                                                uint32_t* __restrict__ ranges) {
  const int64_t n = *n_eff;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = tiles[i];
  if (i == 0 || tiles[i - 1] != t) ranges[2 * size_t(t)] = uint32_t(i);
  if (i == n - 1 || tiles[i + 1] != t) ranges[2 * size_t(t) + 1] = uint32_t(i + 1);
}

__global__ __launch_bounds__(256) void k_keys(TileInfo TI, int n_views, int n, const char* proj,
                                              size_t stride, const uint32_t* __restrict__ tiles,
                                              const uint32_t* __restrict__ vals,
                                              const int64_t* __restrict__ n_eff,
                                              uint64_t* __restrict__ keys) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= *n_eff) return;
  const uint32_t t = tiles[i];
  int v = 0;
  for (int k = 1; k < n_views; ++k) v = (uint32_t(TI.tile_base[k]) <= t) ? k : v;
  const float4 r2 =
      reinterpret_cast<const float4*>(proj + size_t(v) * stride)[3 * size_t(vals[i]) + 2];
  keys[i] = (uint64_t(t) << 32) | uint64_t(__float_as_uint(r2.y));
}

struct WsLayout {
  size_t ikey0, ikey1, ival0, ival1, offs, bsum, hist, dtot, cnt, ptile0, ptile1, pval, total;
  WsLayout(int64_t M, int64_t cap) {
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
    const int64_t mx = M > cap ? M : cap;
    ikey0 = take(4 * M); ikey1 = take(4 * M); ival0 = take(4 * M); ival1 = take(4 * M);
    offs = take(4 * M);
    bsum = take(4 * scan_block_sums(mx));
    hist = take(4 * 256 * size_t((mx + kRTile - 1) / kRTile + 1));
    dtot = take(4 * 256);
    cnt = take(8 * 4);
    ptile0 = take(4 * cap); ptile1 = take(4 * cap); pval = take(4 * cap);
    total = o;
  }
};

int ceil_log2(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x) ++b;
  return b;
}

}  // namespace

size_t bin_sort_radix_ws_bytes(int n_views, int n, int64_t cap) {
  return WsLayout(int64_t(n_views) * n, cap).total;
}

hipError_t launch_bin_sort_radix(const Views& V, int n, char* proj, int64_t cap, void* ws_,
                                 uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                                 int64_t* n_pairs_dev, hipStream_t st) {
  const int64_t M = int64_t(V.n_views) * n;
  const WsLayout W(M, cap);
  char* ws = static_cast<char*>(ws_);
  auto U = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  int64_t* counts = reinterpret_cast<int64_t*>(ws + W.cnt);
  int64_t* n_vis = counts + 0;
  int64_t* n_tot = counts + 1;
  int64_t* n_eff = counts + 2;
  const ProjLayout L(n);
  hipError_t e;

  // 0. the items' pair offsets in index order and the pair total, recorded in
  // proj for the backward (the same values the bucket route records)
  if (proj) {
    e = scan_exclusive(TTSrcItems{proj, L.stride, L.tt, n},
                       ProjGoffDst{proj, L.stride, L.goff, n}, Count{nullptr, M}, M, U(W.bsum),
                       reinterpret_cast<int64_t*>(proj + L.total), nullptr, st);
    if (e != hipSuccess) return e;
  }
  // 1. compact the visible items: key = depth bits, value = item id
  e = scan_exclusive(VisSrc{proj, L.stride, L.tt, n},
                     VisDst{proj, L.stride, n, U(W.ikey0), U(W.ival0)}, Count{nullptr, M}, M,
                     U(W.bsum), n_vis, nullptr, st);
  if (e != hipSuccess) return e;
  // 2. depth digits: four 8-bit passes on the items (even count: ends in buffer 0)
  for (int p = 0; p < 4; ++p) {
    const bool f = (p & 1) == 0;
    e = radix_pass(U(f ? W.ikey0 : W.ikey1), U(f ? W.ival0 : W.ival1), U(f ? W.ikey1 : W.ikey0),
                   U(f ? W.ival1 : W.ival0), Count{n_vis, 0}, M, 8 * p, 8, U(W.hist), U(W.dtot),
                   st);
    if (e != hipSuccess) return e;
  }
  // 3. pair offsets in depth order
  e = scan_exclusive(SortedTTSrc{proj, L.stride, L.tt, n, U(W.ival0)}, OffDst{U(W.offs)},
                     Count{n_vis, 0}, M, U(W.bsum), n_tot, nullptr, st);
  if (e != hipSuccess) return e;
  GS_LAUNCH("k_finalize_count", k_finalize_count, dim3(1), dim3(64), 0, st, n_tot, cap, n_eff, n_pairs_dev);

  // 4. expand: pairs in depth order, tiles row-major within each footprint
  TileInfo TI{};
  for (int v = 0; v < V.n_views; ++v) {
    TI.tile_base[v] = V.v[v].tile_base;
    TI.gw[v] = V.v[v].gw;
  }
  const int tbits = ceil_log2(V.total_tiles);
  const int passes = (tbits + 7) / 8;
  uint32_t* vb[2];
  vb[passes % 2] = vals;
  vb[(passes + 1) % 2] = U(W.pval);
  uint32_t* tb[2] = {U(W.ptile0), U(W.ptile1)};
  if (M > 0) {
    GS_LAUNCH("k_emit", k_emit, dim3(unsigned((M + 255) / 256)), dim3(256), 0, st, TI, V.tile, n,
                       proj, L.stride, U(W.ival0), U(W.offs), n_vis, n_eff, tb[0], vb[0]);
  }
  // 5. tile digits on the pairs (stable: depth order survives within a tile)
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int bits = (tbits - shift + (passes - p) - 1) / (passes - p);
    e = radix_pass(tb[p & 1], vb[p & 1], tb[(p + 1) & 1], vb[(p + 1) & 1], Count{n_eff, 0}, cap,
                   shift, bits, U(W.hist), U(W.dtot), st);
    if (e != hipSuccess) return e;
    shift += bits;
  }
  uint32_t* tiles_sorted = tb[passes & 1];
  // 6. ranges
  const int64_t nr = 2 * int64_t(V.total_tiles);
  GS_LAUNCH("k_fill_u32", k_fill_u32, dim3(unsigned(nr / 256 + 1 < 4096 ? nr / 256 + 1 : 4096)),
                     dim3(256), 0, st, ranges, nr, 0u);
  if (cap > 0) {
    GS_LAUNCH("k_ranges", k_ranges, dim3(unsigned((cap + 255) / 256)), dim3(256), 0, st,
                       tiles_sorted, n_eff, ranges);
    if (keys) {
      GS_LAUNCH("k_keys", k_keys, dim3(unsigned((cap + 255) / 256)), dim3(256), 0, st, TI,
                         V.n_views, n, proj, L.stride, tiles_sorted, vals, n_eff, keys);
    }
  }
  return hipGetLastError();
}

}  // namespace gsk
