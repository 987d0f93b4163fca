// Spatial storage order of the Gaussians: a Morton (Z-order) curve over their
// means, and the row gather that applies a permutation to parameter arrays.
//
// Nothing the rasterizer computes depends on the order of the Gaussians
// (ties of exactly equal depth follow the stored index).  Stored along a
// space-filling curve, the Gaussians a block of consecutive indices holds sit
// close together in space, so:
//   - a block's (tile, Gaussian) pairs fall on few tiles, which the binning
//     counts in LDS before touching the global tile counters;
//   - the Gaussians outside a view's frustum form long index runs, which
//     sparse Adam and the preprocess's colour staging then skip whole;
//   - a tile's list draws its records from few index runs (fewer cache lines).
//
// The order: per axis a, lo_a / hi_a = min / max of the means (exact);
// s_a = 1024 / (hi_a - lo_a) (0 when the box is flat); cell
// q = min(1023, floor((m - lo) s)) with every operation rounded to float32 in
// that order; the code interleaves the ten bits of q_x, q_y, q_z (bit b of q_x
// at 3b, of q_y at 3b+1, of q_z at 3b+2); the permutation is the stable
// ascending sort of the codes (ties keep ascending index), by four LSD radix
// passes over (code, index).
#include <algorithm>

#include "scan.hpp"

namespace gsk {
namespace {

constexpr int kOT = 256;
constexpr int kBoxBlocks = 256;

// per-block min / max of each coordinate: part[a][b] (min), part[3 + a][b] (max)
__global__ __launch_bounds__(kOT) void k_box_partial(int n, const float* __restrict__ means,
                                                     float* __restrict__ part) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * kOT + threadIdx.x; i < n; i += gridDim.x * kOT) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float m = means[3 * size_t(i) + a];
      lo[a] = fminf(lo[a], m);
      hi[a] = fmaxf(hi[a], m);
    }
  }
  __shared__ float s[6][kOT / 64];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      lo[a] = fminf(lo[a], __shfl_xor(lo[a], d, 64));
      hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], d, 64));
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      s[a][threadIdx.x >> 6] = lo[a];
      s[3 + a][threadIdx.x >> 6] = hi[a];
    }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int c = threadIdx.x;
    float r = s[c][0];
#pragma unroll
    for (int w = 1; w < kOT / 64; ++w) r = (c < 3) ? fminf(r, s[c][w]) : fmaxf(r, s[c][w]);
    part[c * kBoxBlocks + blockIdx.x] = r;
  }
}

__device__ __forceinline__ uint32_t spread3(uint32_t q) {  // bit b -> bit 3b, 10 bits
  uint32_t c = 0;
#pragma unroll
  for (int b = 0; b < 10; ++b) c |= ((q >> b) & 1u) << (3 * b);
  return c;
}

// codes of every Gaussian; each block first folds the partial boxes
__global__ __launch_bounds__(kOT) void k_morton(int n, const float* __restrict__ means,
                                                const float* __restrict__ part,
                                                uint32_t* __restrict__ code,
                                                uint32_t* __restrict__ index) {
  __shared__ float s_lo[3], s_s[3];
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    float lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < kBoxBlocks; ++b) {
      lo = fminf(lo, part[a * kBoxBlocks + b]);
      hi = fmaxf(hi, part[(3 + a) * kBoxBlocks + b]);
    }
    const float ext = __fsub_rn(hi, lo);
    s_lo[a] = lo;
    s_s[a] = ext > 0.0f ? __fdiv_rn(1024.0f, ext) : 0.0f;
  }
  __syncthreads();
  const int i = blockIdx.x * kOT + threadIdx.x;
  if (i >= n) return;
  uint32_t c = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float t = __fmul_rn(__fsub_rn(means[3 * size_t(i) + a], s_lo[a]), s_s[a]);
    const float f = floorf(t);
    const uint32_t q = f >= 1023.0f ? 1023u : (f > 0.0f ? uint32_t(f) : 0u);
    c |= spread3(q) << a;
  }
  code[i] = c;
  index[i] = uint32_t(i);
}

struct OrderWs {
  size_t part, k0, v0, k1, v1, hist, dtot, bytes;
  explicit OrderWs(int n) {
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align256(b); return r; };
    part = take(4 * 6 * size_t(kBoxBlocks));
    k0 = take(4 * size_t(n));
    v0 = take(4 * size_t(n));
    k1 = take(4 * size_t(n));
    v1 = take(4 * size_t(n));
    hist = take(4 * radix_hist_words(n));
    dtot = take(4 * 256);
    bytes = o;
  }
};

// dst[a][i * L + j] = src[a][perm[i] * L + j] for every array a (blockIdx.y);
// an index perm[i] >= n leaves row i of every array unwritten
struct GatherArgs {
  const float* src[kGatherMaxArrays];
  float* dst[kGatherMaxArrays];
  int32_t row[kGatherMaxArrays];
};

__global__ __launch_bounds__(256) void k_gather_rows(int n, const uint32_t* __restrict__ perm,
                                                     GatherArgs G) {
  const int a = blockIdx.y;
  const int L = G.row[a];
  const float* __restrict__ src = G.src[a];
  float* __restrict__ dst = G.dst[a];
  const int64_t total = int64_t(n) * L;
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * 256) {
    const int64_t i = e / L;
    const uint32_t from = perm[i];
    if (from < uint32_t(n)) dst[e] = src[int64_t(from) * L + (e - i * L)];
  }
}

}  // namespace

size_t spatial_order_ws_bytes(int n) { return OrderWs(n).bytes; }

hipError_t launch_spatial_order(int n, const float* means, void* ws_, uint32_t* perm,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  const OrderWs W(n);
  char* ws = static_cast<char*>(ws_);
  float* part = reinterpret_cast<float*>(ws + W.part);
  uint32_t* k0 = reinterpret_cast<uint32_t*>(ws + W.k0);
  uint32_t* v0 = reinterpret_cast<uint32_t*>(ws + W.v0);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(ws + W.k1);
  uint32_t* v1 = reinterpret_cast<uint32_t*>(ws + W.v1);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + W.hist);
  uint32_t* dtot = reinterpret_cast<uint32_t*>(ws + W.dtot);
  GS_LAUNCH("k_box_partial", k_box_partial, dim3(kBoxBlocks), dim3(kOT), 0, st, n, means, part);
  GS_LAUNCH("k_morton", k_morton, dim3(unsigned((n + kOT - 1) / kOT)), dim3(kOT), 0, st, n, means,
            part, k0, v0);
  const Count c{nullptr, n};
  // 30-bit codes: digits of 8, 8, 8 and 6 bits; the last pass writes the
  // indices straight into perm
  hipError_t e = radix_pass(k0, v0, k1, v1, c, n, 0, 8, hist, dtot, st);
  if (e == hipSuccess) e = radix_pass(k1, v1, k0, v0, c, n, 8, 8, hist, dtot, st);
  if (e == hipSuccess) e = radix_pass(k0, v0, k1, v1, c, n, 16, 8, hist, dtot, st);
  if (e == hipSuccess) e = radix_pass(k1, v1, k0, perm, c, n, 24, 6, hist, dtot, st);
  return e;
}

hipError_t launch_gather_rows(int n, const uint32_t* perm, int n_arrays, const float* const* src,
                              float* const* dst, const int32_t* row_floats, hipStream_t st) {
  if (n == 0 || n_arrays == 0) return hipSuccess;
  GatherArgs G{};
  int64_t widest = 0;
  for (int a = 0; a < n_arrays; ++a) {
    G.src[a] = src[a];
    G.dst[a] = dst[a];
    G.row[a] = row_floats[a];
    widest = std::max<int64_t>(widest, int64_t(n) * row_floats[a]);
  }
  const int64_t want = (widest + 255) / 256;
  const unsigned gx = unsigned(want < 8192 ? want : 8192);
  GS_LAUNCH("k_gather_rows", k_gather_rows, dim3(gx, unsigned(n_arrays)), dim3(256), 0, st, n,
            perm, G);
  return hipGetLastError();
}

}  // namespace gsk
