// Device-wide exclusive scan of u32 values (reduce-then-scan, no inter-block
// waiting, so it needs no forward-progress guarantee) and block primitives
// on 64-wide wavefronts.  Element counts may live in device memory, so the
// same launches work inside a captured HIP graph.
#pragma once

#include "gs_internal.hpp"

namespace gsk {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096 elements per block

// A count that is either known on the host or read from device memory.
struct Count {
  const int64_t* dev;
  int64_t host;
  __device__ inline int64_t get() const { return dev ? *dev : host; }
};

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan over a 256-thread block; s_tmp holds 4 u32.  All threads
// must call it.  Returns the exclusive prefix and the block total.
__device__ inline uint32_t block_excl_scan256(uint32_t x, uint32_t& total, uint32_t* s_tmp) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(x);
  if (lane == 63) s_tmp[w] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t t = s_tmp[i];
    base += (i < w) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return base + inc - x;
}

// --- kernels; Src is a functor: uint32_t operator()(int64_t i) const
template <class Src>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(Src src, Count cnt,
                                                              uint32_t* block_sums) {
  __shared__ uint32_t s_tmp[4];
  const int64_t n = cnt.get();
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  if (base >= n) return;
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + int64_t(k) * kScanThreads + threadIdx.x;
    if (i < n) acc += src(i);
  }
  uint32_t tot;
  block_excl_scan256(acc, tot, s_tmp);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// One block: exclusive scan of the per-block sums in place; writes the total.
// Chunks of kScanTile sums: coalesced loads into LDS, 16 consecutive sums per
// thread, so a spine of up to 4096 blocks is one pass.
static __global__ __launch_bounds__(kScanThreads) void k_scan_spine(uint32_t* block_sums, Count cnt,
                                                             int64_t* total_out,
                                                             uint32_t* total_out32) {
  __shared__ uint32_t s_v[kScanTile];
  __shared__ uint32_t s_tmp[4];
  const int64_t n = cnt.get();
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  uint32_t carry = 0;
  for (int64_t c = 0; c < nb; c += kScanTile) {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int j = k * kScanThreads + threadIdx.x;
      s_v[j] = (c + j < nb) ? block_sums[c + j] : 0u;
    }
    __syncthreads();
    uint32_t loc[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      loc[k] = s_v[threadIdx.x * kScanItems + k];
      acc += loc[k];
    }
    uint32_t tot;
    uint32_t ex = carry + block_excl_scan256(acc, tot, s_tmp);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      s_v[threadIdx.x * kScanItems + k] = ex;
      ex += loc[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int j = k * kScanThreads + threadIdx.x;
      if (c + j < nb) block_sums[c + j] = s_v[j];
    }
    carry += tot;
    __syncthreads();  // s_v is refilled by the next chunk
  }
  if (threadIdx.x == 0) {
    if (total_out) *total_out = int64_t(carry);
    if (total_out32) *total_out32 = carry;
  }
}

// Dst: functor void operator()(int64_t i, uint32_t excl_prefix, uint32_t value) const
template <class Src, class Dst>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(Src src, Dst dst, Count cnt,
                                                            const uint32_t* block_sums) {
  __shared__ uint32_t s_v[kScanTile];
  __shared__ uint32_t s_p[kScanTile];
  __shared__ uint32_t s_tmp[4];
  const int64_t n = cnt.get();
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  if (base >= n) return;
  // striped (coalesced) loads into LDS, then each thread scans 16 consecutive values
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int j = k * kScanThreads + threadIdx.x;
    const int64_t i = base + j;
    s_v[j] = (i < n) ? src(i) : 0u;
  }
  __syncthreads();
  uint32_t loc[kScanItems];
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    loc[k] = s_v[threadIdx.x * kScanItems + k];
    acc += loc[k];
  }
  uint32_t tot;
  uint32_t ex = block_excl_scan256(acc, tot, s_tmp) + block_sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    s_p[threadIdx.x * kScanItems + k] = ex;
    ex += loc[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int j = k * kScanThreads + threadIdx.x;
    const int64_t i = base + j;
    if (i < n) dst(i, s_p[j], s_v[j]);
  }
}

// Host: enqueue the three scan kernels.  `max_n` bounds the grid; the real
// count comes from `cnt` (host or device).  block_sums needs
// ceil(max_n / 4096) u32.
template <class Src, class Dst>
hipError_t scan_exclusive(Src src, Dst dst, Count cnt, int64_t max_n, uint32_t* block_sums,
                          int64_t* total_out, uint32_t* total_out32, hipStream_t st) {
  const int64_t nb = (max_n + kScanTile - 1) / kScanTile;
  if (nb > 0) {
    GS_LAUNCH("k_scan_reduce", HIP_KERNEL_NAME(k_scan_reduce<Src>), dim3(unsigned(nb)),
                       dim3(kScanThreads), 0, st, src, cnt, block_sums);
  }
  GS_LAUNCH("k_scan_spine", k_scan_spine, dim3(1), dim3(kScanThreads), 0, st, block_sums, cnt,
                     total_out, total_out32);
  if (nb > 0) {
    GS_LAUNCH("k_scan_down", HIP_KERNEL_NAME(k_scan_down<Src, Dst>), dim3(unsigned(nb)),
                       dim3(kScanThreads), 0, st, src, dst, cnt, block_sums);
  }
  return hipGetLastError();
}

inline size_t scan_block_sums(int64_t max_n) {
  return size_t((max_n + kScanTile - 1) / kScanTile + 1);
}

}  // namespace gsk
