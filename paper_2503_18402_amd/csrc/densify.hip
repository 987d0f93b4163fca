// Densification under the primitive schedule (Sec. 4.3; supplementary,
// "Densification of DashGaussian"): prune, then clone or split the candidates
// with the top k densification scores, where k follows Eq. 4 with the budget
// of Eq. 5 (both host arithmetic, in abi.cpp).
//
// Score of a Gaussian: the mean, over the iterations it was seen, of the norm
// of its 2D-mean gradient (accumulated by k_densify_stats).  Candidates:
// unpruned Gaussians whose score reaches the threshold.  The top k are found
// without sorting: a four-pass radix select over the score's float bits
// (positive floats order like their bits) yields the k-th largest key and how
// many of its ties to take; ties go to the lowest indices, ranked by a scan.
// The output keeps index order: a pruned Gaussian writes nothing, a kept one
// itself, a cloned one itself then its copy, a split one its two children at
// mu + R(q) diag(s) z_j with scales s / 1.6 (z given by the caller).  Moments
// are copied for originals and zero for copies and children.
#include <algorithm>
#include <cmath>

#include "scan.hpp"

namespace gsk {
namespace {

constexpr uint32_t kPrune = 1u, kCand = 2u, kSel = 4u, kSplit = 8u;

__global__ __launch_bounds__(256) void k_densify_stats(int n, int n_views, const char* __restrict__ proj,
                                                       size_t stride, size_t tt_off,
                                                       const float* __restrict__ mean2d_abs,
                                                       float scale, float* __restrict__ accum,
                                                       float* __restrict__ count) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  int seen = 0;
  for (int v = 0; v < n_views; ++v)
    seen += reinterpret_cast<const uint32_t*>(proj + size_t(v) * stride + tt_off)[g] > 0u ? 1 : 0;
  if (seen) {
    accum[g] += scale * mean2d_abs[g];
    count[g] += float(seen);
  }
}

__global__ __launch_bounds__(256) void k_densify_classify(int n, const float* __restrict__ accum,
                                                          const float* __restrict__ count,
                                                          const float* __restrict__ opacity_logits,
                                                          float thr, float min_opacity,
                                                          uint32_t* __restrict__ keys,
                                                          uint32_t* __restrict__ flags,
                                                          unsigned long long* __restrict__ counts) {
  __shared__ uint32_t s_c[2];
  if (threadIdx.x < 2) s_c[threadIdx.x] = 0u;
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) {
    const float c = count[g];
    const float score = c > 0.0f ? accum[g] / c : 0.0f;
    const float o = 1.0f / (1.0f + expf(-opacity_logits[g]));
    const bool prune = o < min_opacity;
    const bool cand = !prune && c > 0.0f && score >= thr;
    keys[g] = cand ? __float_as_uint(score) : 0u;
    flags[g] = (prune ? kPrune : 0u) | (cand ? kCand : 0u);
    if (prune) atomicAdd(&s_c[0], 1u);
    if (cand) atomicAdd(&s_c[1], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 2 && s_c[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)s_c[threadIdx.x]);
}

// radix select state: prefix of the k-th key so far, and how many keys equal
// to the prefix (on the fixed digits) are still to be taken
struct SelState {
  uint32_t prefix, mask, k_rem, pad;
};

__global__ __launch_bounds__(256) void k_sel_hist(int n, const uint32_t* __restrict__ keys,
                                                  const SelState* __restrict__ st, int shift,
                                                  uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[256];
  s_h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t prefix = st->prefix, mask = st->mask;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
    const uint32_t k = keys[g];
    if (k != 0u && (k & mask) == prefix) atomicAdd(&s_h[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (s_h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], s_h[threadIdx.x]);
}

// one thread: the digit of the k_rem-th largest key among those matching the prefix
__global__ __launch_bounds__(64) void k_sel_pick(SelState* __restrict__ st, int shift,
                                                 uint32_t* __restrict__ hist) {
  if (threadIdx.x != 0) return;
  uint32_t above = 0u;
  int d = 255;
  for (; d > 0; --d) {
    if (above + hist[d] >= st->k_rem) break;
    above += hist[d];
  }
  st->k_rem -= above;
  st->prefix |= uint32_t(d) << shift;
  st->mask |= 255u << shift;
  for (int i = 0; i < 256; ++i) hist[i] = 0u;
}

__global__ __launch_bounds__(64) void k_sel_init(SelState* __restrict__ st, uint32_t k,
                                                 uint32_t* __restrict__ hist) {
  if (threadIdx.x == 0) *st = SelState{0u, 0u, k, 0u};
  for (int i = threadIdx.x; i < 256; i += 64) hist[i] = 0u;
}

struct TieSrc {  // keys equal to the k-th key, in index order
  const uint32_t* keys;
  const SelState* st;
  __device__ uint32_t operator()(int64_t i) const { return keys[i] == st->prefix ? 1u : 0u; }
};
struct RankDst {
  uint32_t* rank;
  __device__ void operator()(int64_t i, uint32_t pos, uint32_t) const { rank[i] = pos; }
};

// selection (mode 0: the radix-selected top k, 1: every candidate, 2: none)
// and the per-Gaussian output count (0, 1 or 2)
__global__ __launch_bounds__(256) void k_densify_mark(int n, int mode,
                                                      const uint32_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ rank,
                                                      const SelState* __restrict__ st,
                                                      const float* __restrict__ log_scales,
                                                      float max_scale, uint32_t* __restrict__ flags,
                                                      uint32_t* __restrict__ outn) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  uint32_t f = flags[g];
  bool sel = false;
  if ((f & kCand) && mode != 2) {
    const uint32_t k = keys[g];
    sel = mode == 1 || k > st->prefix || (k == st->prefix && rank[g] < st->k_rem);
  }
  if (sel) {
    const float smax = fmaxf(expf(log_scales[3 * g]),
                             fmaxf(expf(log_scales[3 * g + 1]), expf(log_scales[3 * g + 2])));
    f |= kSel | (smax > max_scale ? kSplit : 0u);
  }
  flags[g] = f;
  outn[g] = (f & kPrune) ? 0u : (sel ? 2u : 1u);
}

struct OutnSrc {
  const uint32_t* outn;
  __device__ uint32_t operator()(int64_t i) const { return outn[i]; }
};
struct OffDst {
  uint32_t* off;
  __device__ void operator()(int64_t i, uint32_t pos, uint32_t) const { off[i] = pos; }
};

struct DensifyIO {
  const float* p[5];
  const float* m[5];
  const float* v[5];
  float* po[5];
  float* mo[5];
  float* vo[5];
};

// Output row o -> (source Gaussian g, kind), packed as g << 2 | kind:
// kind 0 the Gaussian itself (moments copied), 1 a clone's copy (fresh
// moments), 2 + j split child j (fresh moments).
__global__ __launch_bounds__(256) void k_densify_src(int n, const uint32_t* __restrict__ flags,
                                                     const uint32_t* __restrict__ off,
                                                     uint32_t* __restrict__ src) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const uint32_t f = flags[g];
  if (f & kPrune) return;
  const uint32_t o = off[g], base = uint32_t(g) << 2;
  if (f & kSplit) {
    src[o] = base | 2u;
    src[o + 1] = base | 3u;
  } else {
    src[o] = base;
    if (f & kSel) src[o + 1] = base | 1u;
  }
}

// One group of the new arrays, one thread per output element (consecutive
// threads write consecutive floats of p, m and v).
template <int G, int W>
__device__ __forceinline__ void apply_group(const DensifyIO& io, const float* __restrict__ z,
                                            const uint32_t* __restrict__ src, uint32_t total) {
  const int64_t E = int64_t(total) * W;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < E; e += stride) {
    const int64_t o = e / W;
    const int k = int(e - o * W);
    const uint32_t sk = src[o];
    const size_t g = sk >> 2;
    const uint32_t kind = sk & 3u;
    const size_t i = g * W + k;
    float pv;
    if (G == 0 && kind >= 2u) {  // child mean: mu + R(q) diag(s) z_j, row k of R
      const float* q = io.p[2] + 4 * g;
      const float qinv = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      const float qw = q[0] * qinv, qx = q[1] * qinv, qy = q[2] * qinv, qz = q[3] * qinv;
      float r0, r1, r2;
      if (k == 0) {
        r0 = 1.0f - 2.0f * (qy * qy + qz * qz);
        r1 = 2.0f * (qx * qy - qw * qz);
        r2 = 2.0f * (qx * qz + qw * qy);
      } else if (k == 1) {
        r0 = 2.0f * (qx * qy + qw * qz);
        r1 = 1.0f - 2.0f * (qx * qx + qz * qz);
        r2 = 2.0f * (qy * qz - qw * qx);
      } else {
        r0 = 2.0f * (qx * qz - qw * qy);
        r1 = 2.0f * (qy * qz + qw * qx);
        r2 = 1.0f - 2.0f * (qx * qx + qy * qy);
      }
      const float* ls = io.p[1] + 3 * g;
      const float* zz = z + 6 * g + 3 * (kind - 2u);
      const float d0 = expf(ls[0]) * zz[0], d1 = expf(ls[1]) * zz[1], d2 = expf(ls[2]) * zz[2];
      pv = io.p[0][i] + (r0 * d0 + r1 * d1 + r2 * d2);
    } else if (G == 1 && kind >= 2u) {
      pv = io.p[1][i] - logf(1.6f);
    } else {
      pv = io.p[G][i];
    }
    io.po[G][e] = pv;
    io.mo[G][e] = kind == 0u ? io.m[G][i] : 0.0f;
    io.vo[G][e] = kind == 0u ? io.v[G][i] : 0.0f;
  }
}

// blockIdx.y selects the group; the row count is the plan's scan total
__global__ __launch_bounds__(256) void k_densify_apply(int n, DensifyIO io,
                                                       const float* __restrict__ z,
                                                       const uint32_t* __restrict__ src,
                                                       const uint32_t* __restrict__ off,
                                                       const uint32_t* __restrict__ outn) {
  const uint32_t total = off[n - 1] + outn[n - 1];
  switch (blockIdx.y) {
    case 0: apply_group<0, 3>(io, z, src, total); break;
    case 1: apply_group<1, 3>(io, z, src, total); break;
    case 2: apply_group<2, 4>(io, z, src, total); break;
    case 3: apply_group<3, 1>(io, z, src, total); break;
    default: apply_group<4, 48>(io, z, src, total); break;
  }
}

__global__ __launch_bounds__(64) void k_zero_u64(unsigned long long* p, int k) {
  if (int(threadIdx.x) < k) p[threadIdx.x] = 0ull;
}

struct DWs {
  size_t keys, flags, rank, outn, off, src, bsum, hist, st, cnt, bytes;
  explicit DWs(int64_t n) {
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align256(b); return r; };
    keys = take(4 * size_t(n));
    flags = take(4 * size_t(n));
    rank = take(4 * size_t(n));
    outn = take(4 * size_t(n));
    off = take(4 * size_t(n));
    src = take(8 * size_t(n));  // up to two output rows per Gaussian
    bsum = take(4 * scan_block_sums(n));
    hist = take(4 * 256);
    st = take(sizeof(SelState));
    cnt = take(8 * 4);
    bytes = o;
  }
};

}  // namespace

size_t densify_ws_bytes(int n) { return DWs(n).bytes; }

hipError_t launch_densify_stats(int n_views, int n, const char* proj, const float* mean2d_abs,
                                float scale, float* accum, float* count, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const ProjLayout L(n);
  GS_LAUNCH("k_densify_stats", k_densify_stats, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st,
            n, n_views, proj, L.stride, L.tt, mean2d_abs, scale, accum, count);
  return hipGetLastError();
}

hipError_t launch_densify_classify(int n, const float* accum, const float* count,
                                   const float* opacity_logits, float thr, float min_opacity,
                                   void* ws_, int64_t* counts_out, hipStream_t st) {
  const DWs W(n);
  char* ws = static_cast<char*>(ws_);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counts_out);
  GS_LAUNCH("k_zero_u64", k_zero_u64, dim3(1), dim3(64), 0, st, cnt, 2);
  if (n > 0)
    GS_LAUNCH("k_densify_classify", k_densify_classify, dim3(unsigned((n + 255) / 256)), dim3(256),
              0, st, n, accum, count, opacity_logits, thr, min_opacity,
              reinterpret_cast<uint32_t*>(ws + W.keys), reinterpret_cast<uint32_t*>(ws + W.flags),
              cnt);
  return hipGetLastError();
}

hipError_t launch_densify_plan(int n, int64_t k, int64_t n_cand, const float* log_scales,
                               float max_scale, void* ws_, int64_t* n_new, hipStream_t st) {
  const DWs W(n);
  char* ws = static_cast<char*>(ws_);
  uint32_t* keys = reinterpret_cast<uint32_t*>(ws + W.keys);
  uint32_t* flags = reinterpret_cast<uint32_t*>(ws + W.flags);
  uint32_t* rank = reinterpret_cast<uint32_t*>(ws + W.rank);
  uint32_t* outn = reinterpret_cast<uint32_t*>(ws + W.outn);
  uint32_t* off = reinterpret_cast<uint32_t*>(ws + W.off);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + W.hist);
  SelState* sst = reinterpret_cast<SelState*>(ws + W.st);
  const uint32_t kk = uint32_t(k > 0 ? (k < n_cand ? k : n_cand) : 0);
  const int mode = kk == 0 ? 2 : (k >= n_cand ? 1 : 0);
  GS_LAUNCH("k_sel_init", k_sel_init, dim3(1), dim3(64), 0, st, sst, kk, hist);
  const unsigned hb = unsigned(std::min<int64_t>((n + 255) / 256, 1024));
  if (mode == 0 && n > 0) {
    for (int shift = 24; shift >= 0; shift -= 8) {
      GS_LAUNCH("k_sel_hist", k_sel_hist, dim3(hb), dim3(256), 0, st, n, keys, sst, shift, hist);
      GS_LAUNCH("k_sel_pick", k_sel_pick, dim3(1), dim3(64), 0, st, sst, shift, hist);
    }
    hipError_t e = scan_exclusive(TieSrc{keys, sst}, RankDst{rank}, Count{nullptr, n}, n,
                                  reinterpret_cast<uint32_t*>(ws + W.bsum), nullptr, nullptr, st);
    if (e != hipSuccess) return e;
  }
  if (n > 0) {
    GS_LAUNCH("k_densify_mark", k_densify_mark, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st,
              n, mode, keys, rank, sst, log_scales, max_scale, flags, outn);
  }
  hipError_t e = scan_exclusive(OutnSrc{outn}, OffDst{off}, Count{nullptr, n}, n,
                                reinterpret_cast<uint32_t*>(ws + W.bsum), n_new, nullptr, st);
  if (e != hipSuccess || n == 0) return e;
  GS_LAUNCH("k_densify_src", k_densify_src, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, n,
            flags, off, reinterpret_cast<uint32_t*>(ws + W.src));
  return hipGetLastError();
}

hipError_t launch_densify_apply(int n, const float* const* p, const float* const* m,
                                const float* const* v, const float* z, const void* ws_,
                                float* const* po, float* const* mo, float* const* vo,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  const DWs W(n);
  const char* ws = static_cast<const char*>(ws_);
  DensifyIO io{};
  for (int t = 0; t < 5; ++t) {
    io.p[t] = p[t];
    io.m[t] = m[t];
    io.v[t] = v[t];
    io.po[t] = po[t];
    io.mo[t] = mo[t];
    io.vo[t] = vo[t];
  }
  const uint32_t* off = reinterpret_cast<const uint32_t*>(ws + W.off);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(ws + W.src);
  // enough blocks for the largest group (48 floats per row, up to 2n rows); the
  // smaller groups' extra blocks find no element and exit
  const unsigned gx = unsigned(std::min<int64_t>((int64_t(n) * 96 + 255) / 256, 8192));
  GS_LAUNCH("k_densify_apply", k_densify_apply, dim3(gx, 5), dim3(256), 0, st, n, io, z, src, off,
            reinterpret_cast<const uint32_t*>(ws + W.outn));
  return hipGetLastError();
}

}  // namespace gsk
