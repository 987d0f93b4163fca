// Fused multi-group Adam (the primitive update after each back-propagation)
// and the L1 photometric loss gradient.  Both are streaming, HBM-bound
// kernels: Adam moves 28 B per element (p, m, v read+write, g read), L1 12 B.
#include "gs_internal.hpp"

namespace gsk {
namespace {

struct AdamArgs {
  float* p[GS_MAX_ADAM_GROUPS];
  const float* g[GS_MAX_ADAM_GROUPS];
  float* m[GS_MAX_ADAM_GROUPS];
  float* v[GS_MAX_ADAM_GROUPS];
  int64_t numel[GS_MAX_ADAM_GROUPS];
  int64_t blk_start[GS_MAX_ADAM_GROUPS + 1];  // first block of each group (prefix)
  float lr[GS_MAX_ADAM_GROUPS];
  int32_t aligned[GS_MAX_ADAM_GROUPS];        // all four arrays 16-byte aligned
  int32_t n_groups;
  float b1, b2, eps, c1, c2;  // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
  const int32_t* step_dev;    // when set: t = *step_dev + 1 and c1, c2 are computed here
};

constexpr int kAdamThreads = 256;
constexpr int kAdamVec = 4;                                    // float4 per thread
constexpr int kAdamBlock = kAdamThreads * kAdamVec * 4;       // elements per block

// One block per 4096-element chunk of one group: every thread issues its four
// float4 loads of each array before any arithmetic (streaming, HBM-bound).
__global__ __launch_bounds__(kAdamThreads) void k_adam(AdamArgs A) {
  AdamCoef C{A.b1, A.b2, A.eps, A.c1, A.c2};
  if (A.step_dev) {  // bias corrections of step *step_dev + 1, once per block
    __shared__ float s_c[2];
    if (threadIdx.x == 0) adam_bias(A.step_dev, A.b1, A.b2, s_c[0], s_c[1]);
    __syncthreads();
    C.c1 = s_c[0];
    C.c2 = s_c[1];
  }
  const int64_t b = blockIdx.x;
  int gi = 0;
  for (int k = 1; k < A.n_groups; ++k) gi = (A.blk_start[k] <= b) ? k : gi;
  const int64_t base = (b - A.blk_start[gi]) * kAdamBlock;
  const int64_t ne = A.numel[gi];
  float* __restrict__ P = A.p[gi];
  const float* __restrict__ G = A.g[gi];
  float* __restrict__ M = A.m[gi];
  float* __restrict__ V = A.v[gi];
  const float lr = A.lr[gi];
  if (A.aligned[gi] && base + kAdamBlock <= ne) {
    float4 p4[kAdamVec], g4[kAdamVec], m4[kAdamVec], v4[kAdamVec];
#pragma unroll
    for (int k = 0; k < kAdamVec; ++k) {
      const int64_t j = base + (int64_t(k) * kAdamThreads + threadIdx.x) * 4;
      p4[k] = *reinterpret_cast<const float4*>(P + j);
      g4[k] = *reinterpret_cast<const float4*>(G + j);
      m4[k] = *reinterpret_cast<const float4*>(M + j);
      v4[k] = *reinterpret_cast<const float4*>(V + j);
    }
#pragma unroll
    for (int k = 0; k < kAdamVec; ++k) {
      adam_one(p4[k].x, g4[k].x, m4[k].x, v4[k].x, lr, C);
      adam_one(p4[k].y, g4[k].y, m4[k].y, v4[k].y, lr, C);
      adam_one(p4[k].z, g4[k].z, m4[k].z, v4[k].z, lr, C);
      adam_one(p4[k].w, g4[k].w, m4[k].w, v4[k].w, lr, C);
      const int64_t j = base + (int64_t(k) * kAdamThreads + threadIdx.x) * 4;
      *reinterpret_cast<float4*>(P + j) = p4[k];
      *reinterpret_cast<float4*>(M + j) = m4[k];
      *reinterpret_cast<float4*>(V + j) = v4[k];
    }
  } else {
    // the group's last chunk, or unaligned arrays: element by element
    const int64_t lim = (base + kAdamBlock < ne) ? base + kAdamBlock : ne;
    for (int64_t j = base + threadIdx.x; j < lim; j += kAdamThreads) {
      float pp = P[j], mm = M[j], vv = V[j];
      adam_one(pp, G[j], mm, vv, lr, C);
      P[j] = pp;
      M[j] = mm;
      V[j] = vv;
    }
  }
}

__global__ __launch_bounds__(64) void k_step_inc(int32_t* step_dev) {
  if (threadIdx.x == 0) *step_dev += 1;
}

// dL = scale * sign(img - tgt); with `vec` (16-byte aligned arrays) four values
// per load, the tail of fewer than four one by one.
__global__ __launch_bounds__(256) void k_l1(int64_t n, int vec, const float* __restrict__ img,
                                            const float* __restrict__ tgt, float scale,
                                            float* __restrict__ dL, float* __restrict__ loss) {
  float acc = 0.0f;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n4 = vec ? n >> 2 : 0;
  const float4* __restrict__ I4 = reinterpret_cast<const float4*>(img);
  const float4* __restrict__ T4 = reinterpret_cast<const float4*>(tgt);
  float4* __restrict__ D4 = reinterpret_cast<float4*>(dL);
  for (int64_t i = t0; i < n4; i += stride) {
    const float4 a = I4[i], b = T4[i];
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, dw = a.w - b.w;
    D4[i] = make_float4(l1_sign(dx, scale), l1_sign(dy, scale), l1_sign(dz, scale),
                        l1_sign(dw, scale));
    acc += (fabsf(dx) + fabsf(dy)) + (fabsf(dz) + fabsf(dw));
  }
  for (int64_t i = 4 * n4 + t0; i < n; i += stride) {
    const float d = img[i] - tgt[i];
    dL[i] = l1_sign(d, scale);
    acc += fabsf(d);
  }
  if (loss) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ float s[4];
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, scale * (s[0] + s[1] + s[2] + s[3]));
  }
}

}  // namespace

hipError_t launch_step_inc(int32_t* step_dev, hipStream_t st) {
  GS_LAUNCH("k_step_inc", k_step_inc, dim3(1), dim3(64), 0, st, step_dev);
  return hipGetLastError();
}

hipError_t launch_adam(const gs_adam_group* groups, int n_groups, int step, float beta1,
                       float beta2, float eps, int32_t* step_dev, hipStream_t st) {
  AdamArgs A{};
  A.step_dev = step_dev;
  A.n_groups = n_groups;
  int64_t blocks = 0;
  auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
  for (int k = 0; k < n_groups; ++k) {
    A.p[k] = groups[k].p;
    A.g[k] = groups[k].g;
    A.m[k] = groups[k].m;
    A.v[k] = groups[k].v;
    A.numel[k] = groups[k].numel;
    A.lr[k] = groups[k].lr;
    A.aligned[k] = al(A.p[k]) && al(A.g[k]) && al(A.m[k]) && al(A.v[k]);
    A.blk_start[k] = blocks;
    blocks += (groups[k].numel + kAdamBlock - 1) / kAdamBlock;
  }
  A.blk_start[n_groups] = blocks;
  A.b1 = beta1;
  A.b2 = beta2;
  A.eps = eps;
  A.c1 = float(1.0 / (1.0 - __builtin_pow(double(beta1), step)));
  A.c2 = float(1.0 / (1.0 - __builtin_pow(double(beta2), step)));
  if (blocks > 0)
    GS_LAUNCH("k_adam", k_adam, dim3(unsigned(blocks)), dim3(kAdamThreads), 0, st, A);
  if (step_dev) GS_LAUNCH("k_step_inc", k_step_inc, dim3(1), dim3(64), 0, st, step_dev);
  return hipGetLastError();
}

hipError_t launch_l1(int64_t numel, const float* image, const float* target, float scale,
                     float* dL, float* loss_sum, hipStream_t st) {
  if (numel == 0) return hipSuccess;
  const int vec = ((reinterpret_cast<uintptr_t>(image) | reinterpret_cast<uintptr_t>(target) |
                    reinterpret_cast<uintptr_t>(dL)) & 15u) == 0 ? 1 : 0;
  int64_t blocks = ((vec ? (numel + 3) / 4 : numel) + 255) / 256;
  if (blocks > 1024) blocks = 1024;  // few blocks: one atomic each for the loss sum
  GS_LAUNCH("k_l1", k_l1, dim3(unsigned(blocks)), dim3(256), 0, st, numel, vec, image, target,
            scale, dL, loss_sum);
  return hipGetLastError();
}

}  // namespace gsk
