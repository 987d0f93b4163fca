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
  int64_t start[GS_MAX_ADAM_GROUPS + 1];  // prefix over groups, in elements
  float lr[GS_MAX_ADAM_GROUPS];
  int32_t n_groups;
  float b1, b2, eps, c1, c2;  // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
};

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr,
                                         const AdamArgs& A) {
  m = fmaf(A.b1, m, (1.0f - A.b1) * g);
  v = fmaf(A.b2, v, (1.0f - A.b2) * g * g);
  const float mh = m * A.c1;
  const float vh = v * A.c2;
  p -= lr * mh / (sqrtf(vh) + A.eps);
}

// grid-stride over the concatenated groups; 4 elements per thread-step where aligned
__global__ __launch_bounds__(256) void k_adam(AdamArgs A) {
  const int64_t total = A.start[A.n_groups];
  const int64_t nthreads = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i4 = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * 4; i4 < total;
       i4 += nthreads * 4) {
    int gi = 0;
    for (int k = 1; k < A.n_groups; ++k) gi = (A.start[k] <= i4) ? k : gi;
    const int64_t j = i4 - A.start[gi];
    const int64_t ne = A.numel[gi];
    float* P = A.p[gi];
    const float* G = A.g[gi];
    float* M = A.m[gi];
    float* V = A.v[gi];
    const float lr = A.lr[gi];
    const bool vec = (j + 4 <= ne) &&
                     ((reinterpret_cast<uintptr_t>(P + j) | reinterpret_cast<uintptr_t>(G + j) |
                       reinterpret_cast<uintptr_t>(M + j) | reinterpret_cast<uintptr_t>(V + j)) &
                      15u) == 0;
    if (vec) {
      float4 p4 = *reinterpret_cast<float4*>(P + j);
      const float4 g4 = *reinterpret_cast<const float4*>(G + j);
      float4 m4 = *reinterpret_cast<float4*>(M + j);
      float4 v4 = *reinterpret_cast<float4*>(V + j);
      adam_one(p4.x, g4.x, m4.x, v4.x, lr, A);
      adam_one(p4.y, g4.y, m4.y, v4.y, lr, A);
      adam_one(p4.z, g4.z, m4.z, v4.z, lr, A);
      adam_one(p4.w, g4.w, m4.w, v4.w, lr, A);
      *reinterpret_cast<float4*>(P + j) = p4;
      *reinterpret_cast<float4*>(M + j) = m4;
      *reinterpret_cast<float4*>(V + j) = v4;
    } else {
      // group tail or unaligned pointers: element by element (group starts are padded to
      // multiples of 4, so the 4 slots of this step belong to group gi; padding is skipped)
      for (int e = 0; e < 4; ++e) {
        const int64_t jj = j + e;
        if (jj >= ne) break;
        float pp = P[jj], mm = M[jj], vv = V[jj];
        adam_one(pp, G[jj], mm, vv, lr, A);
        P[jj] = pp;
        M[jj] = mm;
        V[jj] = vv;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_l1(int64_t n, const float* __restrict__ img,
                                            const float* __restrict__ tgt, float scale,
                                            float* __restrict__ dL, float* __restrict__ loss) {
  float acc = 0.0f;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const float d = img[i] - tgt[i];
    dL[i] = (d > 0.0f) ? scale : ((d < 0.0f) ? -scale : 0.0f);
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

hipError_t launch_adam(const gs_adam_group* groups, int n_groups, int step, float beta1,
                       float beta2, float eps, hipStream_t st) {
  AdamArgs A{};
  A.n_groups = n_groups;
  int64_t acc = 0;
  for (int k = 0; k < n_groups; ++k) {
    A.p[k] = groups[k].p;
    A.g[k] = groups[k].g;
    A.m[k] = groups[k].m;
    A.v[k] = groups[k].v;
    A.numel[k] = groups[k].numel;
    A.lr[k] = groups[k].lr;
    A.start[k] = acc;
    // groups start on a multiple of 4 elements so each vector step stays in one group
    acc += (groups[k].numel + 3) & ~int64_t(3);
  }
  A.start[n_groups] = acc;
  A.b1 = beta1;
  A.b2 = beta2;
  A.eps = eps;
  A.c1 = float(1.0 / (1.0 - __builtin_pow(double(beta1), step)));
  A.c2 = float(1.0 / (1.0 - __builtin_pow(double(beta2), step)));
  if (acc == 0) return hipSuccess;
  int64_t blocks = (acc / 4 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  GS_LAUNCH("k_adam", k_adam, dim3(unsigned(blocks)), dim3(256), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_l1(int64_t numel, const float* image, const float* target, float scale,
                     float* dL, float* loss_sum, hipStream_t st) {
  if (numel == 0) return hipSuccess;
  int64_t blocks = (numel + 255) / 256;
  if (blocks > 1024) blocks = 1024;  // few blocks: one atomic each for the loss sum
  GS_LAUNCH("k_l1", k_l1, dim3(unsigned(blocks)), dim3(256), 0, st, numel, image, target, scale,
                     dL, loss_sum);
  return hipGetLastError();
}

}  // namespace gsk
