// Preprocess: splat every 3D Gaussian into every view (Sec. 3: G_i -> G2D_i)
// and evaluate its view-dependent colour.  One thread per Gaussian; the
// parameters (59 floats) are read once and the views are looped in registers,
// so batched views cost one parameter read.  HBM-bound: 236 B in per Gaussian,
// 56 B out per Gaussian and view.
#include "gs_internal.hpp"

namespace gsk {
namespace {

// Real SH basis with the Condon-Shortley sign kept, k = l*l + l + m.
constexpr float SH0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float SH1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
constexpr float SH2a = 1.0925484305920792f;   // sqrt(15/pi)/2
constexpr float SH2b = 0.31539156525252005f;  // sqrt(5/pi)/4
constexpr float SH2c = 0.54627421529603959f;  // sqrt(15/pi)/4
constexpr float SH3a = 0.59004358992664352f;  // sqrt(35/(2 pi))/4
constexpr float SH3b = 2.8906114426405538f;   // sqrt(105/pi)/2
constexpr float SH3c = 0.45704579946446572f;  // sqrt(21/(2 pi))/4
constexpr float SH3d = 0.37317633259011540f;  // sqrt(7/pi)/4
constexpr float SH3e = 1.4453057213202769f;   // sqrt(105/pi)/4

__device__ inline void sh_basis(float x, float y, float z, int deg, float* Y) {
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

constexpr int kPreThreads = 128;
constexpr int kShStride = GS_SH_COEFFS * 3 + 1;  // odd LDS stride: conflict-free rows

// The view-independent part of a Gaussian: covariance and opacity.
struct Gauss3 {
  float mx, my, mz;
  float S00, S01, S02, S11, S12, S22;
  float o, k2o;
  bool opaque;
};

// One view's splat without the colour: the record words, the tile count, and
// the unit viewing direction for the colour (has_colour: the splat passed the
// culls that precede the footprint, so a colour is evaluated for it).
struct Splat {
  float4 r0, r1, r2;
  uint32_t count;
  bool has_colour;
  float dx, dy, dz;
};

__device__ __forceinline__ Splat splat_geometry(const DevView& cv, const Gauss3& G, int tile,
                                                int mip2d) {
  Splat P;
  P.r0 = make_float4(0.f, 0.f, 0.f, 0.f);
  P.r1 = P.r0;
  P.r2 = P.r0;
  P.count = 0;
  P.has_colour = false;
  P.dx = P.dy = P.dz = 0.0f;
  const float mx = G.mx, my = G.my, mz = G.mz;
  // depth: the exact float32 sequence that defines the sort key
  const float depth = __fadd_rn(
      __fadd_rn(__fadd_rn(__fmul_rn(cv.R[6], mx), __fmul_rn(cv.R[7], my)),
                __fmul_rn(cv.R[8], mz)),
      cv.t[2]);
  if (!(G.opaque && depth > cv.near_plane)) return P;
  const float xc = fmaf(cv.R[0], mx, fmaf(cv.R[1], my, fmaf(cv.R[2], mz, cv.t[0])));
  const float yc = fmaf(cv.R[3], mx, fmaf(cv.R[4], my, fmaf(cv.R[5], mz, cv.t[1])));
  const float iz = 1.0f / depth;
  const float j00 = cv.fx * iz, j11 = cv.fy * iz;
  const float j02 = -cv.fx * xc * iz * iz, j12 = -cv.fy * yc * iz * iz;
  // T = J W (2x3)
  const float t00 = j00 * cv.R[0] + j02 * cv.R[6];
  const float t01 = j00 * cv.R[1] + j02 * cv.R[7];
  const float t02 = j00 * cv.R[2] + j02 * cv.R[8];
  const float t10 = j11 * cv.R[3] + j12 * cv.R[6];
  const float t11 = j11 * cv.R[4] + j12 * cv.R[7];
  const float t12 = j11 * cv.R[5] + j12 * cv.R[8];
  // U = T Sigma, Sigma' = U T^T + low-pass
  const float u00 = t00 * G.S00 + t01 * G.S01 + t02 * G.S02;
  const float u01 = t00 * G.S01 + t01 * G.S11 + t02 * G.S12;
  const float u02 = t00 * G.S02 + t01 * G.S12 + t02 * G.S22;
  const float u10 = t10 * G.S00 + t11 * G.S01 + t12 * G.S02;
  const float u11 = t10 * G.S01 + t11 * G.S11 + t12 * G.S12;
  const float u12 = t10 * G.S02 + t11 * G.S12 + t12 * G.S22;
  const float r00 = u00 * t00 + u01 * t01 + u02 * t02;
  const float r01 = u00 * t10 + u01 * t11 + u02 * t12;
  const float r11 = u10 * t10 + u11 * t11 + u12 * t12;
  const float low = mip2d ? kMip2d : kDilation;  // screen-space low-pass
  const float c00 = r00 + low, c01 = r01, c11 = r11 + low;
  const float det = c00 * c11 - c01 * c01;
  // the 2D mip filter keeps the splat's integral: opacity times sqrt(det ratio)
  float ov = G.o, k2 = G.k2o;
  if (mip2d && det > 0.0f) {
    ov = G.o * sqrtf(fmaxf(r00 * r11 - r01 * r01, 0.0f) / det);
    k2 = fmaxf(0.0f, 2.0f * logf(255.0f * ov));
  }
  if (!(det > 0.0f && ov >= kAlphaMin)) return P;
  P.has_colour = true;
  const float idet = 1.0f / det;
  const float ca = c11 * idet, cb = -c01 * idet, cc = c00 * idet;
  // screen mean in double: float32 spacing at 1000+ px (6e-5 px) would otherwise
  // dominate the error of every pixel offset near the Gaussian
  const double xd = double(cv.R[0]) * mx + double(cv.R[1]) * my + double(cv.R[2]) * mz +
                    double(cv.t[0]);
  const double yd = double(cv.R[3]) * mx + double(cv.R[4]) * my + double(cv.R[5]) * mz +
                    double(cv.t[1]);
  const double zd = double(cv.R[6]) * mx + double(cv.R[7]) * my + double(cv.R[8]) * mz +
                    double(cv.t[2]);
  const double mux = double(cv.fx) * xd / zd + double(cv.cx);
  const double muy = double(cv.fy) * yd / zd + double(cv.cy);
  // the viewing direction of the colour
  float dx = mx - cv.campos[0], dy = my - cv.campos[1], dz = mz - cv.campos[2];
  const float dn = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
  P.dx = dx * dn;
  P.dy = dy * dn;
  P.dz = dz * dn;
  // conservative footprint box of the alpha >= 1/255 ellipse
  const double ex = double(sqrtf(k2 * c00) * (1.0f + kExtRel) + kExtAbs);
  const double ey = double(sqrtf(k2 * c11) * (1.0f + kExtRel) + kExtAbs);
  const double lox = (mux - ex) - 0.5, hix = (mux + ex) - 0.5;
  const double loy = (muy - ey) - 0.5, hiy = (muy + ey) - 0.5;
  const double Wd = double(cv.W), Hd = double(cv.H);
  const int x0 = max(int(ceil(fmin(fmax(lox, -2.0), Wd + 2.0))), 0);
  const int x1 = min(int(floor(fmin(fmax(hix, -2.0), Wd + 2.0))), cv.W - 1);
  const int y0 = max(int(ceil(fmin(fmax(loy, -2.0), Hd + 2.0))), 0);
  const int y1 = min(int(floor(fmin(fmax(hiy, -2.0), Hd + 2.0))), cv.H - 1);
  const int T = tile;
  if (x0 <= x1 && y0 <= y1) P.count = uint32_t((x1 / T - x0 / T + 1) * (y1 / T - y0 / T + 1));
  // the mean is stored relative to the origin of the first tile of the footprint
  const int ox = (x0 <= x1 ? x0 / T : 0) * T, oy = (y0 <= y1 ? y0 / T : 0) * T;
  const float s = -0.5f * kLog2e;
  P.r0 = make_float4(float(mux - double(ox)), float(muy - double(oy)), s * ca, -kLog2e * cb);
  P.r1 = make_float4(s * cc, log2f(ov), 0.0f, 0.0f);
  P.r2 = make_float4(0.0f, depth, __uint_as_float(box_pack(x0 < 0 ? 0 : x0, y0 < 0 ? 0 : y0)),
                     __uint_as_float(box_pack(x1 < 0 ? 0 : x1, y1 < 0 ? 0 : y1)));
  return P;
}

// The SH colour of a splat along its viewing direction into the record words
// (clamped channels flagged); shc holds the coefficients, zero above the degree.
__device__ __forceinline__ void splat_colour(Splat& P, const float* shc, int sh_degree,
                                             uint32_t& flags) {
  float Y[GS_SH_COEFFS];
#pragma unroll
  for (int k = 0; k < GS_SH_COEFFS; ++k) Y[k] = 0.0f;
  sh_basis(P.dx, P.dy, P.dz, sh_degree, Y);
  float rgb[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    // coefficients above the degree are zero in shc and Y
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < GS_SH_COEFFS; ++k) acc = fmaf(Y[k], shc[3 * k + ch], acc);
    acc += 0.5f;
    if (acc < 0.0f) { flags |= 1u << ch; acc = 0.0f; }
    rgb[ch] = acc;
  }
  P.r1.z = rgb[0];
  P.r1.w = rgb[1];
  P.r2.x = rgb[2];
}

__device__ __forceinline__ Gauss3 load_gauss(const Views& V, int g, const float* means,
                                             const float* log_scales, const float* quats,
                                             const float* opacity_logits) {
  Gauss3 G;
  G.mx = means[3 * g + 0];
  G.my = means[3 * g + 1];
  G.mz = means[3 * g + 2];
  const float s0 = expf(log_scales[3 * g + 0]);
  const float s1 = expf(log_scales[3 * g + 1]);
  const float s2 = expf(log_scales[3 * g + 2]);
  const float4 q4 = reinterpret_cast<const float4*>(quats)[g];
  const float qinv = 1.0f / sqrtf(q4.x * q4.x + q4.y * q4.y + q4.z * q4.z + q4.w * q4.w);
  const float qw = q4.x * qinv, qx = q4.y * qinv, qy = q4.z * qinv, qz = q4.w * qinv;
  // rotation of the unit quaternion, times the scales (M = R diag(s))
  const float m00 = (1.0f - 2.0f * (qy * qy + qz * qz)) * s0;
  const float m01 = (2.0f * (qx * qy - qw * qz)) * s1;
  const float m02 = (2.0f * (qx * qz + qw * qy)) * s2;
  const float m10 = (2.0f * (qx * qy + qw * qz)) * s0;
  const float m11 = (1.0f - 2.0f * (qx * qx + qz * qz)) * s1;
  const float m12 = (2.0f * (qy * qz - qw * qx)) * s2;
  const float m20 = (2.0f * (qx * qz - qw * qy)) * s0;
  const float m21 = (2.0f * (qy * qz + qw * qx)) * s1;
  const float m22 = (1.0f - 2.0f * (qx * qx + qy * qy)) * s2;
  // Sigma = M M^T (symmetric), plus the 3D filter's variance on the diagonal
  const float f3 = V.filter3d ? V.filter3d[g] : 0.0f;
  G.S00 = m00 * m00 + m01 * m01 + m02 * m02 + f3;
  G.S01 = m00 * m10 + m01 * m11 + m02 * m12;
  G.S02 = m00 * m20 + m01 * m21 + m02 * m22;
  G.S11 = m10 * m10 + m11 * m11 + m12 * m12 + f3;
  G.S12 = m10 * m20 + m11 * m21 + m12 * m22;
  G.S22 = m20 * m20 + m21 * m21 + m22 * m22 + f3;
  const float o0 = 1.0f / (1.0f + expf(-opacity_logits[g]));
  G.o = V.filter3d ? o0 * filter3d_coef(s0, s1, s2, f3) : o0;
  G.opaque = G.o >= kAlphaMin;
  G.k2o = fmaxf(0.0f, 2.0f * logf(255.0f * G.o));
  return G;
}

// One view: one lane per Gaussian, no LDS.  The geometry decides whether the
// Gaussian has a footprint tile; only then does the lane load its own SH row,
// twelve float4 loads issued together (with the Gaussians stored in spatial
// order, the ones outside the view form long runs of rows never read).  Free
// of LDS and at 79 VGPRs the kernel holds six waves per SIMD, against three for
// the block-staged form, whose 25 KB of LDS per block capped it; the extra
// waves hide the two dependent load phases (measured 44 -> 36 us at 1M
// Gaussians, the same records).
__global__ __launch_bounds__(kPreThreads) void k_preprocess(
    Views V, int n, int sh_degree, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ opacity_logits, const float* __restrict__ sh,
    char* __restrict__ proj) {
  const int g = blockIdx.x * kPreThreads + threadIdx.x;
  if (g >= n) return;
  const ProjLayout L(n);
  const int K = (sh_degree + 1) * (sh_degree + 1);
  const Gauss3 G = load_gauss(V, g, means, log_scales, quats, opacity_logits);
  Splat P = splat_geometry(view_at(V, 0), G, V.tile, V.mip2d);
  uint32_t flags = 0;
  if (P.count > 0) {
    constexpr int F = GS_SH_COEFFS * 3, U = F / 4;  // 12 float4 per row
    const float4* src = reinterpret_cast<const float4*>(sh + size_t(g) * F);
    float4 q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = src[u];
    float shc[F];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      shc[4 * u] = q[u].x;
      shc[4 * u + 1] = q[u].y;
      shc[4 * u + 2] = q[u].z;
      shc[4 * u + 3] = q[u].w;
    }
#pragma unroll
    for (int k = 0; k < F; ++k) shc[k] = (k < 3 * K) ? shc[k] : 0.0f;
    splat_colour(P, shc, sh_degree, flags);
  }
  float4* rec = reinterpret_cast<float4*>(proj + L.rec) + 3 * size_t(g);
  rec[0] = P.r0;
  rec[1] = P.r1;
  rec[2] = P.r2;
  reinterpret_cast<uint32_t*>(proj + L.tt)[g] = P.count;
  reinterpret_cast<uint32_t*>(proj + L.flags)[g] = flags;
}

// Several views: the block's SH coefficients (192 B per Gaussian) arrive
// through LDS once, with coalesced 16-byte loads instead of 192-byte strided
// rows per thread, and every view is splatted from registers.
__device__ __forceinline__ void stage_sh(float* s_sh, const float* __restrict__ sh, int g0,
                                         int rows) {
  constexpr int F = GS_SH_COEFFS * 3, U = F / 4;  // 12 float4 per row
  const float4* src = reinterpret_cast<const float4*>(sh + size_t(g0) * F);
  // a thread's float4s are i = t + u * kPreThreads, u < U (rows <= kPreThreads):
  // all its loads are issued before the first LDS write, so their latencies
  // overlap instead of adding up
  float4 q[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = threadIdx.x + u * kPreThreads;
    if (i < rows * U) q[u] = src[i];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int i = threadIdx.x + u * kPreThreads;
    const int f = 4 * i, row = f / F, k = f - row * F;
    if (i < rows * U) {
      float* d = s_sh + row * kShStride + k;
      d[0] = q[u].x;
      d[1] = q[u].y;
      d[2] = q[u].z;
      d[3] = q[u].w;
    }
  }
}

__global__ __launch_bounds__(kPreThreads) void k_preprocess_views(
    Views V, int n, int sh_degree, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ opacity_logits, const float* __restrict__ sh,
    char* __restrict__ proj) {
  __shared__ float s_sh[kPreThreads * kShStride];
  const int g0 = blockIdx.x * kPreThreads;
  const int g = g0 + threadIdx.x;
  const int rows = min(kPreThreads, n - g0);
  const ProjLayout L(n);
  const int K = (sh_degree + 1) * (sh_degree + 1);
  float shc[GS_SH_COEFFS * 3];
  const float* shg = s_sh + threadIdx.x * kShStride;
  stage_sh(s_sh, sh, g0, rows);
  __syncthreads();
  if (g >= n) return;
  const Gauss3 G = load_gauss(V, g, means, log_scales, quats, opacity_logits);
#pragma unroll
  for (int k = 0; k < GS_SH_COEFFS * 3; ++k) shc[k] = (k < 3 * K) ? shg[k] : 0.0f;
  for (int v = 0; v < V.n_views; ++v) {
    char* base = proj + size_t(v) * L.stride;
    Splat P = splat_geometry(view_at(V, v), G, V.tile, V.mip2d);
    uint32_t flags = 0;
    if (P.has_colour) splat_colour(P, shc, sh_degree, flags);
    float4* rec = reinterpret_cast<float4*>(base + L.rec) + 3 * size_t(g);
    rec[0] = P.r0;
    rec[1] = P.r1;
    rec[2] = P.r2;
    reinterpret_cast<uint32_t*>(base + L.tt)[g] = P.count;
    reinterpret_cast<uint32_t*>(base + L.flags)[g] = flags;
  }
}

constexpr int kF3Threads = 256;

// Mip-Splatting's 3D filter, pass 1 (per chunk of views): nu[g] = the highest
// sampling rate fx / z over the views whose image contains the centre in
// front of the near plane, folded into the previous chunks' value.
__global__ __launch_bounds__(kF3Threads) void k_filter3d_rate(Views V, int n, int first,
                                                              const float* __restrict__ means,
                                                              float* __restrict__ nu_io) {
  const int g = blockIdx.x * kF3Threads + threadIdx.x;
  if (g >= n) return;
  const float mx = means[3 * g + 0], my = means[3 * g + 1], mz = means[3 * g + 2];
  float nu = first ? 0.0f : nu_io[g];
  for (int v = 0; v < V.n_views; ++v) {
    const DevView& cv = V.v[v];
    const float z = fmaf(cv.R[6], mx, fmaf(cv.R[7], my, fmaf(cv.R[8], mz, cv.t[2])));
    if (!(z > cv.near_plane)) continue;
    const float iz = 1.0f / z;
    const float xc = fmaf(cv.R[0], mx, fmaf(cv.R[1], my, fmaf(cv.R[2], mz, cv.t[0])));
    const float yc = fmaf(cv.R[3], mx, fmaf(cv.R[4], my, fmaf(cv.R[5], mz, cv.t[1])));
    const float u = fmaf(cv.fx * xc, iz, cv.cx), w = fmaf(cv.fy * yc, iz, cv.cy);
    if (u >= 0.0f && u <= float(cv.W) && w >= 0.0f && w <= float(cv.H)) nu = fmaxf(nu, cv.fx * iz);
  }
  nu_io[g] = nu;
}

// Pass 2: variance scale / nu^2, or -1 (unseen) for now; the block's largest
// variance goes to *vmax (positive floats order like their bits).
__global__ __launch_bounds__(kF3Threads) void k_filter3d_var(int n, float scale,
                                                             float* __restrict__ var,
                                                             uint32_t* __restrict__ vmax) {
  __shared__ uint32_t s_max[kF3Threads / kWave];
  const int g = blockIdx.x * kF3Threads + threadIdx.x;
  float r = -1.0f;
  if (g < n) {
    const float nu = var[g];
    if (nu > 0.0f) r = scale / (nu * nu);
    var[g] = r;
  }
  uint32_t b = r > 0.0f ? __float_as_uint(r) : 0u;
  for (int off = kWave / 2; off > 0; off >>= 1) b = max(b, uint32_t(__shfl_xor(int(b), off)));
  if ((threadIdx.x & (kWave - 1)) == 0) s_max[threadIdx.x / kWave] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0u;
    for (int k = 0; k < kF3Threads / kWave; ++k) m = max(m, s_max[k]);
    if (m) atomicMax(vmax, m);
  }
}

__global__ __launch_bounds__(64) void k_set_u32(uint32_t* p, uint32_t x) {
  if (threadIdx.x == 0) *p = x;
}

// Pass 3: unseen Gaussians take the largest variance (0 if none was seen).
__global__ __launch_bounds__(kF3Threads) void k_filter3d_unseen(int n, float* __restrict__ var,
                                                                const uint32_t* __restrict__ vmax) {
  const int g = blockIdx.x * kF3Threads + threadIdx.x;
  if (g < n && var[g] < 0.0f) var[g] = __uint_as_float(*vmax);
}

}  // namespace

hipError_t launch_filter3d_rate(const Views& V, int n, int first, const float* means, float* nu,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  GS_LAUNCH("k_filter3d_rate", k_filter3d_rate, dim3(unsigned((n + kF3Threads - 1) / kF3Threads)),
            dim3(kF3Threads), 0, st, V, n, first, means, nu);
  return hipGetLastError();
}

hipError_t launch_filter3d_var(int n, float scale, float* variance, uint32_t* scratch,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned nb = unsigned((n + kF3Threads - 1) / kF3Threads);
  GS_LAUNCH("k_set_u32", k_set_u32, dim3(1), dim3(64), 0, st, scratch, 0u);
  GS_LAUNCH("k_filter3d_var", k_filter3d_var, dim3(nb), dim3(kF3Threads), 0, st, n, scale,
            variance, scratch);
  GS_LAUNCH("k_filter3d_unseen", k_filter3d_unseen, dim3(nb), dim3(kF3Threads), 0, st, n,
            variance, scratch);
  return hipGetLastError();
}

hipError_t launch_preprocess(const Views& V, int n, int sh_degree, const float* means,
                             const float* log_scales, const float* quats,
                             const float* opacity_logits, const float* sh, char* proj,
                             hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int nb = (n + kPreThreads - 1) / kPreThreads;
  if (V.n_views == 1)
    GS_LAUNCH("k_preprocess", k_preprocess, dim3(nb), dim3(kPreThreads), 0, st, V, n, sh_degree,
              means, log_scales, quats, opacity_logits, sh, proj);
  else
    GS_LAUNCH("k_preprocess_views", k_preprocess_views, dim3(nb), dim3(kPreThreads), 0, st, V, n,
              sh_degree, means, log_scales, quats, opacity_logits, sh, proj);
  return hipGetLastError();
}

}  // namespace gsk
