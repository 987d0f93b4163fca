// The frequency-guided resolution schedule (Sec. 4.2, Eq. 2; supplementary
// Eq. 6-7) and the anti-aliased downsampling of the ground-truth views
// (supplementary, "Ground Truth Downsampling").
//
// Frequency map: M(i,j) = (1/N) sum_n ||F^n(i,j)||_2 with F^n the
// unnormalised 2D DFT of view n and the norm taken over the colour channels.
// It is computed once per scene, in FP64, as a direct DFT: a row pass on the
// real image (only the non-negative column frequencies: the rest follow by
// conjugate symmetry) and a column pass per output column, which takes the
// norm over channels.  O(HW(H + W)) work: about 0.5 ms for a 1600x1064 view.
// Views are added in order, so the map is deterministic.  H and W are at most
// kDftMax (both passes keep their twiddles and one line of data in LDS).
//
// Schedule: from the map, X(F_r) is the sum of M over the centred crop
// |k_y| <= H/(2r), |k_x| <= W/(2r) (the spectrum of the ideal downsample by r),
// scaled by 1/r^2 (Eq. 2 with unnormalised DFTs) or by 1/(H W) (each view's
// DFT normalised by its pixel count); r_m solves X(F_r) = X(F)/a, the knots X_1..X_{m-1} are
// spaced linearly between X(F) and X(F_{r_m}) and solved for r_i by
// bisection, and Eq. 7 places them at s_{r_i} = S ln(X_i/X_m) / ln(X_F/X_m).
// This part is host code over a summed-area table of the map.
//
// Downsampling: separable anti-aliased linear resampling; output sample i is
// centred at input coordinate (i + 0.5) * in/out and weighs the inputs with a
// triangle of half-width max(1, in/out), normalised to sum 1.
#include <cmath>
#include <vector>

#include "gs_internal.hpp"

namespace gsk {
namespace {

constexpr int kDftThreads = 256;

// twiddles e^{-2 pi i k / n} for k < n (cos, sin as double2)
__global__ __launch_bounds__(256) void k_twiddles(int n, double2* __restrict__ tw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s, c;
  sincospi(2.0 * double(k) / double(n), &s, &c);
  tw[k] = make_double2(c, -s);
}

// Row pass: one block per (channel, row) of one image; outputs the
// non-negative column frequencies kx = 0 .. W/2 of that row.
__global__ __launch_bounds__(kDftThreads) void k_dft_rows(int H, int W, const float* __restrict__ img,
                                                          const double2* __restrict__ tw,
                                                          double2* __restrict__ rows) {
  extern __shared__ double2 s_tw[];  // W twiddles, then the row (W doubles)
  double* s_row = reinterpret_cast<double*>(s_tw + W);
  const int y = blockIdx.x, c = blockIdx.y;
  const float* src = img + (size_t(c) * H + y) * W;
  for (int x = threadIdx.x; x < W; x += kDftThreads) {
    s_row[x] = double(src[x]);
    s_tw[x] = tw[x];
  }
  __syncthreads();
  const int nk = W / 2 + 1;
  double2* dst = rows + (size_t(c) * H + y) * nk;
  for (int k = threadIdx.x; k < nk; k += kDftThreads) {
    double re = 0.0, im = 0.0;
    int idx = 0;  // (x * k) mod W
    for (int x = 0; x < W; ++x) {
      const double2 w = s_tw[idx];
      re = fma(s_row[x], w.x, re);
      im = fma(s_row[x], w.y, im);
      idx += k;
      if (idx >= W) idx -= W;
    }
    dst[k] = make_double2(re, im);
  }
}

// Column pass: one block per column frequency kx in 0 .. W/2; for each channel
// the column of row spectra goes through LDS and every thread forms its output
// rows ky, summing |F_c|^2 over the channels.  Writes M(ky, kx) and, by
// conjugate symmetry, M(-ky, -kx); the image's norm is added to the running
// mean (first image: overwrite).
constexpr int kColOut = 16;  // outputs per thread: H <= kDftThreads * kColOut

__global__ __launch_bounds__(kDftThreads) void k_dft_cols(int H, int W, const double2* __restrict__ rows,
                                                          const double2* __restrict__ tw,
                                                          double inv_n, int first,
                                                          double* __restrict__ mag) {
  extern __shared__ double2 s_tw[];  // H twiddles, then the column (H values)
  double2* s_col = s_tw + H;
  const int kx = blockIdx.x, nk = W / 2 + 1;
  for (int y = threadIdx.x; y < H; y += kDftThreads) s_tw[y] = tw[y];
  double acc[kColOut];
#pragma unroll
  for (int j = 0; j < kColOut; ++j) acc[j] = 0.0;
  for (int c = 0; c < 3; ++c) {
    __syncthreads();  // the previous channel's column is consumed
    for (int y = threadIdx.x; y < H; y += kDftThreads)
      s_col[y] = rows[(size_t(c) * H + y) * nk + kx];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kColOut; ++j) {
      const int ky = threadIdx.x + j * kDftThreads;
      if (ky < H) {
        double re = 0.0, im = 0.0;
        int idx = 0;  // (y * ky) mod H
        for (int y = 0; y < H; ++y) {
          const double2 a = s_col[y], w = s_tw[idx];
          re = fma(a.x, w.x, fma(-a.y, w.y, re));
          im = fma(a.x, w.y, fma(a.y, w.x, im));
          idx += ky;
          if (idx >= H) idx -= H;
        }
        acc[j] = fma(re, re, fma(im, im, acc[j]));
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kColOut; ++j) {
    const int ky = threadIdx.x + j * kDftThreads;
    if (ky < H) {
      const double v = sqrt(acc[j]) * inv_n;
      const size_t o = size_t(ky) * W + kx;
      mag[o] = first ? v : mag[o] + v;
      // the mirrored frequency (-ky, -kx), when it is a different column
      const int mx = (W - kx) % W;
      if (mx != kx && mx >= nk) {
        const size_t om = size_t((H - ky) % H) * W + mx;
        mag[om] = first ? v : mag[om] + v;
      }
    }
  }
}

// Anti-aliased downsampling of [n][C][H][W] to [n][C][h][w], one thread per
// output value, both axes' triangle weights formed on the fly.  Coordinates,
// weights and sums are FP64: in FP32 the tap centre (i + 0.5) H / h carries an
// error of 1e-4 px near H = 1000, which moves non-integer-factor weights.
__global__ __launch_bounds__(256) void k_downsample(int64_t total, int H, int W, int h, int w,
                                                    const float* __restrict__ src,
                                                    float* __restrict__ dst) {
  const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= total) return;
  const int j = int(o % w), i = int((o / w) % h);
  const int64_t plane = o / (int64_t(w) * h);
  const float* s = src + plane * int64_t(H) * W;
  const double sy = double(H) / double(h), sx = double(W) / double(w);
  const double hy = fmax(sy, 1.0), hx = fmax(sx, 1.0);
  const double cy = (double(i) + 0.5) * sy, cx = (double(j) + 0.5) * sx;
  // inputs with |(p + 0.5) - c| < half lie in (c - half - 0.5, c + half - 0.5)
  const int y0 = max(0, int(floor(cy - hy - 0.5))), y1 = min(H - 1, int(ceil(cy + hy - 0.5)));
  const int x0 = max(0, int(floor(cx - hx - 0.5))), x1 = min(W - 1, int(ceil(cx + hx - 0.5)));
  double wsum_x = 0.0;
  for (int x = x0; x <= x1; ++x) wsum_x += fmax(0.0, 1.0 - fabs((double(x) + 0.5 - cx) / hx));
  double acc = 0.0, wsum_y = 0.0;
  for (int y = y0; y <= y1; ++y) {
    const double wy = fmax(0.0, 1.0 - fabs((double(y) + 0.5 - cy) / hy));
    if (wy == 0.0) continue;
    wsum_y += wy;
    double row = 0.0;
    const float* sr = s + int64_t(y) * W;
    for (int x = x0; x <= x1; ++x)
      row = fma(fmax(0.0, 1.0 - fabs((double(x) + 0.5 - cx) / hx)), double(sr[x]), row);
    acc = fma(wy, row, acc);
  }
  dst[o] = float(acc / (wsum_x * wsum_y));
}

}  // namespace

size_t frequency_map_ws_bytes(int H, int W) {
  return align256(size_t(3) * H * (W / 2 + 1) * sizeof(double2)) +
         align256(size_t(W) * sizeof(double2)) + align256(size_t(H) * sizeof(double2));
}

hipError_t launch_frequency_map(int n_images, int H, int W, const float* images, double* mag,
                                void* ws, hipStream_t st) {
  char* p = static_cast<char*>(ws);
  double2* rows = reinterpret_cast<double2*>(p);
  p += align256(size_t(3) * H * (W / 2 + 1) * sizeof(double2));
  double2* tw_w = reinterpret_cast<double2*>(p);
  p += align256(size_t(W) * sizeof(double2));
  double2* tw_h = reinterpret_cast<double2*>(p);
  GS_LAUNCH("k_twiddles", k_twiddles, dim3(unsigned((W + 255) / 256)), dim3(256), 0, st, W, tw_w);
  GS_LAUNCH("k_twiddles", k_twiddles, dim3(unsigned((H + 255) / 256)), dim3(256), 0, st, H, tw_h);
  const double inv_n = 1.0 / double(n_images);
  for (int k = 0; k < n_images; ++k) {
    const float* img = images + size_t(k) * 3 * H * W;
    GS_LAUNCH("k_dft_rows", k_dft_rows, dim3(unsigned(H), 3u), dim3(kDftThreads),
              size_t(W) * (sizeof(double2) + sizeof(double)), st, H, W, img, tw_w, rows);
    GS_LAUNCH("k_dft_cols", k_dft_cols, dim3(unsigned(W / 2 + 1)), dim3(kDftThreads),
              size_t(H) * 2 * sizeof(double2), st, H, W, rows, tw_h, inv_n, k == 0 ? 1 : 0, mag);
  }
  return hipGetLastError();
}

hipError_t launch_downsample(int n_planes, int H, int W, int h, int w, const float* src, float* dst,
                             hipStream_t st) {
  const int64_t total = int64_t(n_planes) * h * w;
  if (total == 0) return hipSuccess;
  GS_LAUNCH("k_downsample", k_downsample, dim3(unsigned((total + 255) / 256)), dim3(256), 0, st,
            total, H, W, h, w, src, dst);
  return hipGetLastError();
}

// ---- host: crop significance over a summed-area table of the centred map
struct CropTable {
  int H, W;
  std::vector<double> sat;  // (H+1) x (W+1) prefix sums of the map with DC at (H/2, W/2)
  CropTable(const double* mag, int H_, int W_) : H(H_), W(W_), sat(size_t(H_ + 1) * (W_ + 1), 0.0) {
    for (int j = 0; j < H; ++j) {
      const int ky = (j + H - H / 2) % H;  // centred row j holds frequency j - H/2
      double run = 0.0;
      for (int i = 0; i < W; ++i) {
        const int kx = (i + W - W / 2) % W;
        run += mag[size_t(ky) * W + kx];
        sat[size_t(j + 1) * (W + 1) + (i + 1)] = sat[size_t(j) * (W + 1) + (i + 1)] + run;
      }
    }
  }
  // sum of the map over |f_y| <= H/(2r), |f_x| <= W/(2r), times 1/r^2 or 1/(H W)
  bool per_pixel = false;
  double significance(double r) const {
    const int by = int(std::floor(double(H) / (2.0 * r))), bx = int(std::floor(double(W) / (2.0 * r)));
    const int y0 = std::max(0, H / 2 - by), y1 = std::min(H - 1, H / 2 + by);
    const int x0 = std::max(0, W / 2 - bx), x1 = std::min(W - 1, W / 2 + bx);
    const double s = sat[size_t(y1 + 1) * (W + 1) + (x1 + 1)] - sat[size_t(y0) * (W + 1) + (x1 + 1)] -
                     sat[size_t(y1 + 1) * (W + 1) + x0] + sat[size_t(y0) * (W + 1) + x0];
    return per_pixel ? s / (double(H) * double(W)) : s / (r * r);
  }
  // largest r in [1, r_max] with significance(r) >= target (bisection)
  double solve(double target, double r_max) const {
    if (significance(r_max) >= target) return r_max;
    double lo = 1.0, hi = r_max;
    for (int it = 0; it < 60; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (significance(mid) >= target)
        lo = mid;
      else
        hi = mid;
    }
    return lo;
  }
};

void resolution_schedule(const double* mag, int H, int W, double S, double a, int m, double r_max,
                         int per_pixel, double* r_knots, double* s_knots, double* x_knots) {
  CropTable T(mag, H, W);
  T.per_pixel = per_pixel != 0;
  const double XF = T.significance(1.0), Xm = XF / a;
  for (int i = 0; i <= m; ++i) {
    const double Xi = XF - (XF - Xm) * double(i) / double(m);
    r_knots[i] = (i == 0) ? 1.0 : T.solve(Xi, r_max);
    s_knots[i] = S * std::log(Xi / Xm) / std::log(XF / Xm);
    if (x_knots) x_knots[i] = Xi;
  }
}

}  // namespace gsk
