// Membrane force and trapezoid weights on gfx950: the step that produces the far-field
// sum's inputs on the device.
//
//   f = -kappa_b X_ssss + (sigma X_s)_s            (eq. (elastic_force))
//   w = |X_alpha| 2 pi / N                          (the ds of eq. (single_layer))
//
// Arclength derivatives are spectral (Section 2.2.1): d/ds = (1/|X_alpha|) d/dalpha with
// d/dalpha exact on the band-limited interpolant of the N points alpha_k = 2 pi k / N.
// On the grid that operator is the circulant matrix with first column
//   d_0 = 0,  d_m = (1/2) (-1)^m cot(pi m / N)  (N even),  (1/2) (-1)^m csc(pi m / N)  (N odd),
// which equals multiplying Fourier mode k by i k with the even-N Nyquist mode dropped.  The weights sum
// to zero, so the points enter it relative to the vesicle's first point: rounding then scales with the
// vesicle's extent, not with its distance from the origin.  It is applied as
// a direct O(N^2) sum from LDS in float64 (the fourth derivative amplifies rounding by up to (N/2)^4):
// one wavefront per vesicle of up to 64, 128 or 256 points (k_elastic_wave), one workgroup per larger
// vesicle of up to 1024 points (k_elastic), tens of microseconds for a whole suspension.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vesnet_internal.h"

namespace vesnet {

namespace {

constexpr int kMaxN = 1024;
constexpr int kB = 256;
constexpr int kPer = kMaxN / kB;

__device__ __forceinline__ int clamp_i(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// (D u)_i for the points this thread owns, u and d in LDS.
__device__ __forceinline__ void apply_d(const double* __restrict__ d, const double* __restrict__ ux,
                                        const double* __restrict__ uy, int n, double (&ox)[kPer],
                                        double (&oy)[kPer]) {
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = threadIdx.x + k * kB;
    double sx = 0.0, sy = 0.0;
    if (i < n) {
      int idx = i;  // (i - m) mod n, walking m = 0 .. n-1
      for (int m = 0; m < n; ++m) {
        const double c = d[m];
        sx = fma(c, ux[idx], sx);
        sy = fma(c, uy[idx], sy);
        idx = idx == 0 ? n - 1 : idx - 1;
      }
    }
    ox[k] = sx;
    oy[k] = sy;
  }
}

// LDS position of value j in k_elastic_wave's arrays (one spare double every eight), so that lanes reading
// values R apart fall in different banks.
__device__ __forceinline__ int pad8(int j) { return j + (j >> 3); }

// (D u) at the R consecutive points i0 .. i0 + R - 1 of this lane, u stored twice (u2[j] = u2[j + n] = u_j) so
// that u_(i - m) mod n is u2[i + n - m].  A window of the R values slides down one position per m: each step
// reads one new value per component for 2 R FMAs, and every output sums m = 0 .. n-1 in order, as apply_d
// does.  Points beyond n only ever see window values of points beyond n; their outputs are not used.
template <int R>
__device__ __forceinline__ void apply_d_lane(const double* __restrict__ d, const double* __restrict__ ux2,
                                             const double* __restrict__ uy2, int n, int i0, double (&ox)[R],
                                             double (&oy)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) ox[r] = oy[r] = 0.0;
  if (i0 >= n) return;
  double wx[R], wy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    wx[r] = ux2[pad8(i0 + r + n)];
    wy[r] = uy2[pad8(i0 + r + n)];
  }
  for (int m = 0; m < n; ++m) {
    const double c = d[m];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ox[r] = fma(c, wx[r], ox[r]);
      oy[r] = fma(c, wy[r], oy[r]);
    }
#pragma unroll
    for (int r = R - 1; r > 0; --r) {
      wx[r] = wx[r - 1];
      wy[r] = wy[r - 1];
    }
    wx[0] = ux2[pad8(i0 + n - m - 1)];
    wy[0] = uy2[pad8(i0 + n - m - 1)];
  }
}

// k_elastic for vesicles of at most 64 R points: one wavefront per vesicle, lane l owning points R l ..
// R l + R - 1, and LDS sized by 64 R (the derivative weights, then u_x and u_y stored twice), so that many
// vesicles share a compute unit.  Larger vesicles are left to k_elastic.  The arithmetic of every point is
// that of k_elastic, in the same order.
template <int R>
__global__ __launch_bounds__(64) void k_elastic_wave(const double* __restrict__ X, const double* __restrict__ sigma,
                                                     double kappa_b, const int32_t* __restrict__ off, int M, int P,
                                                     double* __restrict__ f, double* __restrict__ w) {
  constexpr int kCap = 64 * R;
  extern __shared__ double es[];
  double* d = es;
  double* ux = es + kCap;
  double* uy = ux + pad8(2 * kCap);
  const double two_pi = 6.28318530717958647693;
  const int lane = threadIdx.x, i0 = R * lane;
  for (int v = blockIdx.x; v < M; v += gridDim.x) {
    const int j0 = clamp_i(off[v], 0, P);
    const int j1 = max(j0, clamp_i(off[v + 1], 0, P));
    const int n = j1 - j0;
    if (n == 0 || n > kCap) continue;
    wave_sync();  // the previous vesicle is done with LDS
    for (int m = lane; m < n; m += 64) {
      double c = 0.0;
      if (m > 0) {
        double s, co;
        sincospi((double)m / (double)n, &s, &co);
        const double sg = (m & 1) ? -0.5 : 0.5;
        c = (n & 1) ? sg / s : sg * co / s;
      }
      d[m] = c;
      ux[pad8(m)] = ux[pad8(m + n)] = X[j0 + m] - X[j0];
      uy[pad8(m)] = uy[pad8(m + n)] = X[P + j0 + m] - X[P + j0];
    }
    wave_sync();
    double ax[R], ay[R], jinv[R], sx[R], sy[R], tx[R], ty[R], bx[R], by[R];
    apply_d_lane<R>(d, ux, uy, n, i0, ax, ay);  // X_alpha
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double J = sqrt(ax[r] * ax[r] + ay[r] * ay[r]);
      jinv[r] = 1.0 / J;
      sx[r] = ax[r] * jinv[r];  // X_s
      sy[r] = ay[r] * jinv[r];
      const int i = i0 + r;
      if (i < n) w[j0 + i] = J * (two_pi / (double)n);
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r;
      if (i < n) {
        ux[pad8(i)] = ux[pad8(i + n)] = sx[r];
        uy[pad8(i)] = uy[pad8(i + n)] = sy[r];
      }
    }
    wave_sync();
    apply_d_lane<R>(d, ux, uy, n, i0, bx, by);  // X_ss * J
#pragma unroll
    for (int r = 0; r < R; ++r) { bx[r] *= jinv[r]; by[r] *= jinv[r]; }
    // tension term (sigma X_s)_s
#pragma unroll
    for (int r = 0; r < R; ++r) tx[r] = ty[r] = 0.0;
    if (sigma) {
      wave_sync();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + r;
        if (i < n) {
          const double sg = sigma[j0 + i];
          ux[pad8(i)] = ux[pad8(i + n)] = sg * sx[r];
          uy[pad8(i)] = uy[pad8(i + n)] = sg * sy[r];
        }
      }
      wave_sync();
      apply_d_lane<R>(d, ux, uy, n, i0, tx, ty);
#pragma unroll
      for (int r = 0; r < R; ++r) { tx[r] *= jinv[r]; ty[r] *= jinv[r]; }
    }
    // X_sss, then X_ssss
    for (int pass = 0; pass < 2; ++pass) {
      wave_sync();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + r;
        if (i < n) {
          ux[pad8(i)] = ux[pad8(i + n)] = bx[r];
          uy[pad8(i)] = uy[pad8(i + n)] = by[r];
        }
      }
      wave_sync();
      apply_d_lane<R>(d, ux, uy, n, i0, bx, by);
#pragma unroll
      for (int r = 0; r < R; ++r) { bx[r] *= jinv[r]; by[r] *= jinv[r]; }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = i0 + r;
      if (i < n) {
        f[j0 + i] = fma(-kappa_b, bx[r], tx[r]);
        f[P + j0 + i] = fma(-kappa_b, by[r], ty[r]);
      }
    }
  }
}

__global__ __launch_bounds__(kB) void k_elastic(const double* __restrict__ X, const double* __restrict__ sigma,
                                                double kappa_b, const int32_t* __restrict__ off, int M, int P,
                                                double* __restrict__ f, double* __restrict__ w, int min_n) {
  __shared__ double d[kMaxN];
  __shared__ double ux[kMaxN];
  __shared__ double uy[kMaxN];
  const double two_pi = 6.28318530717958647693;
  for (int v = blockIdx.x; v < M; v += gridDim.x) {
    const int j0 = clamp_i(off[v], 0, P);
    const int j1 = max(j0, clamp_i(off[v + 1], 0, P));
    const int n = j1 - j0;
    if (n <= min_n) continue;  // empty, or done by k_elastic_wave
    if (n > kMaxN) {
      for (int i = threadIdx.x; i < n; i += kB) {
        f[j0 + i] = NAN;
        f[P + j0 + i] = NAN;
        w[j0 + i] = NAN;
      }
      continue;
    }
    __syncthreads();  // the previous vesicle is done with LDS
    for (int m = threadIdx.x; m < n; m += kB) {
      double c = 0.0;
      if (m > 0) {
        double s, co;
        sincospi((double)m / (double)n, &s, &co);
        const double sg = (m & 1) ? -0.5 : 0.5;
        c = (n & 1) ? sg / s : sg * co / s;
      }
      d[m] = c;
      ux[m] = X[j0 + m] - X[j0];
      uy[m] = X[P + j0 + m] - X[P + j0];
    }
    __syncthreads();

    double ax[kPer], ay[kPer], jinv[kPer], sx[kPer], sy[kPer], tx[kPer], ty[kPer], bx[kPer], by[kPer];
    apply_d(d, ux, uy, n, ax, ay);  // X_alpha
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const double J = sqrt(ax[k] * ax[k] + ay[k] * ay[k]);
      jinv[k] = 1.0 / J;
      sx[k] = ax[k] * jinv[k];  // X_s
      sy[k] = ay[k] * jinv[k];
      const int i = threadIdx.x + k * kB;
      if (i < n) w[j0 + i] = J * (two_pi / (double)n);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = threadIdx.x + k * kB;
      if (i < n) { ux[i] = sx[k]; uy[i] = sy[k]; }
    }
    __syncthreads();
    apply_d(d, ux, uy, n, bx, by);  // X_ss * J
#pragma unroll
    for (int k = 0; k < kPer; ++k) { bx[k] *= jinv[k]; by[k] *= jinv[k]; }
    // tension term (sigma X_s)_s
#pragma unroll
    for (int k = 0; k < kPer; ++k) tx[k] = ty[k] = 0.0;
    if (sigma) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int i = threadIdx.x + k * kB;
        if (i < n) {
          const double sg = sigma[j0 + i];
          ux[i] = sg * sx[k];
          uy[i] = sg * sy[k];
        }
      }
      __syncthreads();
      apply_d(d, ux, uy, n, tx, ty);
#pragma unroll
      for (int k = 0; k < kPer; ++k) { tx[k] *= jinv[k]; ty[k] *= jinv[k]; }
    }
    // X_sss, then X_ssss
    for (int pass = 0; pass < 2; ++pass) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int i = threadIdx.x + k * kB;
        if (i < n) { ux[i] = bx[k]; uy[i] = by[k]; }
      }
      __syncthreads();
      apply_d(d, ux, uy, n, bx, by);
#pragma unroll
      for (int k = 0; k < kPer; ++k) { bx[k] *= jinv[k]; by[k] *= jinv[k]; }
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = threadIdx.x + k * kB;
      if (i < n) {
        f[j0 + i] = fma(-kappa_b, bx[k], tx[k]);
        f[P + j0 + i] = fma(-kappa_b, by[k], ty[k]);
      }
    }
  }
}

// Sum of one value per thread over the workgroup in a fixed order (waves in index order).
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  __syncthreads();  // red is free
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kB / 64; ++k) s += red[k];
  return s;
}

// CreateNearLayers (Algorithm 4, Section 3.3): node a = l * n + k of vesicle v is membrane point
// k moved along the outward unit normal by d_l = (l - 2) h_v / 2, l = 0..4.  The tangent is the
// spectral X_alpha / |X_alpha|; the outward side is fixed by the sign of the enclosed signed area
// (trapezoid rule of (x y_alpha - y x_alpha) / 2), so either orientation of the points works.
__global__ __launch_bounds__(kB) void k_near_layers(const double* __restrict__ X, const double* __restrict__ w,
                                                    const int32_t* __restrict__ off, int M, int P,
                                                    double* __restrict__ layers) {
  __shared__ double d[kMaxN];
  __shared__ double ux[kMaxN];
  __shared__ double uy[kMaxN];
  __shared__ double red[kB / 64];
  const size_t P5 = (size_t)5 * P;
  for (int v = blockIdx.x; v < M; v += gridDim.x) {
    const int j0 = clamp_i(off[v], 0, P);
    const int j1 = max(j0, clamp_i(off[v + 1], 0, P));
    const int n = j1 - j0;
    if (n == 0) continue;
    double* lx = layers + (size_t)5 * j0;
    double* ly = layers + P5 + (size_t)5 * j0;
    if (n > kMaxN || n < 3) {
      for (int a = threadIdx.x; a < 5 * n; a += kB) {
        lx[a] = NAN;
        ly[a] = NAN;
      }
      continue;
    }
    __syncthreads();  // the previous vesicle is done with LDS
    for (int m = threadIdx.x; m < n; m += kB) {
      double c = 0.0;
      if (m > 0) {
        double s, co;
        sincospi((double)m / (double)n, &s, &co);
        const double sg = (m & 1) ? -0.5 : 0.5;
        c = (n & 1) ? sg / s : sg * co / s;
      }
      d[m] = c;
      ux[m] = X[j0 + m] - X[j0];  // relative to the first point (derivative and signed area)
      uy[m] = X[P + j0 + m] - X[P + j0];
    }
    __syncthreads();
    double ax[kPer], ay[kPer];
    apply_d(d, ux, uy, n, ax, ay);  // X_alpha
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = threadIdx.x + k * kB;
      if (i < n) part += ux[i] * ay[k] - uy[i] * ax[k];
    }
    const double orient = block_sum(part, red) >= 0.0 ? 1.0 : -1.0;
    const double h = wave_mean_spacing(w + j0, n);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = threadIdx.x + k * kB;
      if (i < n) {
        const double jinv = 1.0 / sqrt(ax[k] * ax[k] + ay[k] * ay[k]);
        const double nx = orient * ay[k] * jinv;  // tangent turned clockwise: outward when counter-clockwise
        const double ny = -orient * ax[k] * jinv;
#pragma unroll
        for (int l = 0; l < 5; ++l) {
          const double dl = 0.5 * (double)(l - 2) * h;
          lx[l * n + i] = fma(dl, nx, X[j0 + i]);
          ly[l * n + i] = fma(dl, ny, X[P + j0 + i]);
        }
      }
    }
  }
}

}  // namespace

hipError_t launch_near_layers(const double* X, const double* w, const int32_t* off, int M, int P, double* layers,
                              void* stream) {
  if (M == 0 || P == 0) return hipSuccess;
  const int grid = M < 65535 ? M : 65535;
  hipLaunchKernelGGL(k_near_layers, dim3(grid), dim3(kB), 0, reinterpret_cast<hipStream_t>(stream), X, w, off, M, P,
                     layers);
  return hipGetLastError();
}

static size_t pad8_host(int j) { return (size_t)j + (size_t)(j >> 3); }

hipError_t launch_elastic(const double* X, const double* sigma, double kappa_b, const int32_t* off, int M, int P,
                          double* f, double* w, void* stream) {
  if (M == 0 || P == 0) return hipSuccess;
  const int grid = M < 65535 ? M : 65535;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // vesicles of up to 64, 128 or 256 points (the bound from the mean size) take one wavefront each
  const int64_t mean = ((int64_t)P + M - 1) / M;
  int cap = 0;
  if (mean <= 64) {
    cap = 64;
    hipLaunchKernelGGL(k_elastic_wave<1>, dim3(grid), dim3(64), sizeof(double) * (64 + 2 * pad8_host(128)), st, X,
                       sigma, kappa_b, off, M, P, f, w);
  } else if (mean <= 128) {
    cap = 128;
    hipLaunchKernelGGL(k_elastic_wave<2>, dim3(grid), dim3(64), sizeof(double) * (128 + 2 * pad8_host(256)), st, X,
                       sigma, kappa_b, off, M, P, f, w);
  } else if (mean <= 256) {
    cap = 256;
    hipLaunchKernelGGL(k_elastic_wave<4>, dim3(grid), dim3(64), sizeof(double) * (256 + 2 * pad8_host(512)), st, X,
                       sigma, kappa_b, off, M, P, f, w);
  }
  hipLaunchKernelGGL(k_elastic, dim3(grid), dim3(kB), 0, st, X, sigma, kappa_b, off, M, P, f, w, cap);
  return hipGetLastError();
}

}  // namespace vesnet
