// Near-field interpolation on gfx950 (Section 3.3, Algorithm 4 interpolateInNearField).
//
// Each vesicle v carries n = 5 N_v nodes x_a (its five layers) with known velocities u_a.  The
// Gaussian radial basis interpolant  s(x) = sum_a phi(|x - x_a|) c_a,  phi(r) = exp(-r^2 / (eps h_v)^2),
// takes its coefficients from the symmetric positive definite system K c = u, K_ab = phi(|x_a - x_b|),
// which the paper solves by batched Cholesky factorisation.
//
// k_rbf_fit: one workgroup per vesicle factors K = L L^T in float64 by a left-looking blocked
// algorithm on 32 x 32 tiles.  The entries of K are recomputed from the node coordinates when a
// panel needs them, so only L is stored (in a per-workgroup slot of the tile workspace, lower tiles
// packed).  The two right-hand sides ride along as two extra rows below the matrix (the bordered
// form [K; u^T]): the same panel updates and triangular solves that produce L's rows produce
// y = L^{-1} u in them.  A back substitution L^T c = y follows.  The rows are padded to a multiple
// of 32 with an identity block, which leaves the factor and the solution unchanged.
//
// k_rbf_eval_near: one wavefront per near (target, vesicle) pair sums phi c over the vesicle's nodes
// and adds the result into the target's velocity.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vesnet_internal.h"

namespace vesnet {

namespace {

constexpr int kT = 32;           // tile edge
constexpr int kLd = kT + 1;      // LDS row stride in doubles (conflict-free column reads)
constexpr int kCT = 4;           // row tiles per panel chunk
constexpr int kCR = kT * kCT;    // rows per panel chunk
constexpr int kFB = 256;         // threads of the fit kernel (4 wavefronts, one per chunk tile)
constexpr int kMaxNodes = 1280;  // 5 x 256 points
constexpr int kMaxPad = kMaxNodes;

__device__ __forceinline__ int clamp_i(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Packed lower tiles: tile (I, J), J <= I, at index I (I + 1) / 2 + J; the right-hand-side tile row
// I = nb follows the same formula.
__device__ __forceinline__ size_t tile_index(int I, int J) { return (size_t)I * (I + 1) / 2 + J; }

struct NodeView {
  const double* x;  // node coordinates of this vesicle
  const double* y;
  const double* ux;  // node values (right-hand sides)
  const double* uy;
  int n;             // nodes
  int npad;          // nodes rounded up to a multiple of kT
  double inv_w2;     // 1 / (eps h)^2
};

// Entry (row, col) of the bordered, padded matrix [K (+) I; u^T], col < npad, row < npad + kT.
__device__ __forceinline__ double bordered_entry(const NodeView& nv, int row, int col) {
  if (row >= nv.npad) {
    const int q = row - nv.npad;
    if (col >= nv.n || q > 1) return 0.0;
    return q == 0 ? nv.ux[col] : nv.uy[col];
  }
  if (row >= nv.n || col >= nv.n) return row == col ? 1.0 : 0.0;
  const double dx = nv.x[row] - nv.x[col];
  const double dy = nv.y[row] - nv.y[col];
  return exp(-(dx * dx + dy * dy) * nv.inv_w2);
}

__global__ __launch_bounds__(kFB, 2) void k_rbf_fit(const double* __restrict__ layers, const double* __restrict__ vel,
                                                 const double* __restrict__ w, const int32_t* __restrict__ off,
                                                 int M, int P, int nmax, double eps, double* __restrict__ coeffs,
                                                 double* __restrict__ tiles, size_t slot_doubles) {
  __shared__ double A[kCR * kLd];   // panel rows of L (GEMM operand), then the chunk being finished
  __shared__ double B[kT * kLd];    // diagonal tile row of L (GEMM operand)
  __shared__ double Ljj[kT * kLd];  // factored diagonal tile of the current panel
  __shared__ double dinv[kT];       // 1 / L_jj[c][c]
  __shared__ double cv[2 * kMaxPad];
  __shared__ double red[4 * 64];

  const int tid = threadIdx.x;
  const int cg = tid & 7;   // 4 columns: 4 cg .. 4 cg + 3
  const int rg = tid >> 3;  // 4 rows:    4 rg .. 4 rg + 3 of the chunk
  double* slot = tiles + (size_t)blockIdx.x * slot_doubles;
  const size_t P5 = (size_t)5 * P;

  for (int v = blockIdx.x; v < M; v += gridDim.x) {
    const int j0 = clamp_i(off[v], 0, P);
    const int j1 = max(j0, clamp_i(off[v + 1], 0, P));
    const int npts = j1 - j0;
    if (npts == 0) continue;
    const int n = 5 * npts;
    double* cx = coeffs + (size_t)5 * j0;
    double* cy = coeffs + P5 + (size_t)5 * j0;
    if (npts > nmax) {
      for (int a = tid; a < n; a += kFB) {
        cx[a] = NAN;
        cy[a] = NAN;
      }
      continue;
    }
    const double h = wave_mean_spacing(w + j0, npts);
    NodeView nv;
    nv.x = layers + (size_t)5 * j0;
    nv.y = layers + P5 + (size_t)5 * j0;
    nv.ux = vel + (size_t)5 * j0;
    nv.uy = vel + P5 + (size_t)5 * j0;
    nv.n = n;
    const int nb = (n + kT - 1) / kT;
    nv.npad = nb * kT;
    nv.inv_w2 = 1.0 / ((eps * h) * (eps * h));

    // ---- factorisation, panel by panel
    for (int J = 0; J < nb; ++J) {
      for (int I0 = J; I0 <= nb; I0 += kCT) {
        const int ntile = min(kCT, nb + 1 - I0);
        const bool active = rg * 4 < ntile * kT;  // whole wavefronts drop out together
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = active ? bordered_entry(nv, I0 * kT + rg * 4 + i, J * kT + cg * 4 + j) : 0.0;
        // T = A - sum_{k < J} L(rows, k) L(J, k)^T
        for (int k = 0; k < J; ++k) {
          __syncthreads();  // A and B are free
          for (int e = tid; e < ntile * kT * kT; e += kFB) {
            const int r = e >> 5, c = e & 31;
            A[r * kLd + c] = slot[tile_index(I0 + (r >> 5), k) * (kT * kT) + (r & 31) * kT + c];
          }
          for (int e = tid; e < kT * kT; e += kFB) B[(e >> 5) * kLd + (e & 31)] = slot[tile_index(J, k) * (kT * kT) + e];
          __syncthreads();
          if (active) {
#pragma unroll 4
            for (int m = 0; m < kT; ++m) {
              double a[4], b[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) a[i] = A[(rg * 4 + i) * kLd + m];
#pragma unroll
              for (int j = 0; j < 4; ++j) b[j] = B[(cg * 4 + j) * kLd + m];
#pragma unroll
              for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(-a[i], b[j], acc[i][j]);
            }
          }
        }
        __syncthreads();  // A is free: it now holds the chunk
        if (active) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) A[(rg * 4 + i) * kLd + cg * 4 + j] = acc[i][j];
        }
        __syncthreads();
        if (I0 == J) {
          // unblocked Cholesky of the diagonal tile (chunk rows 0..31), in place.  Step c updates the
          // trailing lower triangle with the unscaled column c and the pivot A_cc (one barrier per
          // step); the columns are scaled by 1 / sqrt(pivot) once all steps are done.
          for (int c = 0; c < kT; ++c) {
            const double rp = 1.0 / A[c * kLd + c];
            for (int e = tid; e < kT * kT; e += kFB) {
              const int r = e >> 5, s2 = e & 31;
              if (s2 > c && r >= s2) A[r * kLd + s2] = fma(-A[r * kLd + c] * rp, A[s2 * kLd + c], A[r * kLd + s2]);
            }
            __syncthreads();
          }
          if (tid < kT) dinv[tid] = 1.0 / sqrt(A[tid * kLd + tid]);
          __syncthreads();
          for (int e = tid; e < kT * kT; e += kFB) {
            const int r = e >> 5, s2 = e & 31;
            const double l = s2 > r ? 0.0 : A[r * kLd + s2] * dinv[s2];
            Ljj[r * kLd + s2] = l;
          }
          __syncthreads();
          for (int e = tid; e < kT * kT; e += kFB) A[(e >> 5) * kLd + (e & 31)] = Ljj[(e >> 5) * kLd + (e & 31)];
          __syncthreads();
        }
        // triangular solve of the chunk's other rows: x L_jj^T = t, one thread per row
        const int r = tid;
        const int rlo = I0 == J ? kT : 0;
        if (r >= rlo && r < ntile * kT) {
          double x[kT];
#pragma unroll
          for (int c = 0; c < kT; ++c) x[c] = A[r * kLd + c];
          // column by column: x_c is final once scaled, then removed from the later unknowns
          // (independent updates rather than one dependent chain per unknown)
#pragma unroll
          for (int c = 0; c < kT; ++c) {
            x[c] *= dinv[c];
#pragma unroll
            for (int m = c + 1; m < kT; ++m) x[m] = fma(-x[c], Ljj[m * kLd + c], x[m]);
          }
#pragma unroll
          for (int c = 0; c < kT; ++c) A[r * kLd + c] = x[c];
        }
        __syncthreads();
        for (int e = tid; e < ntile * kT * kT; e += kFB) {
          const int rr = e >> 5, c = e & 31;
          slot[tile_index(I0 + (rr >> 5), J) * (kT * kT) + (rr & 31) * kT + c] = A[rr * kLd + c];
        }
      }
    }
    __syncthreads();

    // ---- back substitution L^T c = y; y sits in rows 0, 1 of the tile row nb
    for (int e = tid; e < 2 * nv.npad; e += kFB) {
      const int q = e / nv.npad, a = e - q * nv.npad;
      cv[e] = slot[tile_index(nb, a >> 5) * (kT * kT) + q * kT + (a & 31)];
    }
    __syncthreads();
    const int comb = tid & 63;  // (right-hand side q, column c)
    const int q = comb >> 5, c = comb & 31;
    const int part = tid >> 6;
    for (int J = nb - 1; J >= 0; --J) {
      // z = y_J - sum_{I > J} L(I, J)^T c_I, rows split over the four wavefronts
      double s = 0.0;
      for (int I = J + 1 + part; I < nb; I += 4) {
        const double* Lt = slot + tile_index(I, J) * (kT * kT);
        const double* cI = cv + q * nv.npad + I * kT;
        for (int rr = 0; rr < kT; ++rr) s = fma(Lt[rr * kT + c], cI[rr], s);
      }
      red[part * 64 + comb] = s;
      for (int e = tid; e < kT * kT; e += kFB)
        Ljj[(e >> 5) * kLd + (e & 31)] = slot[tile_index(J, J) * (kT * kT) + e];
      __syncthreads();
      if (tid < 64) {
        double z = cv[q * nv.npad + J * kT + c] - (((red[comb] + red[64 + comb]) + red[128 + comb]) + red[192 + comb]);
        // L_jj^T x = z, last unknown first; lane (q, c) owns x_c
        double xc = 0.0;
        for (int k = kT - 1; k >= 0; --k) {
          const double xk = __shfl(z, q * 32 + k, 64) / Ljj[k * kLd + k];
          if (c == k) xc = xk;
          if (c < k) z = fma(-Ljj[k * kLd + c], xk, z);
        }
        cv[q * nv.npad + J * kT + c] = xc;
      }
      __syncthreads();
    }
    for (int a = tid; a < n; a += kFB) {
      cx[a] = cv[a];
      cy[a] = cv[nv.npad + a];
    }
    __syncthreads();  // cv and the slot are reused by the next vesicle
  }
}

constexpr int kEB = 256;  // threads of the evaluation kernel: 4 wavefronts, one pair each

__global__ __launch_bounds__(kEB) void k_rbf_eval_near(const double* __restrict__ layers,
                                                       const double* __restrict__ coeffs,
                                                       const double* __restrict__ w, const int32_t* __restrict__ off,
                                                       int M, int P, double eps, const double* __restrict__ tg,
                                                       int n_targets, const int32_t* __restrict__ pairs,
                                                       const int32_t* __restrict__ count, int capacity,
                                                       double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (kEB / 64);
  const int npairs = min(max(*count, 0), capacity);
  const size_t P5 = (size_t)5 * P;
  for (int k = blockIdx.x * (kEB / 64) + (threadIdx.x >> 6); k < npairs; k += waves) {
    const int i = pairs[2 * k];
    const int v = pairs[2 * k + 1];
    if (i < 0 || i >= n_targets || v < 0 || v >= M) continue;  // not a pair of this problem
    const int j0 = clamp_i(off[v], 0, P);
    const int j1 = max(j0, clamp_i(off[v + 1], 0, P));
    const int npts = j1 - j0;
    if (npts == 0) continue;
    const double h = wave_mean_spacing(w + j0, npts);
    const double inv_w2 = 1.0 / ((eps * h) * (eps * h));
    const double px = tg[i], py = tg[n_targets + i];
    const double* nx = layers + (size_t)5 * j0;
    const double* ny = layers + P5 + (size_t)5 * j0;
    const double* cx = coeffs + (size_t)5 * j0;
    const double* cy = coeffs + P5 + (size_t)5 * j0;
    double sx = 0.0, sy = 0.0;
    for (int a = lane; a < 5 * npts; a += 64) {
      const double dx = px - nx[a];
      const double dy = py - ny[a];
      const double g = exp(-(dx * dx + dy * dy) * inv_w2);
      sx = fma(g, cx[a], sx);
      sy = fma(g, cy[a], sy);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      sx += __shfl_xor(sx, m, 64);
      sy += __shfl_xor(sy, m, 64);
    }
    if (lane == 0) {
      atomicAdd(out + i, sx);
      atomicAdd(out + n_targets + i, sy);
    }
  }
}

}  // namespace

size_t rbf_slot_doubles(int nmax) {
  const int nb = (5 * nmax + kT - 1) / kT;
  return (size_t)nb * (nb + 3) / 2 * (kT * kT);
}

hipError_t launch_rbf_fit(const double* layers, const double* vel, const double* w, const int32_t* off, int M, int P,
                          int nmax, double eps, double* coeffs, double* tiles, int slots, void* stream) {
  if (M == 0 || P == 0) return hipSuccess;
  if (5 * nmax > kMaxNodes || slots < 1) return hipErrorInvalidValue;
  const int grid = M < slots ? M : slots;
  hipLaunchKernelGGL(k_rbf_fit, dim3(grid), dim3(kFB), 0, reinterpret_cast<hipStream_t>(stream), layers, vel, w, off,
                     M, P, nmax, eps, coeffs, tiles, rbf_slot_doubles(nmax));
  return hipGetLastError();
}

hipError_t launch_rbf_eval_near(const double* layers, const double* coeffs, const double* w, const int32_t* off,
                                int M, int P, double eps, const double* targets, int n_targets, const int32_t* pairs,
                                const int32_t* count, int capacity, double* out, void* stream) {
  if (capacity == 0 || M == 0 || P == 0 || n_targets == 0) return hipSuccess;
  const int need = (capacity + kEB / 64 - 1) / (kEB / 64);
  const int grid = need < 4096 ? need : 4096;
  hipLaunchKernelGGL(k_rbf_eval_near, dim3(grid), dim3(kEB), 0, reinterpret_cast<hipStream_t>(stream), layers, coeffs,
                     w, off, M, P, eps, targets, n_targets, pairs, count, capacity, out);
  return hipGetLastError();
}

}  // namespace vesnet
