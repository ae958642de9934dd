// Near-field interpolation on gfx950 (Section 3.3, Algorithm 4 interpolateInNearField).
//
// Each vesicle v carries n = 5 N_v nodes x_a (its five layers) with known velocities u_a.  The
// Gaussian radial basis interpolant  s(x) = sum_a phi(|x - x_a|) c_a,  phi(r) = exp(-r^2 / (eps h_v)^2),
// takes its coefficients from the symmetric positive definite system K c = u, K_ab = phi(|x_a - x_b|),
// which the paper solves by batched Cholesky factorisation.
//
// k_rbf_fit: one wavefront per vesicle factors K = L L^T in float64 by a left-looking blocked
// algorithm on 32 x 32 tiles.  The entries of K are recomputed from the node coordinates when a
// panel needs them, so only L is stored (in a per-wavefront slot of the tile workspace, lower tiles
// packed).  The tile products (panel updates T = K - sum L L^T, and L_IJ = T_IJ W^T) run on the FP64
// matrix cores.  Each diagonal tile is factored in registers and inverted, W = L_JJ^{-1}, by 16 x 16
// blocks; W replaces L_JJ in the slot (no later panel reads L_JJ) and stays in registers for the tiles
// below it.  The two right-hand sides ride along as two extra rows below the
// matrix (the bordered form [K; u^T]), so the same steps leave y = L^{-1} u in them; the back
// substitution L^T c = y then takes c_J = W_JJ^T (y_J - sum_{I>J} L_IJ^T c_I), block by block.  The
// rows are padded to a multiple of 32 with an identity block, which leaves the factor and the
// solution unchanged.
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
constexpr int kFW = 64;          // one wavefront per vesicle
constexpr int kMaxNodes = 1000;  // 5 x 200 points: the back substitution's 2 x 1024 + 64 doubles fit the LDS pool

__device__ __forceinline__ int clamp_i(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Packed lower tiles: tile (I, J), J <= I, at index I (I + 1) / 2 + J; the right-hand-side tile row
// I = nb follows the same formula.  The back substitution's two vectors follow the tiles.
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

// 32 x 32 tile from the slot into LDS (row stride kLd): every load is issued before any store.
__device__ __forceinline__ void stage_tile(double* __restrict__ dst, const double* __restrict__ src, int lane) {
  double v[kT * kT / kFW];
#pragma unroll
  for (int t = 0; t < kT * kT / kFW; ++t) v[t] = src[lane + kFW * t];
#pragma unroll
  for (int t = 0; t < kT * kT / kFW; ++t) {
    const int e = lane + kFW * t;
    dst[(e >> 5) * kLd + (e & 31)] = v[t];
  }
}

// Value of v in lane src (src the same in every lane) by two v_readlane.
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// The 32 x 32 tile products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64), as four 16 x 16 blocks
// (R, C).  Accumulator layout: lane l holds column 16 C + (l & 15) and rows 16 R + (l >> 4) + 4 q,
// q = 0..3, of the tile.  Operands: the A operand's element (i, k) and the B operand's element (k, j)
// sit in lane i + 16 k and lane j + 16 k.
typedef double double4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int acc_row(int lane, int R, int q) { return R * 16 + (lane >> 4) + 4 * q; }
__device__ __forceinline__ int acc_col(int lane, int C) { return C * 16 + (lane & 15); }

// This lane's entries (accumulator layout) of tile (I, J) of the bordered, padded matrix, with the
// node coordinates loaded before the Gaussians are formed.
__device__ __forceinline__ void entry_block(const NodeView& nv, int I, int J, int lane, double4v (&acc)[2][2]) {
  const int r0 = I * kT, c0 = J * kT;
  if (r0 >= nv.npad) {  // right-hand-side rows: u_x, u_y, then zeros
#pragma unroll
    for (int R = 0; R < 2; ++R)
#pragma unroll
      for (int C = 0; C < 2; ++C)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int qq = r0 + acc_row(lane, R, q) - nv.npad, col = c0 + acc_col(lane, C);
          acc[R][C][q] = (col >= nv.n || qq > 1) ? 0.0 : (qq == 0 ? nv.ux[col] : nv.uy[col]);
        }
    return;
  }
  double xr[2][4], yr[2][4], xc[2], yc[2];
#pragma unroll
  for (int R = 0; R < 2; ++R)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = min(r0 + acc_row(lane, R, q), nv.n - 1);
      xr[R][q] = nv.x[row];
      yr[R][q] = nv.y[row];
    }
#pragma unroll
  for (int C = 0; C < 2; ++C) {
    const int col = min(c0 + acc_col(lane, C), nv.n - 1);
    xc[C] = nv.x[col];
    yc[C] = nv.y[col];
  }
#pragma unroll
  for (int R = 0; R < 2; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = r0 + acc_row(lane, R, q), col = c0 + acc_col(lane, C);
        if (row >= nv.n || col >= nv.n) {
          acc[R][C][q] = row == col ? 1.0 : 0.0;
        } else {
          const double dx = xr[R][q] - xc[C], dy = yr[R][q] - yc[C];
          acc[R][C][q] = exp(-(dx * dx + dy * dy) * nv.inv_w2);
        }
      }
}

// acc += sign * Ar Bc^T over one 32-wide k-range (Ar, Bc: 32 x 32 tiles in LDS, row stride kLd).
__device__ __forceinline__ void tile_gemm(double4v (&acc)[2][2], const double* __restrict__ Ar,
                                          const double* __restrict__ Bc, int lane, double sign) {
  const int i = lane & 15, k = lane >> 4;
#pragma unroll
  for (int s = 0; s < kT / 4; ++s) {
    const double a0 = sign * Ar[i * kLd + 4 * s + k], a1 = sign * Ar[(16 + i) * kLd + 4 * s + k];
    const double b0 = Bc[i * kLd + 4 * s + k], b1 = Bc[(16 + i) * kLd + 4 * s + k];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__global__ __launch_bounds__(kFW, 2) void k_rbf_fit(const double* __restrict__ layers, const double* __restrict__ vel,
                                                 const double* __restrict__ w, const int32_t* __restrict__ off,
                                                 int M, int P, int nmax, double eps, double* __restrict__ coeffs,
                                                 double* __restrict__ tiles, size_t slot_doubles,
                                                 size_t slot_tile_doubles) {
  // LDS: A (row operand, then the tile being finished) and B (L_Jk, or W = L_JJ^{-1} re-staged from the
  // slot for the tiles below the diagonal); the back substitution reuses the pool for its two vectors
  // (2 npad <= 2048) and one exchange row.  Two tiles (17 KB) let eight wavefronts share a CU.
  __shared__ double pool[2 * kT * kLd];
  double* A = pool;
  double* B = pool + kT * kLd;

  const int lane = threadIdx.x;
  double* slot = tiles + (size_t)blockIdx.x * slot_doubles;
  (void)slot_tile_doubles;
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
      for (int a = lane; a < n; a += kFW) {
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

    // ---- factorisation, panel by panel; tile row nb holds the right-hand sides.  The workgroup is one
    // wavefront, so LDS needs only wave_sync; a tile stored to the slot is read back in later panels
    // only, after the panel's closing barrier has waited for the stores.
    double wreg[kT * kT / kFW];  // W = L_JJ^{-1} of the current panel, element lane + kFW t (row-major)
    for (int J = 0; J < nb; ++J) {
      for (int I = J; I <= nb; ++I) {
        double4v acc[2][2];
        entry_block(nv, I, J, lane, acc);
        // T = A - sum_{k < J} L(I, k) L(J, k)^T
        for (int k = 0; k < J; ++k) {
          wave_sync();  // A and B are free
          stage_tile(B, slot + tile_index(J, k) * (kT * kT), lane);
          if (I != J) stage_tile(A, slot + tile_index(I, k) * (kT * kT), lane);
          wave_sync();
          tile_gemm(acc, I != J ? A : B, B, lane, -1.0);
        }
        wave_sync();  // A is free
#pragma unroll
        for (int R = 0; R < 2; ++R)
#pragma unroll
          for (int C = 0; C < 2; ++C)
#pragma unroll
            for (int q = 0; q < 4; ++q) A[acc_row(lane, R, q) * kLd + acc_col(lane, C)] = acc[R][C][q];
        wave_sync();
        double* dst = slot + tile_index(I, J) * (kT * kT);
        if (I == J) {
          // Cholesky of the diagonal tile with lane i holding row i in registers (lanes 32..63
          // repeat lanes 0..31): column j takes s_i = T[i][j] - sum_{m<j} L[i][m] L[j][m], row j
          // read from lane j; L[j][j] = sqrt(s_j) and L[i][j] = s_i / L[j][j] below it.
          const int i = lane & (kT - 1);
          double row[kT];
#pragma unroll
          for (int c = 0; c < kT; ++c) row[c] = A[i * kLd + c];
          double rinv = 0.0;  // 1 / L[i][i]
#pragma unroll
          for (int j = 0; j < kT; ++j) {
            double sj = row[j];
#pragma unroll
            for (int m = 0; m < j; ++m) sj = fma(-row[m], lane_bcast(row[m], j), sj);
            const double s2 = lane_bcast(sj, j);
            double di = __builtin_amdgcn_rsq(s2);  // 1 / sqrt(s2), refined by two Newton steps
            di = fma(0.5 * di, fma(-s2 * di, di, 1.0), di);
            di = fma(0.5 * di, fma(-s2 * di, di, 1.0), di);
            const double d = s2 * di;
            row[j] = i > j ? sj * di : (i == j ? d : 0.0);
            if (i == j) rinv = di;
          }
          if (lane < kT) {
#pragma unroll
            for (int c = 0; c < kT; ++c) A[i * kLd + c] = row[c];
            A[i * kLd + kT] = rinv;  // the row's padding entry
          }
          wave_sync();
          // W = L^{-1} by 16 x 16 blocks.  W11 = L11^{-1} (lanes 0..15, column i) and W22 = L22^{-1} (lanes
          // 16..31, column i - 16) at once: W[r][i] = (delta_ri - sum_{m<r} L[r][m] W[m][i]) / L[r][r], with
          // L and 1 / L[r][r] read from LDS (the same address in each half).  Then W21 = -W22 (L21 W11) on
          // the matrix cores: the accumulator of L21 W11 is already in the B-operand layout of the second
          // product.  W goes to the slot in place of L_JJ and stays in registers for the tiles below.
          {
            const int o = lane & 16, ic = lane & 15;  // block offset, column within the block
            double wc[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              double t = ic == r ? 1.0 : 0.0;
#pragma unroll
              for (int m = 0; m < r; ++m) t = fma(-A[(o + r) * kLd + o + m], wc[m], t);
              wc[r] = t * A[(o + r) * kLd + kT];
            }
            if (lane < kT) {
#pragma unroll
              for (int r = 0; r < 16; ++r) B[(o + r) * kLd + o + ic] = wc[r];
              if (o != 0) {
#pragma unroll
                for (int r = 0; r < 16; ++r) B[r * kLd + 16 + ic] = 0.0;  // W12
              }
            }
          }
          wave_sync();
          {
            const int i16 = lane & 15, k4 = lane >> 4;
            double4v x = {0.0, 0.0, 0.0, 0.0}, w21 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)  // X = L21 W11
              x = __builtin_amdgcn_mfma_f64_16x16x4f64(A[(16 + i16) * kLd + 4 * s4 + k4], B[(4 * s4 + k4) * kLd + i16], x,
                                                       0, 0, 0);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)  // W21 = -W22 X
              w21 = __builtin_amdgcn_mfma_f64_16x16x4f64(-B[(16 + i16) * kLd + 16 + 4 * s4 + k4], x[s4], w21, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) B[(16 + 4 * q + k4) * kLd + i16] = w21[q];
          }
          wave_sync();
#pragma unroll
          for (int t = 0; t < kT * kT / kFW; ++t) {
            const int e = lane + kFW * t;
            wreg[t] = B[(e >> 5) * kLd + (e & 31)];
            dst[e] = wreg[t];
          }
        } else {
          // L_IJ = T W^T, W written into B from the registers
#pragma unroll
          for (int t = 0; t < kT * kT / kFW; ++t) {
            const int e = lane + kFW * t;
            B[(e >> 5) * kLd + (e & 31)] = wreg[t];
          }
          wave_sync();
          double4v out[2][2];
#pragma unroll
          for (int R = 0; R < 2; ++R)
#pragma unroll
            for (int C = 0; C < 2; ++C) out[R][C] = double4v{0.0, 0.0, 0.0, 0.0};
          tile_gemm(out, A, B, lane, 1.0);
#pragma unroll
          for (int R = 0; R < 2; ++R)
#pragma unroll
            for (int C = 0; C < 2; ++C)
#pragma unroll
              for (int q = 0; q < 4; ++q) dst[acc_row(lane, R, q) * kT + acc_col(lane, C)] = out[R][C][q];
        }
      }
      __syncthreads();  // the panel's tiles are stored before later panels read them
    }

    // ---- back substitution: c_J = W_JJ^T (y_J - sum_{I > J} L_IJ^T c_I); y in rows 0, 1 of tile row nb.
    // Lane (q, c) takes column c of each tile for right-hand side q, all 32 loads of a tile at once.
    // The tiles go in the order J = nb-1 .. 0, within J the L_IJ for I = J+1 .. nb-1 and then W_JJ.
    double* cv = pool;                    // [2][npad]
    double* zx = pool + 2 * nv.npad;      // [2][32]
    for (int e = lane; e < 2 * nv.npad; e += kFW) {
      const int q = e / nv.npad, a = e - q * nv.npad;
      cv[e] = slot[tile_index(nb, a >> 5) * (kT * kT) + q * kT + (a & 31)];
    }
    wave_sync();
    {
      const int q = lane >> 5, c = lane & 31;
      int I = nb - 1, J = nb - 1;  // I == J: the tile W_JJ
      double z = cv[q * nv.npad + J * kT + c];
      while (true) {
        double col[kT];
        {
          const double* Lt = slot + tile_index(I, J) * (kT * kT);
#pragma unroll
          for (int r = 0; r < kT; ++r) col[r] = Lt[r * kT + c];
        }
        if (I == J) {
          zx[q * kT + c] = z;
          wave_sync();
          double x = 0.0;
#pragma unroll
          for (int r = 0; r < kT; ++r) x = fma(col[r], zx[q * kT + r], x);
          cv[q * nv.npad + J * kT + c] = x;
          wave_sync();
          if (J == 0) break;
          --J;
          I = J + 1 < nb ? J + 1 : J;
          z = cv[q * nv.npad + J * kT + c];
        } else {
          const double* cI = cv + q * nv.npad + I * kT;
#pragma unroll
          for (int r = 0; r < kT; ++r) z = fma(-col[r], cI[r], z);
          I = I + 1 < nb ? I + 1 : J;
        }
      }
    }
    for (int a = lane; a < n; a += kFW) {
      cx[a] = cv[a];
      cy[a] = cv[nv.npad + a];
    }
    __syncthreads();  // the slot and LDS are reused by the next vesicle
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

static size_t rbf_slot_tile_doubles(int nmax) {
  const int nb = (5 * nmax + kT - 1) / kT;
  return (size_t)nb * (nb + 3) / 2 * (kT * kT);
}

size_t rbf_slot_doubles(int nmax) {
  const int nb = (5 * nmax + kT - 1) / kT;
  return rbf_slot_tile_doubles(nmax) + (size_t)2 * nb * kT;
}

hipError_t launch_rbf_fit(const double* layers, const double* vel, const double* w, const int32_t* off, int M, int P,
                          int nmax, double eps, double* coeffs, double* tiles, int slots, void* stream) {
  if (M == 0 || P == 0) return hipSuccess;
  if (5 * nmax > kMaxNodes || slots < 1) return hipErrorInvalidValue;
  const int grid = M < slots ? M : slots;
  hipLaunchKernelGGL(k_rbf_fit, dim3(grid), dim3(kFW), 0, reinterpret_cast<hipStream_t>(stream), layers, vel, w, off,
                     M, P, nmax, eps, coeffs, tiles, rbf_slot_doubles(nmax), rbf_slot_tile_doubles(nmax));
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
