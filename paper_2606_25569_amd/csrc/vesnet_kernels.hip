// Far-field Stokeslet kernels for gfx950 (wave64, vector ALUs).
//
// Operation: eq. (single_layer) with the 2D Stokeslet of eq. (Stokeslet), read as
// -ln|r| I + r r^T/|r|^2, discretised by the trapezoid rule (Section 2.2.1), summed
// over the vesicles other than the target's own (U_far of eq. (membrane_velocity),
// DirectSingleLayerIntegral of Algorithm 4), plus its reverse-mode derivative.
//
// Design (one gather kernel template serves the forward and both adjoint passes):
//  * one thread owns T "thread points" (targets in the forward); a wavefront owns 64*T
//    consecutive points, so a wave usually sits inside one vesicle;
//  * the loop runs over source vesicles, then over that vesicle's points; every lane reads
//    the same streamed record, so the compiler turns those reads into scalar loads that
//    land in SGPRs and feed the VALU directly (no LDS staging, no barriers);
//  * per (thread point, source vesicle) the pair sums run in float32 on rescaled local
//    coordinates r' = (x_i - c_v)/|x_i - c_v| - (y_j - c_v)/|x_i - c_v|, so log|r'| is
//    small for distant vesicles; the rr-term is scale free and the log term differs by
//    the exact constant ln(sigma) * sum_j F_j, added in float64 at the vesicle boundary
//    together with the float32 partial (compensated form);
//  * the own vesicle is dropped at the flush with a select, never inside the pair loop.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vesnet_internal.h"

namespace vesnet {

namespace {

constexpr double kLn2 = 0.69314718055994530942;
constexpr float kHalfLn2 = -0.34657359027997265471f;  // -(1/2) ln 2 : converts log2(q) to -ln|r|
constexpr int kTile = 1024;                             // records per LDS tile

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// Per-vesicle reference point, net vector and streamed records.
//   pts  [2][P] : positions of the streamed set,  vec [2][P] : vector carried by each point,
//   wts  [P] or null : weight multiplying vec (w for force densities, none for dL/du).
// Output per vesicle: range (j0, j1) clamped into [0, P], vtab = (c_x, c_y, B_x, B_y) with
// c = mean of the points and B = sum of weighted vectors (float64, fixed-order wave tree);
// per point: vid and the record: P32C (y - c, w vec) float32, P32N (y, w vec) float32,
// P64 (y, w vec) float64.  When f64 / vaux are given: w vec per point in float64, and per
// vesicle the sum of |w vec|_1 (fixed-order wave tree) and the largest squared distance of a
// point from c.
template <int PREC>
__global__ __launch_bounds__(64) void k_prepare(const double* __restrict__ pts, const double* __restrict__ vec,
                                                const double* __restrict__ wts, const int32_t* __restrict__ off_in,
                                                int M, int P, int2* __restrict__ vrange, int32_t* __restrict__ vid,
                                                double4* __restrict__ vtab, double* __restrict__ hlen,
                                                void* __restrict__ rec, double2* __restrict__ f64,
                                                double2* __restrict__ vaux) {
  const int lane = threadIdx.x;
  for (int v = blockIdx.x; v < M; v += gridDim.x) {
    const int j0 = clampi(off_in[v], 0, P);
    const int j1 = max(j0, clampi(off_in[v + 1], 0, P));
    double sx = 0.0, sy = 0.0, bx = 0.0, by = 0.0, sw = 0.0, sa = 0.0;
    for (int j = j0 + lane; j < j1; j += 64) {
      const double wj = wts ? wts[j] : 1.0;
      sx += pts[j];
      sy += pts[P + j];
      const double ex = wj * vec[j], ey = wj * vec[P + j];
      bx += ex;
      by += ey;
      sa += fabs(ex) + fabs(ey);
      sw += wj;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    bx = wave_sum(bx);
    by = wave_sum(by);
    sw = wave_sum(sw);
    if (vaux) sa = wave_sum(sa);
    const int n = j1 - j0;
    const double cx = n > 0 ? sx / n : 0.0;
    const double cy = n > 0 ? sy / n : 0.0;
    if (lane == 0) {
      vrange[v] = make_int2(j0, j1);
      vtab[v] = make_double4(cx, cy, bx, by);
      hlen[v] = n > 0 ? sw / n : 0.0;
    }
    double r2 = 0.0;
    for (int j = j0 + lane; j < j1; j += 64) {
      const double wj = wts ? wts[j] : 1.0;
      const double x = pts[j], y = pts[P + j];
      const double ex = wj * vec[j], ey = wj * vec[P + j];
      vid[j] = v;
      if (f64) f64[j] = make_double2(ex, ey);
      r2 = fmax(r2, (x - cx) * (x - cx) + (y - cy) * (y - cy));
      if constexpr (PREC == P32C) {
        static_cast<float4*>(rec)[j] = make_float4((float)(x - cx), (float)(y - cy), (float)ex, (float)ey);
      } else if constexpr (PREC == P32N) {
        static_cast<float4*>(rec)[j] = make_float4((float)x, (float)y, (float)ex, (float)ey);
      } else {
        static_cast<double4*>(rec)[j] = make_double4(x, y, ex, ey);
      }
    }
    if (vaux) {
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) r2 = fmax(r2, __shfl_xor(r2, m, 64));
      if (lane == 0) vaux[v] = make_double2(sa, r2);
    }
  }
}

template <int PREC> struct Real;
template <> struct Real<P64> { using T = double; using R = double4; };
template <> struct Real<P32C> { using T = float; using R = float4; };
template <> struct Real<P32N> { using T = float; using R = float4; };

// Near-field masking (FindNearFieldPoints of Algorithm 4; near-field rule of Section 2.2):
// vesicle v is near target i when min_j |x_i - y_j| <= h_v, the mean arclength spacing
// sum_j w_j / N_v of v.  Near vesicles are dropped from the sum and the pair (i, v) is
// appended to a list through an atomic counter (order unspecified; entries past the
// capacity are counted but not stored).
struct NearOut {
  const double* hlen;    // [M] h_v
  int32_t* count;        // [1] pairs found (zeroed before the launch)
  int32_t* pairs;        // [capacity][2] (target, vesicle)
  int32_t capacity;
};

// Accumulated results of one thread point.
template <int PREC>
struct Acc {
  double vx, vy;   // sum of G(r) b      (float64 except for the naive form)
  double gx, gy;   // sum of grad phi    (float64)
  float nvx, nvy;  // naive form: float32 totals
};

// The gather over source vesicles [v_begin, v_end) for the thread points
// [i_begin, i_end) of this workgroup.  Streamed records carry (position, b);
// the thread points carry position and (NEED_GRAD) a vector a.
//   NEED_V    : acc.v += sum_j G(r) b_j               (r = p_i - q_j)
//   NEED_GRAD : acc.g += sum_j grad_r [a_i^T G(r) b_j]
// Both without the 1/(4 pi mu) factor.
// LDS = false: records are read at wave-uniform addresses (scalar loads into SGPRs).
// LDS = true : the workgroup stages up to kTile consecutive records in LDS and every lane
//              reads them back with broadcast LDS loads into VGPRs.  The tile window only
//              moves forward through uniform control flow, so its barriers are block-wide.
// NEAR = true: also track min_j |r|^2 per (thread point, vesicle) and apply NearOut.
// MF = true (compensated forward only): the four accumulations of a pair move to the
//   matrix cores.  With r' = d' + n s_j (n = -sigma), sum_j t_j r'_j = d' sum_j t_j + n sum_j t_j s_j
//   and sum_j L_j F_j are products of a per-target value (t_j or L_j) with per-source
//   features (1, s_x, s_y) and (F_x, F_y): one v_mfma_f32_4x4x1f32 each, with the features
//   in the A operand (lane 4b+m of block b carries feature m) and the per-target value in
//   the B operand, so lane l's accumulator row m is feature m's sum for its own target.
template <int PREC, int T, int B, bool NEED_V, bool NEED_GRAD, bool LDS, bool NEAR = false, bool MF = false>
__device__ __forceinline__ void gather(int i_begin, int i_end, int v_begin, int v_end, const double* __restrict__ pts,
                                       const double* __restrict__ avec, const double* __restrict__ awts, int P,
                                       const int32_t* __restrict__ vid, const int2* __restrict__ vrange,
                                       const double4* __restrict__ vtab,
                                       const typename Real<PREC>::R* __restrict__ rec, Acc<PREC> (&acc)[T],
                                       int (&idx)[T], bool (&valid)[T], NearOut near = NearOut{}) {
  using real = typename Real<PREC>::T;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wbase = i_begin + wave * 64 * T;

  double px[T], py[T];
  real ax[T], ay[T];
  int myv[T];
#pragma unroll
  for (int k = 0; k < T; ++k) {
    idx[k] = wbase + k * 64 + lane;
    valid[k] = idx[k] < i_end;
    const int ii = valid[k] ? idx[k] : i_begin;
    px[k] = pts[ii];
    py[k] = pts[P + ii];
    myv[k] = valid[k] ? vid[ii] : -1;
    if constexpr (NEED_GRAD) {
      const double wa = awts ? awts[ii] : 1.0;
      ax[k] = (real)(wa * avec[ii]);
      ay[k] = (real)(wa * avec[P + ii]);
    } else {
      ax[k] = ay[k] = (real)0;
    }
    acc[k].vx = acc[k].vy = acc[k].gx = acc[k].gy = 0.0;
    acc[k].nvx = acc[k].nvy = 0.0f;
  }
  float pxf[T], pyf[T];
  if constexpr (PREC == P32N) {
#pragma unroll
    for (int k = 0; k < T; ++k) { pxf[k] = (float)px[k]; pyf[k] = (float)py[k]; }
  }

  using Rec = typename Real<PREC>::R;
  __shared__ Rec tile[LDS ? kTile : 1];
  int tile_lo = 0, tile_hi = 0;
  // float64: the logarithm's table (one entry per lane of the first wavefront)
  __shared__ double2 ltab[PREC == P64 ? kLogTab : 1];
  if constexpr (PREC == P64) {
    if (threadIdx.x < kLogTab) ltab[threadIdx.x] = log_tab_entry(threadIdx.x);
    __syncthreads();
  }

  for (int v = v_begin; v < v_end; ++v) {
    if constexpr (!LDS) {
      // Skip a vesicle that is the own vesicle of every live point of this wave.
      bool all_own = true;
#pragma unroll
      for (int k = 0; k < T; ++k) all_own = all_own && (!valid[k] || myv[k] == v);
      if (__all(all_own)) continue;
    }

    const int2 jr = vrange[v];
    const double4 vt = vtab[v];

    // Per (thread point, vesicle) set-up.
    real dx[T], dy[T], ns[T];
    float sig[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
      if constexpr (PREC == P32C) {
        const double ddx = px[k] - vt.x, ddy = py[k] - vt.y;
        const double D = ddx * ddx + ddy * ddy;
        const float Df = (float)D;
        const float s = (Df > 1e-30f && Df < 1e30f) ? __builtin_amdgcn_rsqf(Df) : 1.0f;
        sig[k] = s;
        dx[k] = (float)(ddx * (double)s);
        dy[k] = (float)(ddy * (double)s);
        ns[k] = -s;
      } else if constexpr (PREC == P32N) {
        dx[k] = pxf[k];
        dy[k] = pyf[k];
        ns[k] = -1.0f;
        sig[k] = 1.0f;
      } else {
        dx[k] = px[k];
        dy[k] = py[k];
        ns[k] = -1.0;
        sig[k] = 1.0f;
      }
    }

    real lx[T], ly[T], rvx[T], rvy[T], s1[T], gx[T], gy[T], hx[T], hy[T], qmin[T];
    floatx4 mt[T], ml[T];
#pragma unroll
    for (int k = 0; k < T; ++k) {
      lx[k] = ly[k] = rvx[k] = rvy[k] = s1[k] = gx[k] = gy[k] = hx[k] = hy[k] = (real)0;
      qmin[k] = (real)3.0e38f;
      mt[k] = floatx4{0.f, 0.f, 0.f, 0.f};
      ml[k] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    // Per-lane feature selectors of the A operand (lane 4b+m carries feature m), applied
    // with FMAs so that the selection stays branch-free.
    const int q4 = threadIdx.x & 3;
    const float sel0 = q4 == 0 ? 1.0f : 0.0f, sel1 = q4 == 1 ? 1.0f : 0.0f, sel2 = q4 == 2 ? 1.0f : 0.0f;

    auto pair = [&](const typename Real<PREC>::R& s) __attribute__((always_inline)) {
      float fa = 0.f, fb = 0.f;
      if constexpr (MF) {
        fa = fmaf(sel1, (float)s.x, fmaf(sel2, (float)s.y, sel0));  // (1, s_x, s_y, 0)
        fb = fmaf(sel0, (float)s.z, sel1 * (float)s.w);             // (F_x, F_y, 0, 0)
      }
#pragma unroll
      for (int k = 0; k < T; ++k) {
        real rx, ry;
        if constexpr (PREC == P64) {
          rx = dx[k] - s.x;
          ry = dy[k] - s.y;
        } else if constexpr (PREC == P32N) {
          rx = dx[k] - s.x;
          ry = dy[k] - s.y;
        } else {
          rx = fmaf(s.x, ns[k], dx[k]);
          ry = fmaf(s.y, ns[k], dy[k]);
        }
        const real q = ry * ry + rx * rx;
        if constexpr (NEAR) qmin[k] = q < qmin[k] ? q : qmin[k];
        real rho;
        if constexpr (PREC == P64) rho = recip(q);
        else rho = __builtin_amdgcn_rcpf(q);
        const real beta = ry * s.w + rx * s.z;  // r . b
        if constexpr (NEED_V) {
          real L;
          if constexpr (PREC == P64) L = log_reduced(q, ltab);
          else L = __builtin_amdgcn_logf(q);
          const real t = beta * rho;
          if constexpr (MF) {
            mt[k] = __builtin_amdgcn_mfma_f32_4x4x1f32(fa, (float)t, mt[k], 0, 0, 0);
            ml[k] = __builtin_amdgcn_mfma_f32_4x4x1f32(fb, (float)L, ml[k], 0, 0, 0);
          } else {
            lx[k] += L * s.z;
            ly[k] += L * s.w;
            rvx[k] += t * rx;
            rvy[k] += t * ry;
          }
        }
        if constexpr (NEED_GRAD) {
          const real alpha = ry * ay[k] + rx * ax[k];  // a . r
          const real gam = ay[k] * s.w + ax[k] * s.z;  // a . b
          const real abr = (alpha * beta) * rho;
          const real kap = (real)-2 * abr - gam;
          const real kr = kap * rho, ar = alpha * rho, br = beta * rho;
          s1[k] += br;
          gx[k] += s.z * ar;
          gy[k] += s.w * ar;
          hx[k] += rx * kr;
          hy[k] += ry * kr;
        }
      }
    };

    if constexpr (LDS) {
      int j = jr.x;
      while (j < jr.y) {
        if (j < tile_lo || j >= tile_hi) {
          tile_lo = j;
          tile_hi = min(j + kTile, P);
          __syncthreads();
          for (int e = threadIdx.x; e < tile_hi - tile_lo; e += B) tile[e] = rec[tile_lo + e];
          __syncthreads();
        }
        const int je = min(jr.y, tile_hi) - tile_lo;
        int jj = j - tile_lo;
        for (; jj + 4 <= je; jj += 4) {
          const Rec s0 = tile[jj], sA = tile[jj + 1], sB = tile[jj + 2], sC = tile[jj + 3];
          pair(s0);
          pair(sA);
          pair(sB);
          pair(sC);
        }
        for (; jj < je; ++jj) pair(tile[jj]);
        j = je + tile_lo;
      }
    } else {
      int j = jr.x;
      for (; j + 4 <= jr.y; j += 4) {
        const Rec s0 = rec[j], sA = rec[j + 1], sB = rec[j + 2], sC = rec[j + 3];
        pair(s0);
        pair(sA);
        pair(sB);
        pair(sC);
      }
      for (; j < jr.y; ++j) pair(rec[j]);
    }

    // Flush the per-vesicle partials (own vesicle dropped by a select).
#pragma unroll
    for (int k = 0; k < T; ++k) {
      bool keep = myv[k] != v;
      if constexpr (NEAR) {
        // squared distance test in the precision of the pair loop: on the rescaled
        // coordinates of the compensated form the threshold scales by sigma^2
        const double h = near.hlen[v];
        bool is_near;
        if constexpr (PREC == P32C) {
          const float th = (float)(h * (double)sig[k]);
          is_near = qmin[k] <= th * th;
        } else if constexpr (PREC == P32N) {
          const float th = (float)h;
          is_near = qmin[k] <= th * th;
        } else {
          is_near = qmin[k] <= h * h;
        }
        if (keep && valid[k] && is_near) {
          const int slot = atomicAdd(near.count, 1);
          if (slot < near.capacity) {
            near.pairs[2 * slot] = idx[k];
            near.pairs[2 * slot + 1] = v;
          }
        }
        keep = keep && !is_near;
      }
      if constexpr (MF) {
        // sum t r' = d' sum t + n sum t s  (n = ns = -sigma)
        lx[k] = ml[k][0];
        ly[k] = ml[k][1];
        rvx[k] = fmaf(ns[k], mt[k][1], dx[k] * mt[k][0]);
        rvy[k] = fmaf(ns[k], mt[k][2], dy[k] * mt[k][0]);
      }
      if constexpr (NEED_V) {
        if constexpr (PREC == P32C) {
          const float pvx = fmaf(kHalfLn2, lx[k], rvx[k]);
          const float pvy = fmaf(kHalfLn2, ly[k], rvy[k]);
          int e;
          const float m = frexpf(sig[k], &e);
          const double lnsig = ((double)e + (double)__builtin_amdgcn_logf(m)) * kLn2;
          const double cvx = fma(lnsig, vt.z, (double)pvx);
          const double cvy = fma(lnsig, vt.w, (double)pvy);
          acc[k].vx += keep ? cvx : 0.0;
          acc[k].vy += keep ? cvy : 0.0;
        } else if constexpr (PREC == P32N) {
          const float pvx = fmaf(kHalfLn2, lx[k], rvx[k]);
          const float pvy = fmaf(kHalfLn2, ly[k], rvy[k]);
          acc[k].nvx += keep ? pvx : 0.0f;
          acc[k].nvy += keep ? pvy : 0.0f;
        } else {
          const double pvx = fma(-0.5, lx[k], rvx[k]);
          const double pvy = fma(-0.5, ly[k], rvy[k]);
          acc[k].vx += keep ? pvx : 0.0;
          acc[k].vy += keep ? pvy : 0.0;
        }
      }
      if constexpr (NEED_GRAD) {
        const real pgx = ax[k] * s1[k] + gx[k] + hx[k];
        const real pgy = ay[k] * s1[k] + gy[k] + hy[k];
        if constexpr (PREC == P32C) {
          const double sg = (double)sig[k];
          acc[k].gx += keep ? sg * (double)pgx : 0.0;
          acc[k].gy += keep ? sg * (double)pgy : 0.0;
        } else {
          acc[k].gx += keep ? (double)pgx : 0.0;
          acc[k].gy += keep ? (double)pgy : 0.0;
        }
      }
    }
  }
  if constexpr (PREC == P32N) {
#pragma unroll
    for (int k = 0; k < T; ++k) { acc[k].vx = acc[k].nvx; acc[k].vy = acc[k].nvy; }
  }
}

// ----------------------------------------------------------------------------- forward

template <int PREC, int T, int B, bool LDS, bool MF>
__global__ __launch_bounds__(B) void k_forward(const double* __restrict__ tg, int P, int M,
                                               const int32_t* __restrict__ vid, const int2* __restrict__ vrange,
                                               const double4* __restrict__ vtab,
                                               const typename Real<PREC>::R* __restrict__ rec, double scale,
                                               int splits, double* __restrict__ out, double* __restrict__ partial) {
  const int tile = B * T;
  const int i_begin = blockIdx.x * tile;
  if (i_begin >= P) return;
  const int i_end = min(P, i_begin + tile);
  const int split = blockIdx.y;
  const int v_begin = (int)(((int64_t)M * split) / splits);
  const int v_end = (int)(((int64_t)M * (split + 1)) / splits);
  Acc<PREC> acc[T];
  int idx[T];
  bool valid[T];
  gather<PREC, T, B, true, false, LDS, false, MF>(i_begin, i_end, v_begin, v_end, tg, nullptr, nullptr, P, vid,
                                                  vrange, vtab, rec, acc, idx, valid);
#pragma unroll
  for (int k = 0; k < T; ++k) {
    if (!valid[k]) continue;
    if (splits == 1) {
      out[idx[k]] = scale * acc[k].vx;
      out[P + idx[k]] = scale * acc[k].vy;
    } else {
      partial[(size_t)(2 * split) * P + idx[k]] = acc[k].vx;
      partial[(size_t)(2 * split + 1) * P + idx[k]] = acc[k].vy;
    }
  }
}

// Forward sum with near-field vesicles masked out (see NearOut).
template <int PREC, int T, int B, bool LDS>
__global__ __launch_bounds__(B) void k_forward_near(const double* __restrict__ tg, int P, int M,
                                                    const int32_t* __restrict__ vid, const int2* __restrict__ vrange,
                                                    const double4* __restrict__ vtab,
                                                    const typename Real<PREC>::R* __restrict__ rec, double scale,
                                                    int splits, double* __restrict__ out, double* __restrict__ partial,
                                                    NearOut near) {
  const int tile = B * T;
  const int i_begin = blockIdx.x * tile;
  if (i_begin >= P) return;
  const int i_end = min(P, i_begin + tile);
  const int split = blockIdx.y;
  const int v_begin = (int)(((int64_t)M * split) / splits);
  const int v_end = (int)(((int64_t)M * (split + 1)) / splits);
  Acc<PREC> acc[T];
  int idx[T];
  bool valid[T];
  gather<PREC, T, B, true, false, LDS, true>(i_begin, i_end, v_begin, v_end, tg, nullptr, nullptr, P, vid, vrange,
                                             vtab, rec, acc, idx, valid, near);
#pragma unroll
  for (int k = 0; k < T; ++k) {
    if (!valid[k]) continue;
    if (splits == 1) {
      out[idx[k]] = scale * acc[k].vx;
      out[P + idx[k]] = scale * acc[k].vy;
    } else {
      partial[(size_t)(2 * split) * P + idx[k]] = acc[k].vx;
      partial[(size_t)(2 * split + 1) * P + idx[k]] = acc[k].vy;
    }
  }
}

__global__ void k_zero_i32(int32_t* __restrict__ p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0;
}

__global__ __launch_bounds__(256) void k_reduce_splits(const double* __restrict__ partial, int P, int splits,
                                                       double scale, double* __restrict__ out) {
  const int64_t n = 2 * (int64_t)P;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / P);
    const int64_t i = e - (int64_t)c * P;
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += partial[(size_t)(2 * k + c) * P + i];
    out[e] = scale * s;
  }
}

// ----------------------------------------------------------------------------- batched

// Plan, step 1: size of each suspension (points), work items per suspension.
__global__ void k_plan_sizes(const int32_t* __restrict__ sus_off, int S, int M, const int2* __restrict__ vrange,
                             int tile, int32_t* __restrict__ psz, int32_t* __restrict__ nitems) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
    const int vb = clampi(sus_off[s], 0, M);
    const int ve = max(vb, clampi(sus_off[s + 1], 0, M));
    int p = 0;
    if (ve > vb) p = max(0, vrange[ve - 1].y - vrange[vb].x);
    psz[s] = p;
    nitems[s] = (p + tile - 1) / tile;
  }
}

// Plan, step 2: order suspensions by size, largest first (ties by index).
__global__ void k_plan_rank(const int32_t* __restrict__ psz, int S, int32_t* __restrict__ order) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < S; s += gridDim.x * blockDim.x) {
    const int ps = psz[s];
    int r = 0;
    for (int t = 0; t < S; ++t) {
      const int pt = psz[t];
      r += (pt > ps) || (pt == ps && t < s);
    }
    order[r] = s;
  }
}

// Plan, step 3: item offsets in that order, and reset of the work counter.
__global__ __launch_bounds__(256) void k_plan_scan(const int32_t* __restrict__ order, const int32_t* __restrict__ nitems,
                                                   int S, int32_t* __restrict__ item_start, int32_t* __restrict__ counter) {
  __shared__ int32_t part[256];
  const int t = threadIdx.x;
  const int per = (S + 255) / 256;
  const int b = min(S, t * per), e = min(S, b + per);
  int32_t loc = 0;
  for (int r = b; r < e; ++r) loc += nitems[order[r]];
  part[t] = loc;
  __syncthreads();
  if (t == 0) {
    int32_t run = 0;
    for (int k = 0; k < 256; ++k) { const int32_t x = part[k]; part[k] = run; run += x; }
  }
  __syncthreads();
  int32_t run = part[t];
  for (int r = b; r < e; ++r) { item_start[r] = run; run += nitems[order[r]]; }
  if (t == 255) item_start[S] = run;
  if (t == 0) counter[0] = 0;
}

template <int PREC, int T, int B, bool LDS>
__global__ __launch_bounds__(B) void k_forward_batched(const double* __restrict__ tg, int P, int M,
                                                       const int32_t* __restrict__ vid,
                                                       const int2* __restrict__ vrange,
                                                       const double4* __restrict__ vtab,
                                                       const typename Real<PREC>::R* __restrict__ rec,
                                                       const int32_t* __restrict__ sus_off,
                                                       const double* __restrict__ mu, int S,
                                                       const int32_t* __restrict__ order,
                                                       const int32_t* __restrict__ item_start,
                                                       int32_t* __restrict__ counter, double* __restrict__ out) {
  __shared__ int32_t s_item;
  const int tile = B * T;
  const int total = item_start[S];
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int k = s_item;
    __syncthreads();
    if (k >= total) break;
    int lo = 0, hi = S;  // item_start[lo] <= k < item_start[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (item_start[mid] <= k) lo = mid; else hi = mid;
    }
    const int s = order[lo];
    const int blk = k - item_start[lo];
    const int vb = clampi(sus_off[s], 0, M);
    const int ve = max(vb, clampi(sus_off[s + 1], 0, M));
    if (ve <= vb) continue;
    const int pb = vrange[vb].x;
    const int pe = max(pb, vrange[ve - 1].y);
    const int i_begin = pb + blk * tile;
    if (i_begin >= pe) continue;
    const int i_end = min(pe, i_begin + tile);
    const double scale = 1.0 / (4.0 * 3.14159265358979323846 * mu[s]);
    Acc<PREC> acc[T];
    int idx[T];
    bool valid[T];
    gather<PREC, T, B, true, false, LDS>(i_begin, i_end, vb, ve, tg, nullptr, nullptr, P, vid, vrange, vtab, rec,
                                         acc, idx, valid);
#pragma unroll
    for (int q = 0; q < T; ++q) {
      if (!valid[q]) continue;
      out[idx[q]] = scale * acc[q].vx;
      out[P + idx[q]] = scale * acc[q].vy;
    }
  }
}

// ----------------------------------------------------------------------------- adjoint

// Pass over targets: grad_targets_i = c * sum_j grad_r phi(x_i - y_j; g_i, F_j).
// blockIdx.y selects a chunk of source vesicles; with several chunks the unscaled
// partial sums go to partial[(2*chunk + comp)*P + i] and a second kernel adds them.
template <int PREC, int T, int B>
__global__ __launch_bounds__(B) void k_bwd_targets(const double* __restrict__ tg, const double* __restrict__ gout,
                                                   int P, int M, const int32_t* __restrict__ vid,
                                                   const int2* __restrict__ vrange, const double4* __restrict__ vtab,
                                                   const typename Real<PREC>::R* __restrict__ rec, double scale,
                                                   int splits, double* __restrict__ grad_t,
                                                   double* __restrict__ partial) {
  const int tile = B * T;
  const int i_begin = blockIdx.x * tile;
  if (i_begin >= P) return;
  const int i_end = min(P, i_begin + tile);
  const int split = blockIdx.y;
  const int v_begin = (int)(((int64_t)M * split) / splits);
  const int v_end = (int)(((int64_t)M * (split + 1)) / splits);
  Acc<PREC> acc[T];
  int idx[T];
  bool valid[T];
  gather<PREC, T, B, false, true, true>(i_begin, i_end, v_begin, v_end, tg, gout, nullptr, P, vid, vrange, vtab,
                                         rec, acc, idx, valid);
#pragma unroll
  for (int k = 0; k < T; ++k) {
    if (!valid[k]) continue;
    if (splits == 1) {
      grad_t[idx[k]] = scale * acc[k].gx;
      grad_t[P + idx[k]] = scale * acc[k].gy;
    } else {
      partial[(size_t)(2 * split) * P + idx[k]] = acc[k].gx;
      partial[(size_t)(2 * split + 1) * P + idx[k]] = acc[k].gy;
    }
  }
}

// Epilogue of the pass over sources from the (unscaled) sums g (grad phi) and v (G g).
__device__ __forceinline__ void finish_source(int j, int P, double gx, double gy, double vx, double vy, double scale,
                                              const double* __restrict__ f, const double* __restrict__ w,
                                              double* __restrict__ grad_s, double* __restrict__ grad_f,
                                              double* __restrict__ grad_w) {
  if (grad_s) {
    grad_s[j] = scale * gx;
    grad_s[P + j] = scale * gy;
  }
  const double sx = scale * vx, sy = scale * vy;
  if (grad_f) {
    grad_f[j] = w[j] * sx;
    grad_f[P + j] = w[j] * sy;
  }
  if (grad_w) grad_w[j] = f[j] * sx + f[P + j] * sy;
}

// Pass over sources: with r~ = y_j - x_i (G even, grad phi odd and symmetric in its vectors)
//   grad_sources_j = c * sum_i grad phi(r~; F_j, g_i),  v_j = c * sum_i G(r~) g_i,
//   grad_f_j = w_j v_j,  grad_w_j = f_j . v_j.
// Chunked like the pass over targets, with four partial components (g_x, g_y, v_x, v_y).
template <int PREC, int T, int B>
__global__ __launch_bounds__(B) void k_bwd_sources(const double* __restrict__ src, const double* __restrict__ f,
                                                   const double* __restrict__ w, int P, int M,
                                                   const int32_t* __restrict__ vid, const int2* __restrict__ vrange,
                                                   const double4* __restrict__ vtab,
                                                   const typename Real<PREC>::R* __restrict__ rec, double scale,
                                                   int splits, double* __restrict__ grad_s,
                                                   double* __restrict__ grad_f, double* __restrict__ grad_w,
                                                   double* __restrict__ partial) {
  const int tile = B * T;
  const int i_begin = blockIdx.x * tile;
  if (i_begin >= P) return;
  const int i_end = min(P, i_begin + tile);
  const int split = blockIdx.y;
  const int v_begin = (int)(((int64_t)M * split) / splits);
  const int v_end = (int)(((int64_t)M * (split + 1)) / splits);
  Acc<PREC> acc[T];
  int idx[T];
  bool valid[T];
  gather<PREC, T, B, true, true, true>(i_begin, i_end, v_begin, v_end, src, f, w, P, vid, vrange, vtab, rec, acc,
                                        idx, valid);
#pragma unroll
  for (int k = 0; k < T; ++k) {
    if (!valid[k]) continue;
    const int j = idx[k];
    if (splits == 1) {
      finish_source(j, P, acc[k].gx, acc[k].gy, acc[k].vx, acc[k].vy, scale, f, w, grad_s, grad_f, grad_w);
    } else {
      partial[(size_t)(4 * split) * P + j] = acc[k].gx;
      partial[(size_t)(4 * split + 1) * P + j] = acc[k].gy;
      partial[(size_t)(4 * split + 2) * P + j] = acc[k].vx;
      partial[(size_t)(4 * split + 3) * P + j] = acc[k].vy;
    }
  }
}

__global__ __launch_bounds__(256) void k_reduce_sources(const double* __restrict__ partial, int P, int splits,
                                                        double scale, const double* __restrict__ f,
                                                        const double* __restrict__ w, double* __restrict__ grad_s,
                                                        double* __restrict__ grad_f, double* __restrict__ grad_w) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < P; j += gridDim.x * blockDim.x) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < splits; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] += partial[(size_t)(4 * k + c) * P + j];
    finish_source(j, P, a[0], a[1], a[2], a[3], scale, f, w, grad_s, grad_f, grad_w);
  }
}

}  // namespace

// ----------------------------------------------------------------------------- launchers

static inline hipStream_t S_(void* s) { return reinterpret_cast<hipStream_t>(s); }

hipError_t launch_prepare(int prec, const double* pts, const double* vec, const double* wts, const int32_t* off,
                          int M, int P, const PreparedView& pv, void* stream) {
  if (M == 0) return hipSuccess;
  const int grid = M < 65535 ? M : 65535;
  switch (prec) {
    case P64: hipLaunchKernelGGL(k_prepare<P64>, dim3(grid), dim3(64), 0, S_(stream), pts, vec, wts, off, M, P,
                                 pv.vrange, pv.vid, pv.vtab, pv.hlen, pv.rec, pv.f64, pv.vaux); break;
    case P32C: hipLaunchKernelGGL(k_prepare<P32C>, dim3(grid), dim3(64), 0, S_(stream), pts, vec, wts, off, M, P,
                                  pv.vrange, pv.vid, pv.vtab, pv.hlen, pv.rec, pv.f64, pv.vaux); break;
    case P32N: hipLaunchKernelGGL(k_prepare<P32N>, dim3(grid), dim3(64), 0, S_(stream), pts, vec, wts, off, M, P,
                                  pv.vrange, pv.vid, pv.vtab, pv.hlen, pv.rec, pv.f64, pv.vaux); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC, int T, int B, bool LDS, bool MF>
static void fwd_one(const double* tg, int P, int M, const PreparedView& pv, double scale, int splits, double* out,
                    double* partial, hipStream_t st) {
  const int tile = B * T;
  dim3 grid((P + tile - 1) / tile, splits);
  hipLaunchKernelGGL((k_forward<PREC, T, B, LDS, MF>), grid, dim3(B), 0, st, tg, P, M, pv.vid, pv.vrange, pv.vtab,
                     static_cast<const typename Real<PREC>::R*>(pv.rec), scale, splits, out, partial);
}

template <int PREC, bool MF>
static bool fwd_dispatch(int T, int B, bool lds, const double* tg, int P, int M, const PreparedView& pv, double scale,
                         int splits, double* out, double* partial, hipStream_t st) {
#define VESNET_FWD_CASE(TT, BB)                                                                   \
  if (T == TT && B == BB) {                                                                       \
    if (lds) fwd_one<PREC, TT, BB, true, MF>(tg, P, M, pv, scale, splits, out, partial, st);      \
    else fwd_one<PREC, TT, BB, false, MF>(tg, P, M, pv, scale, splits, out, partial, st);         \
    return true;                                                                                  \
  }
  VESNET_FWD_CASE(1, 64) VESNET_FWD_CASE(1, 128) VESNET_FWD_CASE(1, 256)
  VESNET_FWD_CASE(2, 64) VESNET_FWD_CASE(2, 128) VESNET_FWD_CASE(2, 256)
  VESNET_FWD_CASE(4, 64) VESNET_FWD_CASE(4, 128) VESNET_FWD_CASE(4, 256)
#undef VESNET_FWD_CASE
  return false;
}

hipError_t launch_forward(int prec, int T, int B, bool lds, bool mf, int splits, const double* tg, int P, int M,
                          const PreparedView& pv, double scale, double* out, double* partial, void* stream) {
  if (P == 0) return hipSuccess;
  hipStream_t st = S_(stream);
  bool ok = false;
  switch (prec) {
    case P64: ok = !mf && fwd_dispatch<P64, false>(T, B, lds, tg, P, M, pv, scale, splits, out, partial, st); break;
    case P32C:
      ok = mf ? fwd_dispatch<P32C, true>(T, B, lds, tg, P, M, pv, scale, splits, out, partial, st)
              : fwd_dispatch<P32C, false>(T, B, lds, tg, P, M, pv, scale, splits, out, partial, st);
      break;
    case P32N: ok = !mf && fwd_dispatch<P32N, false>(T, B, lds, tg, P, M, pv, scale, splits, out, partial, st); break;
    default: break;
  }
  if (!ok) return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  const int64_t n = 2 * (int64_t)P;
  const int grid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
  hipLaunchKernelGGL(k_reduce_splits, dim3(grid), dim3(256), 0, st, partial, P, splits, scale, out);
  return hipGetLastError();
}

template <int PREC, int T, bool LDS>
static void near_one(const double* tg, int P, int M, const PreparedView& pv, double scale, int splits, double* out,
                     double* partial, const NearOut& nr, hipStream_t st) {
  constexpr int B = 256;
  const int tile = B * T;
  dim3 grid((P + tile - 1) / tile, splits);
  hipLaunchKernelGGL((k_forward_near<PREC, T, B, LDS>), grid, dim3(B), 0, st, tg, P, M, pv.vid, pv.vrange, pv.vtab,
                     static_cast<const typename Real<PREC>::R*>(pv.rec), scale, splits, out, partial, nr);
}

hipError_t launch_forward_near(int prec, int T, bool lds, int splits, const double* tg, int P, int M,
                               const PreparedView& pv, double scale, double* out, double* partial, int32_t* count,
                               int32_t* pairs, int32_t capacity, void* stream) {
  hipStream_t st = S_(stream);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, count);
  if (P == 0) return hipGetLastError();
  const NearOut nr{pv.hlen, count, pairs, capacity};
#define VESNET_NEAR(PR)                                                                         \
  if (T == 1) { if (lds) near_one<PR, 1, true>(tg, P, M, pv, scale, splits, out, partial, nr, st);    \
                else near_one<PR, 1, false>(tg, P, M, pv, scale, splits, out, partial, nr, st); }   \
  else { if (lds) near_one<PR, 2, true>(tg, P, M, pv, scale, splits, out, partial, nr, st);          \
         else near_one<PR, 2, false>(tg, P, M, pv, scale, splits, out, partial, nr, st); }
  switch (prec) {
    case P64: VESNET_NEAR(P64) break;
    case P32C: VESNET_NEAR(P32C) break;
    case P32N: VESNET_NEAR(P32N) break;
    default: return hipErrorInvalidValue;
  }
#undef VESNET_NEAR
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  const int64_t n = 2 * (int64_t)P;
  const int grid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
  hipLaunchKernelGGL(k_reduce_splits, dim3(grid), dim3(256), 0, st, partial, P, splits, scale, out);
  return hipGetLastError();
}

hipError_t launch_plan(const int32_t* sus_off, int S, int M, const PreparedView& pv, int tile, const PlanView& pl,
                       void* stream) {
  hipStream_t st = S_(stream);
  const int g = (S + 255) / 256;
  hipLaunchKernelGGL(k_plan_sizes, dim3(g > 0 ? g : 1), dim3(256), 0, st, sus_off, S, M, pv.vrange, tile, pl.psz,
                     pl.nitems);
  hipLaunchKernelGGL(k_plan_rank, dim3(g > 0 ? g : 1), dim3(256), 0, st, pl.psz, S, pl.order);
  hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(256), 0, st, pl.order, pl.nitems, S, pl.item_start, pl.counter);
  return hipGetLastError();
}

template <int PREC, int T, int B, bool LDS>
static void bat_one(int grid, const double* tg, int P, int M, const PreparedView& pv, const int32_t* sus_off,
                    const double* mu, int S, const PlanView& pl, double* out, hipStream_t st) {
  hipLaunchKernelGGL((k_forward_batched<PREC, T, B, LDS>), dim3(grid), dim3(B), 0, st, tg, P, M, pv.vid, pv.vrange,
                     pv.vtab, static_cast<const typename Real<PREC>::R*>(pv.rec), sus_off, mu, S, pl.order,
                     pl.item_start, pl.counter, out);
}

template <int PREC>
static bool bat_dispatch(int T, int B, bool lds, int grid, const double* tg, int P, int M, const PreparedView& pv,
                         const int32_t* sus_off, const double* mu, int S, const PlanView& pl, double* out,
                         hipStream_t st) {
#define VESNET_BAT_CASE(TT, BB)                                                                    \
  if (T == TT && B == BB) {                                                                        \
    if (lds) bat_one<PREC, TT, BB, true>(grid, tg, P, M, pv, sus_off, mu, S, pl, out, st);         \
    else bat_one<PREC, TT, BB, false>(grid, tg, P, M, pv, sus_off, mu, S, pl, out, st);            \
    return true;                                                                                   \
  }
  VESNET_BAT_CASE(1, 64) VESNET_BAT_CASE(1, 128) VESNET_BAT_CASE(1, 256)
  VESNET_BAT_CASE(2, 64) VESNET_BAT_CASE(2, 128) VESNET_BAT_CASE(2, 256)
  VESNET_BAT_CASE(4, 64) VESNET_BAT_CASE(4, 128) VESNET_BAT_CASE(4, 256)
#undef VESNET_BAT_CASE
  return false;
}

hipError_t launch_batched(int prec, int T, int B, bool lds, int grid, const double* tg, int P, int M,
                          const PreparedView& pv, const int32_t* sus_off, const double* mu, int S, const PlanView& pl,
                          double* out, void* stream) {
  hipStream_t st = S_(stream);
  bool ok = false;
  switch (prec) {
    case P64: ok = bat_dispatch<P64>(T, B, lds, grid, tg, P, M, pv, sus_off, mu, S, pl, out, st); break;
    case P32C: ok = bat_dispatch<P32C>(T, B, lds, grid, tg, P, M, pv, sus_off, mu, S, pl, out, st); break;
    case P32N: ok = bat_dispatch<P32N>(T, B, lds, grid, tg, P, M, pv, sus_off, mu, S, pl, out, st); break;
    default: break;
  }
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int PREC, int T, int B>
static void bwd_one(const double* tg, const double* src, const double* f, const double* w, const double* gout, int P,
                    int M, int splits, const PreparedView& pvS, const PreparedView& pvT, double scale,
                    double* grad_t, double* grad_s, double* grad_f, double* grad_w, double* part_t, double* part_s,
                    hipStream_t st) {
  const int tile = B * T;
  const dim3 grid((P + tile - 1) / tile, splits);
  const int rgrid = (P + 255) / 256 < 16384 ? (P + 255) / 256 : 16384;
  if (grad_t) {
    hipLaunchKernelGGL((k_bwd_targets<PREC, T, B>), grid, dim3(B), 0, st, tg, gout, P, M, pvS.vid, pvS.vrange,
                       pvS.vtab, static_cast<const typename Real<PREC>::R*>(pvS.rec), scale, splits, grad_t, part_t);
    if (splits > 1) {
      const int g2 = (2 * P + 255) / 256 < 16384 ? (2 * P + 255) / 256 : 16384;
      hipLaunchKernelGGL(k_reduce_splits, dim3(g2), dim3(256), 0, st, part_t, P, splits, scale, grad_t);
    }
  }
  if (grad_s || grad_f || grad_w) {
    hipLaunchKernelGGL((k_bwd_sources<PREC, T, B>), grid, dim3(B), 0, st, src, f, w, P, M, pvT.vid, pvT.vrange,
                       pvT.vtab, static_cast<const typename Real<PREC>::R*>(pvT.rec), scale, splits, grad_s, grad_f,
                       grad_w, part_s);
    if (splits > 1)
      hipLaunchKernelGGL(k_reduce_sources, dim3(rgrid), dim3(256), 0, st, part_s, P, splits, scale, f, w, grad_s,
                         grad_f, grad_w);
  }
}

hipError_t launch_backward(int prec, int T, int splits, const double* tg, const double* src, const double* f,
                           const double* w, const double* gout, int P, int M, const PreparedView& pvS,
                           const PreparedView& pvT, double scale, double* grad_t, double* grad_s, double* grad_f,
                           double* grad_w, double* part_t, double* part_s, void* stream) {
  if (P == 0) return hipSuccess;
  hipStream_t st = S_(stream);
#define VESNET_BWD(PR, TT) \
  bwd_one<PR, TT, 256>(tg, src, f, w, gout, P, M, splits, pvS, pvT, scale, grad_t, grad_s, grad_f, grad_w, part_t, part_s, st)
  if (prec == P64) {
    if (T == 1) VESNET_BWD(P64, 1); else VESNET_BWD(P64, 2);
  } else if (prec == P32C) {
    if (T == 1) VESNET_BWD(P32C, 1); else VESNET_BWD(P32C, 2);
  } else {
    return hipErrorInvalidValue;
  }
#undef VESNET_BWD
  return hipGetLastError();
}

}  // namespace vesnet
