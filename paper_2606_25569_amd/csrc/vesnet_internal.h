// Internal interfaces between the host API (vesnet_api.hip) and the kernels
// (vesnet_kernels.hip).  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vesnet {

enum Prec { P64 = 0, P32C = 1, P32N = 2 };

// Orders the LDS accesses of one wavefront around this point (a workgroup of one wavefront needs no
// s_barrier: its LDS instructions execute in issue order).  Global memory is not ordered by it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Mean arclength spacing h_v = sum_j w_j / n of the n weights w[0..n-1], formed by one
// whole wavefront (all 64 lanes call it with the same arguments) in a fixed order, so
// that every kernel that needs h_v gets the same bits.
__device__ inline double wave_mean_spacing(const double* __restrict__ w, int n) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += w[j];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  return s / (double)n;
}

// ---- float64 reciprocal and logarithm without division (used by the float64 pair loops and the trees)

// 1 / x for finite x != 0 whose reciprocal is a normal number: the hardware estimate r0 (relative error
// measured below 5e-8 on gfx950) refined by one third-order step, r0 (1 + e + e^2) with e = 1 - x r0 (the
// exact reciprocal is r0 / (1 - e)): three FMAs leave a truncation of order e^3 < 1e-22 and about one
// rounding, within an ulp or so of the correctly rounded quotient, as two Newton steps (four FMAs) do.
__device__ __forceinline__ double recip(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// Natural log of a finite q > 0, in about 20 FP64 operations: q = m 2^e with m in [1/sqrt 2, sqrt 2),
// ln m = 2 atanh(s) = 2 sum_k s^(2k+1) / (2k+1), s = (m - 1) / (m + 1), |s| <= 0.1716; the terms
// after s^21 are below 3e-17 of ln m.  ln 2 is split into a 32-bit high part (exact products with e)
// and a low part.  Against 40-digit references the series with an exact quotient stays within 2 ulp;
// the refined reciprocal adds at most about one more.
__device__ __forceinline__ double log_pos(double q) {
  constexpr double kLn2Hi = 6.93147180369123816490e-01;
  constexpr double kLn2Lo = 1.90821492927058770002e-10;
  int e;
  double m = frexp(q, &e);
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    --e;
  }
  const double s = (m - 1.0) * recip(m + 1.0);
  const double s2 = s * s;
  double pol = 1.0 / 21.0;
  pol = fma(pol, s2, 1.0 / 19.0);
  pol = fma(pol, s2, 1.0 / 17.0);
  pol = fma(pol, s2, 1.0 / 15.0);
  pol = fma(pol, s2, 1.0 / 13.0);
  pol = fma(pol, s2, 1.0 / 11.0);
  pol = fma(pol, s2, 1.0 / 9.0);
  pol = fma(pol, s2, 1.0 / 7.0);
  pol = fma(pol, s2, 1.0 / 5.0);
  pol = fma(pol, s2, 1.0 / 3.0);
  pol = fma(pol, s2, 1.0);
  return fma((double)e, kLn2Hi, fma((double)e, kLn2Lo, 2.0 * s * pol));
}

// Table of the reduced log below, N = 2^k entries: entry i (mantissa interval [1 + i/N, 1 + (i+1)/N)) holds
// 2a, with a an approximation of 1 / (1 + (i + 0.5) / N) to 1/(16 N), and -ln 2a (from log_pos).
template <int N>
__device__ __forceinline__ double2 log_tab_entry_n(int i) {
  const double c = 1.0 + ((double)i + 0.5) / N;
  const double a2 = rint(8.0 * N / c) / (4.0 * N);
  return make_double2(a2, -log_pos(a2));
}

// Natural log of a finite q > 0 with an N-entry table: q = mant 2^e, mant in [1/2, 1); r = mant (2a) - 1
// (exact product, one rounding), |r| <= 1/(2Nc) + c/(16N) (c in [1, 2), to first order), ln mant =
// -ln 2a + log1p(r), log1p by its series; ln 2 in a high and a low part as in log_pos.  The series stops
// where the next term is below 5e-18: through r^7 for N = 64 (|r| < 0.0089), through r^5 for N = 512
// (|r| < 0.0012).  Both forms are accurate in absolute terms (near q = 1 the result is a difference of
// terms of order ln 2, and the table entry alone carries up to about 5e-17).  The 512-entry form adds
// e ln 2 with one FMA and ln 2 rounded to a double, an extra absolute error of at most |e| 2.3e-17 (a
// quarter of an ulp of ln q at |e| = 20).  About 18 (N = 64) or 15 (N = 512) operations, no division.
template <int N>
__device__ __forceinline__ double log_reduced_n(double q, const double2* __restrict__ tab) {
  static_assert(N == 64 || N == 512, "series lengths are set for 64 and 512 entries");
  constexpr int kShift = N == 64 ? 14 : 11;  // the top log2(N) mantissa bits end at bit 19 of the high word
  constexpr double kLn2Hi = 6.93147180369123816490e-01;
  constexpr double kLn2Lo = 1.90821492927058770002e-10;
  int e;
  const double mant = frexp(q, &e);
  const int i = (__double2hiint(mant) >> kShift) & (N - 1);  // in range for every input
  const double2 t = tab[i];
  const double r = fma(mant, t.x, -1.0);
  double pol;
  if constexpr (N == 64) {
    pol = 1.0 / 7.0;
    pol = fma(pol, r, -1.0 / 6.0);
    pol = fma(pol, r, 1.0 / 5.0);
  } else {
    pol = 1.0 / 5.0;
  }
  pol = fma(pol, r, -1.0 / 4.0);
  pol = fma(pol, r, 1.0 / 3.0);
  pol = fma(pol, r, -0.5);
  pol = fma(pol, r, 1.0);
  const double ed = (double)e;
  if constexpr (N == 64) return fma(ed, kLn2Hi, fma(ed, kLn2Lo, fma(r, pol, t.y)));
  return fma(ed, 0.69314718055994530942, fma(r, pol, t.y));
}

// The 64-entry form (one entry per lane of a wavefront), used by the direct float64 kernel and the trees.
constexpr int kLogTab = 64;
__device__ __forceinline__ double2 log_tab_entry(int i) { return log_tab_entry_n<kLogTab>(i); }
__device__ __forceinline__ double log_reduced(double q, const double2* __restrict__ tab) {
  return log_reduced_n<kLogTab>(q, tab);
}

// Device views of a prepared workspace region.
struct PreparedView {
  int2* vrange;    // [M]   clamped point range (j0, j1) of each vesicle
  int32_t* vid;    // [P]   vesicle id of each point
  double4* vtab;   // [M]   (c_x, c_y, B_x, B_y): reference point and net weighted vector
  double* hlen;    // [M]   mean arclength spacing sum_j w_j / N_v
  void* rec;       // [P]   streamed records: float4 (P32C, P32N) or double4 (P64)
  double2* f64;    // [P]   forward P32C only: w_j f_j in float64 (the symmetric form's corrections)
  double2* vaux;   // [M]   forward P32C only: (sum_j |w_j f_j|_1, max_j |y_j - c_v|^2) per vesicle
};

// Device views of the symmetric form's region (after the prepared region).
struct SymmetricView {
  int4* cyc;                 // [P/16 + M + 1] cycles: (first point, count <= 16, vesicle, 0)
  int32_t* meta;             // [64] plan values: [0] number of cycles, [1] fixed-point exponent S, [2] number of
                             // blocks (one suspension) or of units (batched; then [4..12] the XCD queues and
                             // [16..23] their counters)
  double2* fcyc;             // [P/16 + M + 1] float64 net force w f of each cycle
  unsigned long long* acc;   // [2][P] fixed-point sums (two's complement int64 at 2^-S); float64 form:
                             // [2][2][P], the high words then the low words at 2^-(S + 40)
};

// Device views of the batched symmetric form's plan (after the symmetric region).
struct SymBatchView {
  int4* stab;       // [S]   per suspension: (first cycle, end cycle, blocks, fixed-point exponent)
  int32_t* ustart;  // [S+1] first unit of each suspension
  int32_t* pstart;  // [S+1] first point of each suspension
  int2* vr;         // [S]   vesicle range of each suspension, clamped, disjoint and non-decreasing
};

// Device views of the batched work plan.
struct PlanView {
  int32_t* psz;         // [S]   points per suspension
  int32_t* nitems;      // [S]   work items per suspension
  int32_t* order;       // [S]   suspensions, largest first
  int32_t* item_start;  // [S+1] first item of each suspension in that order
  int32_t* counter;     // [1]   next item to hand out
};

hipError_t launch_prepare(int prec, const double* pts, const double* vec, const double* wts, const int32_t* off,
                          int M, int P, const PreparedView& pv, void* stream);
hipError_t launch_forward(int prec, int T, int B, bool lds, bool mf, int splits, const double* tg, int P, int M,
                          const PreparedView& pv, double scale, double* out, double* partial, void* stream);
// Symmetric form (float32-compensated, targets = sources): sizes of its tables and the launch.
int sym_cycles_per_block(int T);
int64_t sym_max_cycles(int P, int M);
int64_t sym_max_blocks(int P, int M, int T);
int64_t sym_units(int64_t nb);
// whether the unit count of the symmetric form at T targets per thread fits one launch (2^31 - 1)
bool sym_fits(int P, int M, int T);
hipError_t launch_forward_symmetric(int T, int P, int M, const PreparedView& pv, const SymmetricView& sv,
                                    double scale, double* out, void* stream);
// The float64 symmetric form (T = 1 or 2; sv.acc holds 4P words: the high words of both components, then
// the low words).
hipError_t launch_forward_symmetric64(int T, int P, int M, const PreparedView& pv, const SymmetricView& sv,
                                      double scale, double* out, void* stream);
// Batched symmetric form (float32-compensated, targets = sources, S independent suspensions): a bound
// of its unit count, the workgroups of its persistent kernel one compute unit holds, and the launch
// (plan, cycle forces, persistent kernel on `grid` workgroups, conversion with each suspension's mu).
int64_t symb_max_units(int P, int M, int S, int T);
int symb_units_per_cu(int T);
hipError_t launch_batched_symmetric(int T, int grid, int P, int M, const PreparedView& pv, const SymmetricView& sv,
                                    const SymBatchView& bv, const int32_t* sus_off, const int32_t* off, int S,
                                    const double* mu, double* out, void* stream);
// a[e] += b[e] for e < n (float64)
hipError_t launch_add_f64(double* a, const double* b, int64_t n, void* stream);
// Its adjoint for targets = sources: pvF prepared from (points, f, w), pvG from (points, dL/du, no
// weights); vsum is a [2][P] float64 scratch; grad_points is required, grad_f and grad_w may be null.
hipError_t launch_backward_symmetric(int T, int P, int M, const PreparedView& pvF, const PreparedView& pvG,
                                     const SymmetricView& sv, double* vsum, const double* f, const double* w,
                                     double scale, double* grad_points, double* grad_f, double* grad_w,
                                     void* stream);
// The same in float64 (T = 1 or 2; pvF and pvG prepared in float64 with forces).
hipError_t launch_backward_symmetric64(int T, int P, int M, const PreparedView& pvF, const PreparedView& pvG,
                                       const SymmetricView& sv, double* vsum, const double* f, const double* w,
                                       double scale, double* grad_points, double* grad_f, double* grad_w,
                                       void* stream);
hipError_t launch_forward_near(int prec, int T, bool lds, int splits, const double* tg, int P, int M,
                               const PreparedView& pv, double scale, double* out, double* partial, int32_t* count,
                               int32_t* pairs, int32_t capacity, void* stream);
hipError_t launch_elastic(const double* X, const double* sigma, double kappa_b, const int32_t* off, int M, int P,
                          double* f, double* w, void* stream);
hipError_t launch_near_layers(const double* X, const double* w, const int32_t* off, int M, int P, double* layers,
                              void* stream);
// Gaussian RBF fit of every vesicle's five layers: the tile workspace holds `slots` regions of
// rbf_slot_doubles(nmax) doubles, one per concurrently running workgroup.
size_t rbf_slot_doubles(int nmax);
hipError_t launch_rbf_fit(const double* layers, const double* vel, const double* w, const int32_t* off, int M, int P,
                          int nmax, double eps, double* coeffs, double* tiles, int slots, void* stream);
hipError_t launch_rbf_eval_near(const double* layers, const double* coeffs, const double* w, const int32_t* off,
                                int M, int P, double eps, const double* targets, int n_targets,
                                const int32_t* pairs, const int32_t* count, int capacity, double* out, void* stream);
// Treecode far field (targets = sources): workspace size and the whole build + evaluation.
size_t treecode_workspace_bytes(int P, int depth, int p);
hipError_t launch_treecode(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                           double scale, int p, int depth, double* out, void* ws, void* stream);
// Fast multipole far field on the same tree: workspace size and the whole build + evaluation.
size_t fmm_workspace_bytes(int P, int depth, int p);
hipError_t launch_fmm(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                      double scale, int p, int depth, double* out, void* ws, void* stream);
// Sets a device int32 to zero with a kernel (so that callers may capture it in a graph).
hipError_t launch_zero_count(int32_t* count, void* stream);
// The same with near-field masking of Algorithm 4 and the near-pair list.
size_t fmm_near_workspace_bytes(int P, int M, int depth, int p);
hipError_t launch_fmm_nearmasked(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                                 double scale, int p, int depth, double* out, int32_t* pairs, int capacity,
                                 int32_t* count, void* ws, void* stream);
hipError_t launch_plan(const int32_t* sus_off, int S, int M, const PreparedView& pv, int tile, const PlanView& pl,
                       void* stream);
hipError_t launch_batched(int prec, int T, int B, bool lds, int grid, const double* tg, int P, int M,
                          const PreparedView& pv, const int32_t* sus_off, const double* mu, int S, const PlanView& pl,
                          double* out, void* stream);
hipError_t launch_backward(int prec, int T, int splits, const double* tg, const double* src, const double* f,
                           const double* w, const double* gout, int P, int M, const PreparedView& pvS,
                           const PreparedView& pvT, double scale, double* grad_t, double* grad_s, double* grad_f,
                           double* grad_w, double* part_t, double* part_s, void* stream);

}  // namespace vesnet
