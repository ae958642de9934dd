// Symmetric far-field kernels for gfx950: each unordered cross-vesicle pair is evaluated once.
//
// The Stokeslet of eq. (Stokeslet), read as -ln|r| I + r r^T/|r|^2, is even in r, and the
// trapezoid sum of eq. (single_layer) (Section 2.2.1) taken at the discretisation points
// themselves uses every point as target and as source.  One evaluation of r, |r|^2, its
// logarithm and its reciprocal therefore serves both ordered pairs (i <- j and j <- i), which
// halves the transcendental instructions of the direct gather (26 issue slots per unordered pair,
// 13 per ordered pair, against 19.6).
// This file holds, on one schedule: the float32-compensated forward (k_sym_main) and its batched
// persistent form (k_symb_*), the float64 forward (k_sym64_main), and the adjoints of one point
// array in float32-compensated (k_sym_bwd) and float64 (k_sym64_bwd) form.  The description below is
// the float32-compensated forward's; the other kernels state where they differ.
//
// Work decomposition
//  * Points are cut into "cycles" of at most 16 consecutive points of one vesicle (a vesicle of
//    N points gives ceil(N/16) cycles); CB = 16 T consecutive cycles form a block.
//  * A unit is an unordered pair of blocks {bx, by}, by = bx + d (mod nb), d = 0 .. nb/2 (the
//    circulant schedule visits every unordered pair of blocks once; for even nb the pairs at
//    d = nb/2 are taken by bx < nb/2 only).  One workgroup of 256 threads (4 wavefronts, 16 rows
//    of 16 lanes) evaluates a unit: row r holds target cycles r, r + 16, ... of block bx (T of
//    them, one point per lane), and the source cycles of block by stream through LDS in chunks
//    of 8 cycles.  With T = 3 (the float32-compensated default: 768-point blocks, 112 VGPRs, 32 KB of
//    LDS) four units share a compute unit; with T = 2 (512-point blocks, 94 VGPRs, 27 KB) five.
//  * Each row is a ring: at step s lane p pairs its T targets with source (p + s) mod 16 of the
//    current source cycle, read from LDS (each cycle is stored twice so that the address is the
//    lane's base plus an immediate offset).  The source's column sum travels with it around the
//    ring, by a DPP row rotation folded into the add that closes each step.  After 16 steps two
//    lane swaps (v_permlane32_swap, v_permlane16_swap) add the four rows of a wavefront, the
//    column sums go to LDS, and after each chunk the workgroup adds its 4 wavefronts in a fixed
//    order.
//  * Own vesicle and the diagonal unit (d = 0): a (target cycle, source vesicle) pair is active
//    when the vesicles differ and, for d = 0, when the target's vesicle index is the smaller one,
//    so every unordered cross-vesicle pair is evaluated once.  Inactive targets sit at a far
//    point with zero force: their column contributions are exact zeros and their row partials
//    are dropped by a select.  Slots of a cycle past its count hold a copy of the cycle's first
//    point with zero force (exact zeros in the rows; their column sums are never read).
//
// Compensation (float32 pairs, float64 corrections)
//  * For a target of vesicle A and a source vesicle B the pair loop runs on the rescaled
//    difference r' = 2^-k (x_i - y_j) = 2^-k (xi_i + c_A - c_B) - 2^-k xi_j, with xi the float32
//    local coordinates about each vesicle's point mean c (c_A - c_B rounded once from float64) and
//    k = floor(e/2) for |c_A - c_B|^2 + R_A^2 + R_B^2 = m 2^e (R the largest |xi| of a vesicle):
//    |r'| is of order one for distant vesicles and bounded for overlapping hulls.  Scaling by a
//    power of two is exact, so ln|r|^2 = ln 2 (log2|r'|^2 + 2k) exactly, and the rr-term is
//    unchanged.  (Plain subtractions on unscaled coordinates with the scale applied to |r|^2 give
//    the same bits but one more instruction per pair, and measured 4% slower.)
//  * Row (target, segment of B in the block): float32 partial of -1/2 ln2 log2|r'|^2 F_j + rr-term,
//    then in float64  - k ln2 F_seg, F_seg the float64 net force of the segment (the sum of its
//    cycles' float64 net forces).
//  * Column (source j of B, from the targets of one wavefront): float32 partial of the same terms
//    with the targets' forces; the log correction - ln2 sum_cycles k F_cycle (float64) is the same
//    for every source of B and is formed once per (wavefront, B).
//    A distant force-free vesicle's nearly constant log therefore never enters a float32 sum.
//
// Accumulation across workgroups is deterministic: every row and column partial is added in
// float64, rounded to a 64-bit fixed-point integer at 2^-S (S from a bound on every partial sum,
// 520 sum_j |F_j|_1 < 2^(62 - S)) and added with 64-bit integer atomics, whose result does not
// depend on their order.  A last kernel converts the integers back and scales by 1/(4 pi mu).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "vesnet_internal.h"

namespace vesnet {

namespace {

constexpr int kRing = 16;                          // sources per ring cycle (one DPP row)
constexpr int kXcds = 8;                           // XCDs of the MI355X (workgroups are dealt to them in turn)
constexpr int kSymThreads = 256;                   // threads per unit (4 wavefronts, one per SIMD)
constexpr int kSymWaves = kSymThreads / 64;
constexpr int kRows = kSymThreads / kRing;         // rows of 16 lanes per unit
constexpr int kChunk = 8;                          // source cycles per LDS chunk
static_assert(kChunk * 2 * kRing <= kSymThreads, "one thread per staged record and per column sum of a chunk");
constexpr double kLn2d = 0.69314718055994530942;
constexpr double kPi = 3.14159265358979323846;
constexpr float kHalfLn2f = -0.34657359027997265471f;  // -(1/2) ln 2: log2|r|^2 -> -ln|r|
constexpr float kFar = 1152921504606846976.0f;         // 2^60: position of an inactive target
constexpr int kMaxShift = 60;                          // |k| bound of the power-of-two rescaling

__device__ __forceinline__ float bitsf(unsigned x) { return __builtin_bit_cast(float, x); }
__device__ __forceinline__ unsigned bitsu(float x) { return __builtin_bit_cast(unsigned, x); }

// x from the lane one position up in the same row of 16 lanes (lane p reads lane (p + 1) mod 16).
__device__ __forceinline__ float ring_next(float x) {
  return bitsf((unsigned)__builtin_amdgcn_update_dpp(0, (int)bitsu(x), 0x12F, 0xF, 0xF, true));
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

// Plan: the cycle table of every vesicle in point order, the number of blocks and the
// fixed-point exponent.  One workgroup of 1024 threads; everything in a fixed order.
__global__ __launch_bounds__(1024) void k_sym_plan(const int2* __restrict__ vrange, const double2* __restrict__ vaux,
                                                   int M, int cb, int ncyc_max, int4* __restrict__ cyc,
                                                   int32_t* __restrict__ meta) {
  __shared__ int32_t s_wsum[16];
  __shared__ double s_dsum[16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int run = 0;
  double fa = 0.0;
  for (int base = 0; base < M; base += 1024) {
    const int v = base + t;
    const int2 r = v < M ? vrange[v] : make_int2(0, 0);
    const int n = max(0, r.y - r.x);
    const int cnt = (n + kRing - 1) / kRing;
    if (v < M) fa += vaux[v].x;
    int x = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_wsum[wv] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      const int s = s_wsum[k];
      pre += k < wv ? s : 0;
      tot += s;
    }
    const int first = run + pre + x - cnt;
    for (int c = 0; c < cnt; ++c) {
      const int e = first + c;
      if (e < ncyc_max) cyc[e] = make_int4(r.x + kRing * c, min(kRing, n - kRing * c), v, 0);
    }
    run += tot;
    __syncthreads();
  }
  fa = wave_sum_d(fa);
  if (lane == 0) s_dsum[wv] = fa;
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;
    for (int k = 0; k < 16; ++k) tot += s_dsum[k];
    const int ncyc = min(run, ncyc_max);
    meta[0] = ncyc;
    // Every term of every partial sum is at most (|ln q|/2 + 1) |F|_1 <= 520 |F|_1 in magnitude
    // (log2|r'|^2 within the float32 range, |k| <= 60), so every partial sum of the fixed-point
    // integers stays below 2^62.
    const double bound = 520.0 * tot;
    int S = 0;
    if (bound > 0.0 && isfinite(bound)) {
      int e;
      frexp(bound, &e);  // bound < 2^e
      S = 62 - e;
    }
    meta[1] = S;
    meta[2] = (ncyc + cb - 1) / cb;
  }
}

// Float64 net force of every cycle (its points in order), and the zeroed fixed-point
// accumulator (grid-stride over all 2P entries).
__global__ __launch_bounds__(256) void k_sym_cycles(const int4* __restrict__ cyc, const int32_t* __restrict__ meta,
                                                    const double2* __restrict__ f64, int P,
                                                    double2* __restrict__ fcyc, unsigned long long* __restrict__ acc) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t first = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t e = first; e < 2 * (int64_t)P; e += stride) acc[e] = 0ull;
  const int ncyc = meta[0];
  for (int64_t c = first; c < ncyc; c += stride) {
    const int4 cy = cyc[c];
    double sx = 0.0, sy = 0.0;
    for (int m = 0; m < cy.y; ++m) {
      const double2 F = f64[cy.x + m];
      sx += F.x;
      sy += F.y;
    }
    fcyc[c] = make_double2(sx, sy);
  }
}

// The unit (row block bx, column block by) of this workgroup, false when it has none.  Units are the
// pairs {bx, bx + d mod nb}, d = 0 .. nb/2 (for even nb, d = nb/2 only for bx < nb/2), numbered row
// block by row block.  Workgroups are handed to the eight XCDs in turn (workgroup g to XCD g mod 8), so
// each XCD is given one contiguous range of that numbering: its concurrent units share a row block and
// a window of about nb/2 consecutive column blocks, which stays in the XCD's own L2.
// Unit number L (0 <= L < nb (nb + 1) / 2) of nb blocks, row block by row block, as the pair {bx, by}.
__device__ __forceinline__ void sym_unit_blocks(int nb, int L, int& bx, int& by) {
  const int h = nb >> 1;
  int d;
  if (L < h * (h + 1) || (nb & 1)) {
    bx = L / (h + 1);
    d = L - bx * (h + 1);
  } else {
    const int L2 = L - h * (h + 1);
    bx = h + L2 / h;
    d = L2 - (bx - h) * h;
  }
  by = bx + d;
  if (by >= nb) by -= nb;
}

__device__ __forceinline__ bool sym_unit(int nb, int& bx, int& by) {
  const int h = nb >> 1;
  const int units = (nb & 1) ? nb * (h + 1) : nb * h + h;
  const int g = blockIdx.x;
  if (g >= units) return false;
  const int q = units / kXcds, r = units % kXcds;
  const int x = g % kXcds;
  sym_unit_blocks(nb, x * q + min(x, r) + g / kXcds, bx, by);
  return true;
}

// One unit: target cycles [tc0, tc1) against source cycles [sc0, sc1) (diag: the two blocks are one),
// fixed-point exponent S (see the file header).  Called by the whole workgroup.
template <int T>
__device__ __forceinline__ void sym_eval_unit(int P, const double4* __restrict__ vtab,
                                              const double2* __restrict__ vaux, const float4* __restrict__ rec,
                                              const int4* __restrict__ cyc, const double2* __restrict__ fcyc, int S,
                                              int tc0, int tc1, int sc0, int sc1, bool diag,
                                              unsigned long long* __restrict__ acc) {
  constexpr int CB = kRows * T;  // cycles per block
  __shared__ float4 s_tx[CB][kRing];               // target records (local coordinates, w f)
  __shared__ double4 s_tc[CB];                     // (c_A, F_cycle) of each target cycle
  __shared__ double s_tr[CB];                      // R_A^2
  __shared__ int4 s_ti[CB];                        // (vesicle or -1, count, first point, 0)
  __shared__ float4 s_rec[2][kChunk][2 * kRing];   // source cycles, each stored twice
  __shared__ float s_col[2][kSymWaves][kChunk][2][kRing];
  __shared__ double2 s_E[2][kSymWaves][kChunk];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, p = lane & 15;
  const int row = tid >> 4;

  // Target block into LDS.
  for (int e = tid; e < CB * kRing; e += kSymThreads) {
    const int t = e / kRing, m = e % kRing;
    const int c = tc0 + t;
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    if (c < tc1) {
      const int4 cy = cyc[c];
      if (m < cy.y) r = rec[cy.x + m];
    }
    s_tx[t][m] = r;
  }
  for (int t = tid; t < CB; t += kSymThreads) {
    const int c = tc0 + t;
    if (c < tc1) {
      const int4 cy = cyc[c];
      const double4 vt = vtab[cy.z];
      const double2 F = fcyc[c];
      s_tc[t] = make_double4(vt.x, vt.y, F.x, F.y);
      s_tr[t] = vaux[cy.z].y;
      s_ti[t] = make_int4(cy.z, cy.y, cy.x, 0);
    } else {
      s_tc[t] = make_double4(0.0, 0.0, 0.0, 0.0);
      s_tr[t] = 0.0;
      s_ti[t] = make_int4(-1, 0, 0, 0);
    }
  }

  // State of the current source segment, per target slot k (target cycle k * 16 + row).
  float dx[T], dy[T], ns[T], fcx[T], fcy[T], fhx[T], fhy[T], lx[T], ly[T], rvx[T], rvy[T];
  double ax[T], ay[T];
  int kq[T];
  int actm = 0;
  double Ex = 0.0, Ey = 0.0, Fsx = 0.0, Fsy = 0.0;
#pragma unroll
  for (int k = 0; k < T; ++k) {
    dx[k] = dy[k] = ns[k] = fcx[k] = fcy[k] = fhx[k] = fhy[k] = 0.f;
    lx[k] = ly[k] = rvx[k] = rvy[k] = 0.f;
    ax[k] = ay[k] = 0.0;
    kq[k] = 0;
  }

  auto setup = [&](int B) {
    const double4 vb = vtab[B];
    const double rb2 = vaux[B].y;
    double ex = 0.0, ey = 0.0;
    actm = 0;
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const int t = k * kRows + row;
      const int4 ti = s_ti[t];
      const double4 tc = s_tc[t];
      const float4 tx = s_tx[t][p];
      const double Dx = tc.x - vb.x, Dy = tc.y - vb.y;
      const double D = fma(Dy, Dy, fma(Dx, Dx, s_tr[t] + rb2));
      int e;
      frexp(D, &e);
      const int kk = min(kMaxShift, max(-kMaxShift, e >> 1));
      const bool rowact = ti.x >= 0 && ti.x != B && (!diag || ti.x < B);
      const bool act = rowact && p < ti.y;
      actm |= act ? (1 << k) : 0;
      const float sc = ldexpf(1.0f, -kk);
      dx[k] = act ? fmaf(tx.x, sc, (float)ldexp(Dx, -kk)) : kFar;
      dy[k] = act ? fmaf(tx.y, sc, (float)ldexp(Dy, -kk)) : 0.f;
      ns[k] = -sc;
      fcx[k] = act ? tx.z : 0.f;
      fcy[k] = act ? tx.w : 0.f;
      fhx[k] = kHalfLn2f * fcx[k];
      fhy[k] = kHalfLn2f * fcy[k];
      kq[k] = kk;
      lx[k] = ly[k] = rvx[k] = rvy[k] = 0.f;
      ex += rowact ? (double)kk * tc.z : 0.0;
      ey += rowact ? (double)kk * tc.w : 0.0;
    }
    // the 16 lanes of a row hold the same value: add the four rows of the wavefront
    ex += __shfl_xor(ex, 16, 64);
    ey += __shfl_xor(ey, 16, 64);
    ex += __shfl_xor(ex, 32, 64);
    ey += __shfl_xor(ey, 32, 64);
    Ex = -kLn2d * ex;
    Ey = -kLn2d * ey;
    Fsx = Fsy = 0.0;
  };

  auto flush = [&]() {
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const float pvx = fmaf(kHalfLn2f, lx[k], rvx[k]);
      const float pvy = fmaf(kHalfLn2f, ly[k], rvy[k]);
      const double c = -kLn2d * (double)kq[k];
      const bool act = (actm >> k) & 1;
      ax[k] += act ? fma(c, Fsx, (double)pvx) : 0.0;
      ay[k] += act ? fma(c, Fsy, (double)pvy) : 0.0;
    }
  };

  // One ring cycle over the 16 sources of LDS cycle slot cc.
  auto ring = [&](int buf, int cc) {
    const float4* rb = &s_rec[buf][cc][p];
    float cax = 0.f, cay = 0.f;
#pragma unroll 1
    for (int s = 0; s < kRing; ++s) {
      const float4 sr = rb[s];
      float lcx = 0.f, lcy = 0.f;
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const float rx = fmaf(sr.x, ns[k], dx[k]);
        const float ry = fmaf(sr.y, ns[k], dy[k]);
        const float q = fmaf(ry, ry, rx * rx);
        const float L = __builtin_amdgcn_logf(q);
        const float rho = __builtin_amdgcn_rcpf(q);
        const float rxr = rx * rho, ryr = ry * rho;
        const float b = fmaf(ryr, sr.w, rxr * sr.z);       // (r . F_j)/q
        lx[k] = fmaf(L, sr.z, lx[k]);
        ly[k] = fmaf(L, sr.w, ly[k]);
        rvx[k] = fmaf(b, rx, rvx[k]);
        rvy[k] = fmaf(b, ry, rvy[k]);
        const float b2 = fmaf(ryr, fcy[k], rxr * fcx[k]);  // (r . F_i)/q
        if (k == 0) {
          lcx = L * fhx[k];
          lcy = L * fhy[k];
        } else {
          lcx = fmaf(L, fhx[k], lcx);
          lcy = fmaf(L, fhy[k], lcy);
        }
        lcx = fmaf(b2, rx, lcx);
        lcy = fmaf(b2, ry, lcy);
      }
      cax = ring_next(cax) + lcx;
      cay = ring_next(cay) + lcy;
    }
    // lane p now holds source (p + 15) mod 16 of its row; add the four rows: x sums end in lanes
    // 0-31, y sums in lanes 32-63, then every row of a half holds the half's total
    const auto h = __builtin_amdgcn_permlane32_swap(bitsu(cax), bitsu(cay), false, false);
    const float z = bitsf(h[0]) + bitsf(h[1]);
    const auto r16 = __builtin_amdgcn_permlane16_swap(bitsu(z), bitsu(z), false, false);
    const float tot = bitsf(r16[0]) + bitsf(r16[1]);
    if ((lane & 16) == 0) s_col[buf][wv][cc][lane >> 5][(p + kRing - 1) & (kRing - 1)] = tot;
  };

  // Records of source chunk g: slots 0..15 and again 16..31; slots past the cycle's count repeat
  // its first point with zero force.
  const int nchunks = (sc1 - sc0 + kChunk - 1) / kChunk;
  const bool stager = tid < kChunk * 2 * kRing;
  const int st_cc = tid >> 5, st_q = tid & 31, st_m = st_q & (kRing - 1);
  auto stage_load = [&](int g) {
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    const int c = sc0 + g * kChunk + st_cc;
    if (stager && c < sc1) {
      const int4 cy = cyc[c];
      r = rec[cy.x + (st_m < cy.y ? st_m : 0)];
      if (st_m >= cy.y) r.z = r.w = 0.f;
    }
    return r;
  };
  auto stage_store = [&](int buf, const float4& r) {
    if (stager) s_rec[buf][st_cc][st_q] = r;
  };

  // Column sums of chunk g: the wavefronts and their log corrections added in a fixed order,
  // then one fixed-point integer per (source, component).
  auto reduce = [&](int g, int buf) {
    if (tid >= kChunk * 2 * kRing) return;
    const int cc = tid >> 5, comp = (tid >> 4) & 1, m = tid & (kRing - 1);
    const int c = sc0 + g * kChunk + cc;
    if (c >= sc1) return;
    const int4 cy = cyc[c];
    if (m >= cy.y) return;
    double s = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < kSymWaves; ++w2) s += (double)s_col[buf][w2][cc][comp][m];
    double e = 0.0;
#pragma unroll
    for (int w2 = 0; w2 < kSymWaves; ++w2) {
      const double2 E = s_E[buf][w2][cc];
      e += comp ? E.y : E.x;
    }
    const long long X = (long long)rint(ldexp(s + e, S));
    atomicAdd(&acc[(size_t)comp * P + cy.x + m], (unsigned long long)X);
  };

  int curB = -1;
  stage_store(0, stage_load(0));
  __syncthreads();
  for (int g = 0; g < nchunks; ++g) {
    const int buf = g & 1;
    const float4 nxt = stage_load(g + 1);
    if (g > 0) reduce(g - 1, buf ^ 1);
    const int cbase = sc0 + g * kChunk;
    const int ncc = min(kChunk, sc1 - cbase);
    for (int cc = 0; cc < ncc; ++cc) {
      const int4 cy = cyc[cbase + cc];
      if (cy.z != curB) {
        if (curB >= 0) flush();
        setup(cy.z);
        curB = cy.z;
      }
      const double2 Fc = fcyc[cbase + cc];
      Fsx += Fc.x;
      Fsy += Fc.y;
      ring(buf, cc);
      if (lane == 0) s_E[buf][wv][cc] = make_double2(Ex, Ey);
    }
    stage_store(buf ^ 1, nxt);
    __syncthreads();
  }
  if (nchunks > 0) {
    reduce(nchunks - 1, (nchunks - 1) & 1);
    flush();
  }
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const int4 ti = s_ti[k * kRows + row];
    if (ti.x >= 0 && p < ti.y) {
      const int i = ti.z + p;
      atomicAdd(&acc[i], (unsigned long long)(long long)rint(ldexp(ax[k], S)));
      atomicAdd(&acc[(size_t)P + i], (unsigned long long)(long long)rint(ldexp(ay[k], S)));
    }
  }
}

// One unit {bx, by} per workgroup (see the file header).
template <int T>
__global__ __launch_bounds__(kSymThreads) void k_sym_main(
    int P, const double4* __restrict__ vtab, const double2* __restrict__ vaux, const float4* __restrict__ rec,
    const int4* __restrict__ cyc, const double2* __restrict__ fcyc, const int32_t* __restrict__ meta,
    unsigned long long* __restrict__ acc) {
  constexpr int CB = kRows * T;
  const int ncyc = meta[0];
  const int S = meta[1];
  const int nb = meta[2];
  if (nb <= 0) return;
  int bx, by;
  if (!sym_unit(nb, bx, by)) return;
  const int tc0 = bx * CB, sc0 = by * CB;
  sym_eval_unit<T>(P, vtab, vaux, rec, cyc, fcyc, S, tc0, min(ncyc, tc0 + CB), sc0, min(ncyc, sc0 + CB), bx == by,
                   acc);
}

// ------------------------------------------------------------------ float64 symmetric form
// The same schedule (cycles, blocks, circulant units, rings of 16 lanes) in float64 on global coordinates:
// float64 needs no compensation, so a segment's set-up only selects the target or a far point with zero
// force, and its rows are flushed without a log correction.  The logarithm is the table logarithm of the
// direct float64 kernel with a 512-entry table (two fewer series terms than its 64 entries), the reciprocal
// that kernel's refined hardware estimate; column sums travel around the ring
// by DPP moves of both halves of each double.  Sums leave the workgroup as two 64-bit fixed-point words:
// hi = rint(x 2^S) and lo = rint((x - hi 2^-S) 2^(S + kLoBits)) (the first difference is exact), each added
// by an integer atomic, so the result is again independent of the order of the atomics while the
// resolution is 2^-(S + kLoBits), far below float64 rounding of the sum.  |lo| <= 2^(kLoBits - 1), so up to
// 2^(62 - kLoBits + 1) partials per point stay exact.
constexpr int kLoBits = 40;
constexpr int kChunk64 = 4;                         // source cycles per LDS chunk
constexpr int kLogTab64 = 512;                     // entries of the float64 kernels' log table (8 KB of LDS)
constexpr double kFar64 = 3.2733906078961419e150;   // 2^500: position of an inactive target
static_assert(kChunk64 * 2 * kRing <= kSymThreads, "one thread per staged record and per column sum of a chunk");

// x from lane (p + 1) mod 16 of the same row (both halves of the double moved by DPP).
__device__ __forceinline__ double ring_next64(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x12F, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x12F, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ unsigned long long dlo(double x) { return __builtin_bit_cast(unsigned long long, x); }
__device__ __forceinline__ double dfrom(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Adds x to the two fixed-point words of one accumulator entry (hi at a, lo at a + 2P).
__device__ __forceinline__ void fixed_add2(unsigned long long* __restrict__ a, size_t two_p, double x, int S) {
  const double h = rint(ldexp(x, S));
  const double r = x - ldexp(h, -S);  // exact
  atomicAdd(a, (unsigned long long)(long long)h);
  atomicAdd(a + two_p, (unsigned long long)(long long)rint(ldexp(r, S + kLoBits)));
}

template <int T>
__global__ __launch_bounds__(kSymThreads) void k_sym64_main(
    int P, const double4* __restrict__ rec, const int4* __restrict__ cyc, const int32_t* __restrict__ meta,
    unsigned long long* __restrict__ acc) {
  constexpr int CB = kRows * T;
  __shared__ int4 s_ti[CB];                          // (vesicle or -1, count, first point, 0)
  __shared__ double4 s_rec[2][kChunk64][2 * kRing];  // source cycles (x, y, F_x, F_y), each stored twice
  __shared__ double s_col[2][kSymWaves][kChunk64][2][kRing];
  __shared__ double2 ltab[kLogTab64];

  const int ncyc = meta[0];
  const int S = meta[1];
  const int nb = meta[2];
  if (nb <= 0) return;
  int bx, by;
  if (!sym_unit(nb, bx, by)) return;
  const bool diag = bx == by;
  const int tc0 = bx * CB, tc1 = min(ncyc, tc0 + CB);
  const int sc0 = by * CB, sc1 = min(ncyc, sc0 + CB);
  const size_t two_p = 2 * (size_t)P;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, p = lane & 15;
  const int row = tid >> 4;
  for (int e = tid; e < kLogTab64; e += kSymThreads) ltab[e] = log_tab_entry_n<kLogTab64>(e);
  for (int t = tid; t < CB; t += kSymThreads) {
    const int c = tc0 + t;
    if (c < tc1) {
      const int4 cy = cyc[c];
      s_ti[t] = make_int4(cy.z, cy.y, cy.x, 0);
    } else {
      s_ti[t] = make_int4(-1, 0, 0, 0);
    }
  }
  __syncthreads();

  // this lane's targets (slot k: target cycle k * 16 + row, point p of it)
  double4 tr[T];
  int4 ti[T];
#pragma unroll
  for (int k = 0; k < T; ++k) {
    ti[k] = s_ti[k * kRows + row];
    tr[k] = ti[k].x >= 0 && p < ti[k].y ? rec[ti[k].z + p] : make_double4(0.0, 0.0, 0.0, 0.0);
  }
  double dx[T], dy[T], fcx[T], fcy[T], fhx[T], fhy[T], lx[T], ly[T], rvx[T], rvy[T], ax[T], ay[T];
  int actm = 0;
#pragma unroll
  for (int k = 0; k < T; ++k) {
    dx[k] = dy[k] = fcx[k] = fcy[k] = fhx[k] = fhy[k] = 0.0;
    lx[k] = ly[k] = rvx[k] = rvy[k] = ax[k] = ay[k] = 0.0;
  }

  auto setup = [&](int B) {
    actm = 0;
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const bool act = ti[k].x >= 0 && ti[k].x != B && (!diag || ti[k].x < B) && p < ti[k].y;
      actm |= act ? (1 << k) : 0;
      dx[k] = act ? tr[k].x : kFar64;
      dy[k] = act ? tr[k].y : 0.0;
      fcx[k] = act ? tr[k].z : 0.0;
      fcy[k] = act ? tr[k].w : 0.0;
      fhx[k] = -0.5 * fcx[k];
      fhy[k] = -0.5 * fcy[k];
      lx[k] = ly[k] = rvx[k] = rvy[k] = 0.0;
    }
  };

  auto flush = [&]() {
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const bool act = (actm >> k) & 1;
      ax[k] += act ? fma(-0.5, lx[k], rvx[k]) : 0.0;
      ay[k] += act ? fma(-0.5, ly[k], rvy[k]) : 0.0;
    }
  };

  auto ring = [&](int buf, int cc) {
    const double4* rb = &s_rec[buf][cc][p];
    double cax = 0.0, cay = 0.0;
#pragma unroll 1
    for (int s = 0; s < kRing; ++s) {
      const double4 sr = rb[s];
      double lcx = 0.0, lcy = 0.0;
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const double rx = dx[k] - sr.x;
        const double ry = dy[k] - sr.y;
        const double q = fma(ry, ry, rx * rx);
        const double L = log_reduced_n<kLogTab64>(q, ltab);
        const double rho = recip(q);
        const double rxr = rx * rho, ryr = ry * rho;
        const double b = fma(ryr, sr.w, rxr * sr.z);       // (r . F_j)/q
        lx[k] = fma(L, sr.z, lx[k]);
        ly[k] = fma(L, sr.w, ly[k]);
        rvx[k] = fma(b, rx, rvx[k]);
        rvy[k] = fma(b, ry, rvy[k]);
        const double b2 = fma(ryr, fcy[k], rxr * fcx[k]);  // (r . F_i)/q
        if (k == 0) {
          lcx = L * fhx[k];
          lcy = L * fhy[k];
        } else {
          lcx = fma(L, fhx[k], lcx);
          lcy = fma(L, fhy[k], lcy);
        }
        lcx = fma(b2, rx, lcx);
        lcy = fma(b2, ry, lcy);
      }
      cax = ring_next64(cax) + lcx;
      cay = ring_next64(cay) + lcy;
    }
    // lane p holds source (p + 15) mod 16 of its row; add the four rows: x sums end in lanes 0-31, y sums
    // in lanes 32-63 (both halves of each double swapped alike), then every row of a half holds the total
    const unsigned long long bx_ = dlo(cax), by_ = dlo(cay);
    const auto hl = __builtin_amdgcn_permlane32_swap((unsigned)bx_, (unsigned)by_, false, false);
    const auto hh = __builtin_amdgcn_permlane32_swap((unsigned)(bx_ >> 32), (unsigned)(by_ >> 32), false, false);
    const double z = dfrom(hl[0], hh[0]) + dfrom(hl[1], hh[1]);
    const unsigned long long bz = dlo(z);
    const auto gl = __builtin_amdgcn_permlane16_swap((unsigned)bz, (unsigned)bz, false, false);
    const auto gh = __builtin_amdgcn_permlane16_swap((unsigned)(bz >> 32), (unsigned)(bz >> 32), false, false);
    const double tot = dfrom(gl[0], gh[0]) + dfrom(gl[1], gh[1]);
    if ((lane & 16) == 0) s_col[buf][wv][cc][lane >> 5][(p + kRing - 1) & (kRing - 1)] = tot;
  };

  const int nchunks = (sc1 - sc0 + kChunk64 - 1) / kChunk64;
  const bool stager = tid < kChunk64 * 2 * kRing;
  const int st_cc = tid >> 5, st_q = tid & 31, st_m = st_q & (kRing - 1);
  auto stage_load = [&](int g) {
    double4 r = make_double4(0.0, 0.0, 0.0, 0.0);
    const int c = sc0 + g * kChunk64 + st_cc;
    if (stager && c < sc1) {
      const int4 cy = cyc[c];
      r = rec[cy.x + (st_m < cy.y ? st_m : 0)];
      if (st_m >= cy.y) r.z = r.w = 0.0;
    }
    return r;
  };
  auto stage_store = [&](int buf, const double4& r) {
    if (stager) s_rec[buf][st_cc][st_q] = r;
  };
  // column sums of chunk g: the four wavefronts added in a fixed order, then two fixed-point words
  auto reduce = [&](int g, int buf) {
    if (tid >= kChunk64 * 2 * kRing) return;
    const int cc = tid >> 5, comp = (tid >> 4) & 1, m = tid & (kRing - 1);
    const int c = sc0 + g * kChunk64 + cc;
    if (c >= sc1) return;
    const int4 cy = cyc[c];
    if (m >= cy.y) return;
    const double v = ((s_col[buf][0][cc][comp][m] + s_col[buf][1][cc][comp][m]) + s_col[buf][2][cc][comp][m]) +
                     s_col[buf][3][cc][comp][m];
    fixed_add2(&acc[(size_t)comp * P + cy.x + m], two_p, v, S);
  };

  int curB = -1;
  stage_store(0, stage_load(0));
  __syncthreads();
  for (int g = 0; g < nchunks; ++g) {
    const int buf = g & 1;
    const double4 nxt = stage_load(g + 1);
    if (g > 0) reduce(g - 1, buf ^ 1);
    const int cbase = sc0 + g * kChunk64;
    const int ncc = min(kChunk64, sc1 - cbase);
    for (int cc = 0; cc < ncc; ++cc) {
      const int4 cy = cyc[cbase + cc];
      if (cy.z != curB) {
        if (curB >= 0) flush();
        setup(cy.z);
        curB = cy.z;
      }
      ring(buf, cc);
    }
    stage_store(buf ^ 1, nxt);
    __syncthreads();
  }
  if (nchunks > 0) {
    reduce(nchunks - 1, (nchunks - 1) & 1);
    flush();
  }
#pragma unroll
  for (int k = 0; k < T; ++k) {
    if (ti[k].x >= 0 && p < ti[k].y) {
      const int i = ti[k].z + p;
      fixed_add2(&acc[i], two_p, ax[k], S);
      fixed_add2(&acc[(size_t)P + i], two_p, ay[k], S);
    }
  }
}

__global__ __launch_bounds__(256) void k_sym64_finish(const unsigned long long* __restrict__ acc,
                                                      const int32_t* __restrict__ meta, int P, double scale,
                                                      double* __restrict__ out) {
  const int S = meta[1];
  const int64_t n = 2 * (int64_t)P;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double hi = (double)(long long)acc[e];
    const double lo = (double)(long long)acc[n + e];
    out[e] = ldexp(fma(lo, ldexp(1.0, -kLoBits), hi) * scale, -S);
  }
}

// ------------------------------------------------------------------ batched symmetric form
// Many independent suspensions in one persistent launch.  Each suspension's cycles are contiguous (its
// vesicles in order), its blocks of CB cycles never reach into another suspension, and its units are the
// circulant pairs of its own blocks, so no pair across suspensions is formed.  The units of all
// suspensions are numbered suspension by suspension (row block by row block inside each), and that
// numbering is cut into eight contiguous ranges, one queue per XCD: a workgroup takes units from its own
// XCD's queue by an atomic counter and, once that queue is empty, from the next XCDs' in turn.
// Every unit does the same work (up to the last block of a suspension), so the order needs no sorting.

// Slots of the plan values in the symmetric region's meta array.
constexpr int kMetaUnits = 2;    // total number of units
constexpr int kMetaQueue = 4;    // [kXcds + 1] first unit of each XCD's queue
constexpr int kMetaCount = 16;   // [kXcds] next position in each queue
static_assert(kMetaCount + kXcds <= 64, "plan values fit the 256-byte meta slot");

__device__ __forceinline__ int wave_scan_incl(int x, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Plan: per suspension s, stab[s] = (first cycle, end cycle, blocks, fixed-point exponent), ustart[s] its
// first unit, pstart[s] its first point (ustart[S], pstart[S]: totals); the cycle table; meta[0] the
// number of cycles, the XCD queues and their zeroed counters.  One workgroup of 1024 threads, in a fixed
// order; the exponent of a suspension is the one the single-suspension plan gives it.
// The suspensions' vesicle ranges are first clamped to [0, M] and made disjoint and non-decreasing
// (vr[s] = (v0, v1), v0 = max(offset s, every earlier end), v1 = max(offset s + 1, v0)): valid offsets are
// unchanged, and no input can make the cycles outrun their table.
__global__ __launch_bounds__(1024) void k_symb_plan(const int2* __restrict__ vrange, const double2* __restrict__ vaux,
                                                    const int32_t* __restrict__ sus_off, int M, int P, int nsus,
                                                    int cb, int ncyc_max, int4* __restrict__ cyc,
                                                    int4* __restrict__ stab, int32_t* __restrict__ ustart,
                                                    int32_t* __restrict__ pstart, int2* __restrict__ vr,
                                                    int32_t* __restrict__ meta) {
  __shared__ int s_wc[16], s_wu[16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // disjoint, non-decreasing vesicle ranges (a running maximum of the clamped ends)
  int pm = 0;
  for (int base = 0; base < nsus; base += 1024) {
    const int s = base + t;
    const int a = s < nsus ? min(max(sus_off[s], 0), M) : 0;
    const int b = s < nsus ? min(max(sus_off[s + 1], 0), M) : 0;
    int x = b;  // inclusive running maximum of the ends within the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x = max(x, y);
    }
    if (lane == 63) s_wc[wv] = x;
    __syncthreads();
    int pre = pm, tot = pm;
    for (int k = 0; k < 16; ++k) {
      pre = k < wv ? max(pre, s_wc[k]) : pre;
      tot = max(tot, s_wc[k]);
    }
    int ex = __shfl_up(x, 1, 64);  // the maximum over the earlier lanes of this wavefront
    ex = lane == 0 ? pre : max(pre, ex);
    if (s < nsus) {
      const int v0 = max(a, ex);
      vr[s] = make_int2(v0, max(b, v0));
    }
    pm = tot;
    __syncthreads();
  }
  __syncthreads();
  // cycles and the bound of the partial sums of each suspension, one wavefront per suspension
  for (int s = wv; s < nsus; s += 16) {
    const int2 rs = vr[s];
    const int v0 = rs.x, v1 = rs.y;
    int cnt = 0;
    double fs = 0.0;
    for (int v = v0 + lane; v < v1; v += 64) {
      const int2 r = vrange[v];
      cnt += (max(0, r.y - r.x) + kRing - 1) / kRing;
      fs += vaux[v].x;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) cnt += __shfl_xor(cnt, m, 64);
    fs = wave_sum_d(fs);
    if (lane == 0) {
      const double bound = 520.0 * fs;  // as in k_sym_plan
      int S = 0;
      if (bound > 0.0 && isfinite(bound)) {
        int e;
        frexp(bound, &e);
        S = 62 - e;
      }
      stab[s] = make_int4(cnt, 0, (cnt + cb - 1) / cb, S);
    }
  }
  __syncthreads();
  // exclusive scans over the suspensions: first cycle and first unit
  int runc = 0, runu = 0;
  for (int base = 0; base < nsus; base += 1024) {
    const int s = base + t;
    const int4 st = s < nsus ? stab[s] : make_int4(0, 0, 0, 0);
    const int nu = (int)((int64_t)st.z * (st.z + 1) / 2);
    const int xc = wave_scan_incl(st.x, lane), xu = wave_scan_incl(nu, lane);
    if (lane == 63) {
      s_wc[wv] = xc;
      s_wu[wv] = xu;
    }
    __syncthreads();
    int prec_ = 0, preu = 0, totc = 0, totu = 0;
    for (int k = 0; k < 16; ++k) {
      prec_ += k < wv ? s_wc[k] : 0;
      preu += k < wv ? s_wu[k] : 0;
      totc += s_wc[k];
      totu += s_wu[k];
    }
    if (s < nsus) {
      const int c0 = runc + prec_ + xc - st.x;
      stab[s] = make_int4(c0, c0 + st.x, st.z, st.w);
      ustart[s] = runu + preu + xu - nu;
      const int v0 = vr[s].x;
      pstart[s] = v0 < M ? vrange[v0].x : P;
    }
    runc += totc;
    runu += totu;
    __syncthreads();
  }
  if (t == 0) {
    ustart[nsus] = runu;
    pstart[nsus] = P;
    meta[0] = min(runc, ncyc_max);
    meta[kMetaUnits] = runu;
    const int q = runu / kXcds, r = runu % kXcds;
    for (int x = 0; x <= kXcds; ++x) meta[kMetaQueue + x] = x * q + min(x, r);
  }
  if (t < kXcds) meta[kMetaCount + t] = 0;
  __syncthreads();
  // the cycles of every vesicle, one wavefront per suspension
  for (int s = wv; s < nsus; s += 16) {
    const int2 rs = vr[s];
    const int v0 = rs.x, v1 = rs.y;
    int c = stab[s].x;
    for (int vb = v0; vb < v1; vb += 64) {
      const int v = vb + lane;
      const int2 r = v < v1 ? vrange[v] : make_int2(0, 0);
      const int n = max(0, r.y - r.x);
      const int cnt = (n + kRing - 1) / kRing;
      const int x = wave_scan_incl(cnt, lane);
      const int first = c + x - cnt;
      for (int k = 0; k < cnt; ++k)
        if (first + k < ncyc_max) cyc[first + k] = make_int4(r.x + kRing * k, min(kRing, n - kRing * k), v, 0);
      c += __shfl(x, 63, 64);
    }
  }
}

// Persistent batched kernel: units from the XCD queues until all are empty (see above).
template <int T>
__global__ __launch_bounds__(kSymThreads) __attribute__((amdgpu_waves_per_eu(T == 2 ? 5 : T == 3 ? 4 : 1))) void k_symb_main(
    int P, const double4* __restrict__ vtab, const double2* __restrict__ vaux, const float4* __restrict__ rec,
    const int4* __restrict__ cyc, const double2* __restrict__ fcyc, const int4* __restrict__ stab,
    const int32_t* __restrict__ ustart, int nsus, int32_t* __restrict__ meta, unsigned long long* __restrict__ acc) {
  constexpr int CB = kRows * T;
  __shared__ int s_job[2];
  const int xcd = blockIdx.x % kXcds;
  int probe = 0;                    // thread 0: queues found empty so far
  int slo = 0, shi = 0, scur = 0;   // thread 0: unit range of the last suspension found
  for (;;) {
    if (threadIdx.x == 0) {
      int u = -1;
      while (probe < kXcds) {
        const int q = xcd + probe < kXcds ? xcd + probe : xcd + probe - kXcds;
        const int lo = meta[kMetaQueue + q], n = meta[kMetaQueue + q + 1] - lo;
        const int k = atomicAdd(&meta[kMetaCount + q], 1);
        if (k < n) {
          u = lo + k;
          break;
        }
        ++probe;
      }
      if (u >= 0 && (u < slo || u >= shi)) {
        int lo = 0, hi = nsus;  // ustart[lo] <= u < ustart[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (ustart[mid] <= u)
            lo = mid;
          else
            hi = mid;
        }
        scur = lo;
        slo = ustart[lo];
        shi = ustart[lo + 1];
      }
      s_job[0] = u;
      s_job[1] = scur;
    }
    __syncthreads();
    const int u = s_job[0], sus = s_job[1];
    __syncthreads();
    if (u < 0) return;
    const int4 st = stab[sus];
    int bx, by;
    sym_unit_blocks(st.z, u - ustart[sus], bx, by);
    const int tc0 = st.x + bx * CB, sc0 = st.x + by * CB;
    sym_eval_unit<T>(P, vtab, vaux, rec, cyc, fcyc, st.w, tc0, min(st.y, tc0 + CB), sc0, min(st.y, sc0 + CB),
                     bx == by, acc);
    __syncthreads();
  }
}

// out = acc 2^-S_s / (4 pi mu_s) for the points of suspension s.
__global__ __launch_bounds__(256) void k_symb_finish(const unsigned long long* __restrict__ acc,
                                                     const int4* __restrict__ stab, const int32_t* __restrict__ pstart,
                                                     const double* __restrict__ mu, int nsus, int P,
                                                     double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 2 * (int64_t)P;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(e < P ? e : e - P);
    int lo = 0, hi = nsus;  // pstart[lo] <= j < pstart[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pstart[mid] <= j)
        lo = mid;
      else
        hi = mid;
    }
    const double scale = 1.0 / (4.0 * kPi * mu[lo]);
    out[e] = ldexp((double)(long long)acc[e] * scale, -stab[lo].w);
  }
}

// Adjoint of the symmetric form, for targets = sources = X (the positions differentiated in both
// roles, w and f held fixed).  With c = 1/(4 pi mu), g = dL/du and phi(r; a, b) = a^T G(r) b:
//   v_k      = sum_{m not in ves(k)} G(X_k - X_m) g_m                (then dL/df = c w v, dL/dw = c f . v)
//   dL/dX_k  = c sum_{m not in ves(k)} H(X_k - X_m),  H(r) = grad phi(r; g_k, F_m) + grad phi(r; F_k, g_m),
//   grad phi(r; a, b) = [ -(a . b) r + a (r . b) + b (a . r) ] / |r|^2 - 2 (a . r)(r . b) r / |r|^4.
// G is even and grad phi odd in r (and symmetric in a, b), so the pair (k, m) adds H to k and -H to m,
// and G(r) g_k to v_m: one evaluation of r, |r|^2, its logarithm and reciprocal serves all four.
// The ring, units and compensation are those of k_sym_main, with g in place of F for v; H is of degree
// -1 in r, so on the rescaled r' = 2^-k r it is computed as H' = 2^k H and scaled back by 2^-k (rows at
// the flush, columns per pair inside the column sum).  Sums are added with float64 atomics.
template <int T>
__global__ __launch_bounds__(kSymThreads) void k_sym_bwd(
    const double4* __restrict__ vtab, const double2* __restrict__ vaux, const float4* __restrict__ recF,
    const float4* __restrict__ recG, const int4* __restrict__ cyc, const double2* __restrict__ gcyc,
    const int32_t* __restrict__ meta, int P, double* __restrict__ gsum, double* __restrict__ vsum) {
  constexpr int CB = kRows * T;
  __shared__ float4 s_tx[CB][kRing];               // target records (local coordinates, w f)
  __shared__ float2 s_tg[CB][kRing];               // target g
  __shared__ double4 s_tc[CB];                     // (c_A, G_cycle) of each target cycle
  __shared__ double s_tr[CB];                      // R_A^2
  __shared__ int4 s_ti[CB];                        // (vesicle or -1, count, first point, 0)
  __shared__ float4 s_rec[2][kChunk][2 * kRing];   // source cycles (local coordinates, w f), twice
  __shared__ float2 s_reg[2][kChunk][2 * kRing];   // source g, twice
  __shared__ float s_col[2][kSymWaves][kChunk][4][kRing];
  __shared__ double2 s_E[2][kSymWaves][kChunk];

  const int ncyc = meta[0];
  const int nb = meta[2];
  if (nb <= 0) return;
  int bx, by;
  if (!sym_unit(nb, bx, by)) return;
  const bool diag = bx == by;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, p = lane & 15;
  const int row = tid >> 4;
  const int tc0 = bx * CB, tc1 = min(ncyc, tc0 + CB);
  const int sc0 = by * CB, sc1 = min(ncyc, sc0 + CB);

  for (int e = tid; e < CB * kRing; e += kSymThreads) {
    const int t = e / kRing, m = e % kRing;
    const int c = tc0 + t;
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    float2 g = make_float2(0.f, 0.f);
    if (c < tc1) {
      const int4 cy = cyc[c];
      if (m < cy.y) {
        r = recF[cy.x + m];
        const float4 rg = recG[cy.x + m];
        g = make_float2(rg.z, rg.w);
      }
    }
    s_tx[t][m] = r;
    s_tg[t][m] = g;
  }
  for (int t = tid; t < CB; t += kSymThreads) {
    const int c = tc0 + t;
    if (c < tc1) {
      const int4 cy = cyc[c];
      const double4 vt = vtab[cy.z];
      const double2 G = gcyc[c];
      s_tc[t] = make_double4(vt.x, vt.y, G.x, G.y);
      s_tr[t] = vaux[cy.z].y;
      s_ti[t] = make_int4(cy.z, cy.y, cy.x, 0);
    } else {
      s_tc[t] = make_double4(0.0, 0.0, 0.0, 0.0);
      s_tr[t] = 0.0;
      s_ti[t] = make_int4(-1, 0, 0, 0);
    }
  }

  // per target slot k: rescaled position d and -2^-k, the target's F and g (zero when inactive),
  // -1/2 ln2 g, -2^-k for the column gradient, float32 partials of the segment, float64 sums
  float dx[T], dy[T], ns[T], fix[T], fiy[T], gix[T], giy[T], ghx[T], ghy[T];
  float lvx[T], lvy[T], rvx[T], rvy[T], gax[T], gay[T];
  double avx[T], avy[T], agx[T], agy[T];
  int kq[T];
  int actm = 0;
  double Ex = 0.0, Ey = 0.0, Gsx = 0.0, Gsy = 0.0;
#pragma unroll
  for (int k = 0; k < T; ++k) {
    dx[k] = dy[k] = ns[k] = fix[k] = fiy[k] = gix[k] = giy[k] = ghx[k] = ghy[k] = 0.f;
    lvx[k] = lvy[k] = rvx[k] = rvy[k] = gax[k] = gay[k] = 0.f;
    avx[k] = avy[k] = agx[k] = agy[k] = 0.0;
    kq[k] = 0;
  }

  auto setup = [&](int B) {
    const double4 vb = vtab[B];
    const double rb2 = vaux[B].y;
    double ex = 0.0, ey = 0.0;
    actm = 0;
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const int t = k * kRows + row;
      const int4 ti = s_ti[t];
      const double4 tc = s_tc[t];
      const float4 tx = s_tx[t][p];
      const float2 tg = s_tg[t][p];
      const double Dx = tc.x - vb.x, Dy = tc.y - vb.y;
      const double D = fma(Dy, Dy, fma(Dx, Dx, s_tr[t] + rb2));
      int e;
      frexp(D, &e);
      const int kk = min(kMaxShift, max(-kMaxShift, e >> 1));
      const bool rowact = ti.x >= 0 && ti.x != B && (!diag || ti.x < B);
      const bool act = rowact && p < ti.y;
      actm |= act ? (1 << k) : 0;
      const float sc = ldexpf(1.0f, -kk);
      dx[k] = act ? fmaf(tx.x, sc, (float)ldexp(Dx, -kk)) : kFar;
      dy[k] = act ? fmaf(tx.y, sc, (float)ldexp(Dy, -kk)) : 0.f;
      ns[k] = -sc;
      fix[k] = act ? tx.z : 0.f;
      fiy[k] = act ? tx.w : 0.f;
      gix[k] = act ? tg.x : 0.f;
      giy[k] = act ? tg.y : 0.f;
      ghx[k] = kHalfLn2f * gix[k];
      ghy[k] = kHalfLn2f * giy[k];
      kq[k] = kk;
      lvx[k] = lvy[k] = rvx[k] = rvy[k] = gax[k] = gay[k] = 0.f;
      ex += rowact ? (double)kk * tc.z : 0.0;
      ey += rowact ? (double)kk * tc.w : 0.0;
    }
    ex += __shfl_xor(ex, 16, 64);
    ey += __shfl_xor(ey, 16, 64);
    ex += __shfl_xor(ex, 32, 64);
    ey += __shfl_xor(ey, 32, 64);
    Ex = -kLn2d * ex;
    Ey = -kLn2d * ey;
    Gsx = Gsy = 0.0;
  };

  auto flush = [&]() {
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const bool act = (actm >> k) & 1;
      const float pvx = fmaf(kHalfLn2f, lvx[k], rvx[k]);
      const float pvy = fmaf(kHalfLn2f, lvy[k], rvy[k]);
      const double c = -kLn2d * (double)kq[k];
      const double sg = ldexp(1.0, -kq[k]);
      avx[k] += act ? fma(c, Gsx, (double)pvx) : 0.0;
      avy[k] += act ? fma(c, Gsy, (double)pvy) : 0.0;
      agx[k] += act ? sg * (double)gax[k] : 0.0;
      agy[k] += act ? sg * (double)gay[k] : 0.0;
    }
  };

  auto ring = [&](int buf, int cc) {
    const float4* rb = &s_rec[buf][cc][p];
    const float2* gb = &s_reg[buf][cc][p];
    float cvx = 0.f, cvy = 0.f, cgx = 0.f, cgy = 0.f;
#pragma unroll 1
    for (int s = 0; s < kRing; ++s) {
      const float4 sr = rb[s];
      const float2 sg = gb[s];
      float lvcx = 0.f, lvcy = 0.f, lgcx = 0.f, lgcy = 0.f;
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const float rx = fmaf(sr.x, ns[k], dx[k]);
        const float ry = fmaf(sr.y, ns[k], dy[k]);
        const float q = fmaf(ry, ry, rx * rx);
        const float L = __builtin_amdgcn_logf(q);
        const float rho = __builtin_amdgcn_rcpf(q);
        const float ux = rx * rho, uy = ry * rho;
        const float p3 = fmaf(uy, sg.y, ux * sg.x);        // (r . g_j)/q
        const float p2 = fmaf(uy, giy[k], ux * gix[k]);    // (r . g_i)/q
        const float p1 = fmaf(uy, sr.w, ux * sr.z);        // (r . F_j)/q
        const float p4 = fmaf(uy, fiy[k], ux * fix[k]);    // (r . F_i)/q
        // v: G(r) g_j into the row, G(r) g_i into the column
        lvx[k] = fmaf(L, sg.x, lvx[k]);
        lvy[k] = fmaf(L, sg.y, lvy[k]);
        rvx[k] = fmaf(p3, rx, rvx[k]);
        rvy[k] = fmaf(p3, ry, rvy[k]);
        // H' = -(rho (g_i . F_j + F_i . g_j) + 2 (p1 p2 + p3 p4)) r + g_i p1 + F_j p2 + F_i p3 + g_j p4
        const float ab = fmaf(gix[k], sr.z, fmaf(giy[k], sr.w, fmaf(fix[k], sg.x, fiy[k] * sg.y)));
        const float m = fmaf(2.0f, fmaf(p1, p2, p3 * p4), rho * ab);
        const float hx = fmaf(sg.x, p4, fmaf(fix[k], p3, fmaf(sr.z, p2, fmaf(gix[k], p1, -m * rx))));
        const float hy = fmaf(sg.y, p4, fmaf(fiy[k], p3, fmaf(sr.w, p2, fmaf(giy[k], p1, -m * ry))));
        gax[k] += hx;
        gay[k] += hy;
        if (k == 0) {
          lvcx = L * ghx[k];
          lvcy = L * ghy[k];
          lgcx = ns[k] * hx;
          lgcy = ns[k] * hy;
        } else {
          lvcx = fmaf(L, ghx[k], lvcx);
          lvcy = fmaf(L, ghy[k], lvcy);
          lgcx = fmaf(ns[k], hx, lgcx);
          lgcy = fmaf(ns[k], hy, lgcy);
        }
        lvcx = fmaf(p2, rx, lvcx);
        lvcy = fmaf(p2, ry, lvcy);
      }
      cvx = ring_next(cvx) + lvcx;
      cvy = ring_next(cvy) + lvcy;
      cgx = ring_next(cgx) + lgcx;
      cgy = ring_next(cgy) + lgcy;
    }
    // add the four rows: v in the first swap, the gradient in the second
    const auto hv = __builtin_amdgcn_permlane32_swap(bitsu(cvx), bitsu(cvy), false, false);
    const float zv = bitsf(hv[0]) + bitsf(hv[1]);
    const auto rv16 = __builtin_amdgcn_permlane16_swap(bitsu(zv), bitsu(zv), false, false);
    const float totv = bitsf(rv16[0]) + bitsf(rv16[1]);
    const auto hg = __builtin_amdgcn_permlane32_swap(bitsu(cgx), bitsu(cgy), false, false);
    const float zg = bitsf(hg[0]) + bitsf(hg[1]);
    const auto rg16 = __builtin_amdgcn_permlane16_swap(bitsu(zg), bitsu(zg), false, false);
    const float totg = bitsf(rg16[0]) + bitsf(rg16[1]);
    if ((lane & 16) == 0) {
      const int slot = (p + kRing - 1) & (kRing - 1);
      s_col[buf][wv][cc][lane >> 5][slot] = totv;
      s_col[buf][wv][cc][2 + (lane >> 5)][slot] = totg;
    }
  };

  const int nchunks = (sc1 - sc0 + kChunk - 1) / kChunk;
  const bool stager = tid < kChunk * 2 * kRing;
  const int st_cc = tid >> 5, st_q = tid & 31, st_m = st_q & (kRing - 1);
  auto stage_load = [&](int g, float2& gg) {
    float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
    gg = make_float2(0.f, 0.f);
    const int c = sc0 + g * kChunk + st_cc;
    if (stager && c < sc1) {
      const int4 cy = cyc[c];
      const int j = cy.x + (st_m < cy.y ? st_m : 0);
      r = recF[j];
      const float4 rg = recG[j];
      if (st_m >= cy.y) {
        r.z = r.w = 0.f;
      } else {
        gg = make_float2(rg.z, rg.w);
      }
    }
    return r;
  };
  auto stage_store = [&](int buf, const float4& r, const float2& gg) {
    if (stager) {
      s_rec[buf][st_cc][st_q] = r;
      s_reg[buf][st_cc][st_q] = gg;
    }
  };

  // Column sums of chunk g: v (with its log correction) and the gradient, added over the
  // wavefronts in a fixed order, then one float64 atomic addition per (source, component).
  auto reduce = [&](int g, int buf) {
    for (int e = tid; e < kChunk * 4 * kRing; e += kSymThreads) {
      const int cc = e / (4 * kRing), comp = (e / kRing) & 3, m = e & (kRing - 1);
      const int c = sc0 + g * kChunk + cc;
      if (c >= sc1) continue;
      const int4 cy = cyc[c];
      if (m >= cy.y) continue;
      double s = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < kSymWaves; ++w2) s += (double)s_col[buf][w2][cc][comp][m];
      if (comp < 2) {
#pragma unroll
        for (int w2 = 0; w2 < kSymWaves; ++w2) {
          const double2 E = s_E[buf][w2][cc];
          s += comp ? E.y : E.x;
        }
        atomicAdd(&vsum[(size_t)comp * P + cy.x + m], s);
      } else {
        atomicAdd(&gsum[(size_t)(comp - 2) * P + cy.x + m], s);
      }
    }
  };

  int curB = -1;
  {
    float2 gg;
    const float4 r = stage_load(0, gg);
    stage_store(0, r, gg);
  }
  __syncthreads();
  for (int g = 0; g < nchunks; ++g) {
    const int buf = g & 1;
    float2 ngg;
    const float4 nxt = stage_load(g + 1, ngg);
    if (g > 0) reduce(g - 1, buf ^ 1);
    const int cbase = sc0 + g * kChunk;
    const int ncc = min(kChunk, sc1 - cbase);
    for (int cc = 0; cc < ncc; ++cc) {
      const int4 cy = cyc[cbase + cc];
      if (cy.z != curB) {
        if (curB >= 0) flush();
        setup(cy.z);
        curB = cy.z;
      }
      const double2 Gc = gcyc[cbase + cc];
      Gsx += Gc.x;
      Gsy += Gc.y;
      ring(buf, cc);
      if (lane == 0) s_E[buf][wv][cc] = make_double2(Ex, Ey);
    }
    stage_store(buf ^ 1, nxt, ngg);
    __syncthreads();
  }
  if (nchunks > 0) {
    reduce(nchunks - 1, (nchunks - 1) & 1);
    flush();
  }
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const int4 ti = s_ti[k * kRows + row];
    if (ti.x >= 0 && p < ti.y) {
      const int i = ti.z + p;
      atomicAdd(&vsum[i], avx[k]);
      atomicAdd(&vsum[(size_t)P + i], avy[k]);
      atomicAdd(&gsum[i], agx[k]);
      atomicAdd(&gsum[(size_t)P + i], agy[k]);
    }
  }
}

// Float64 adjoint for targets = sources, on the schedule of k_sym64_main: per pair the same v (G(r) g_j to
// the row, G(r) g_i to the column) and H (+H to the row, -H to the column) as k_sym_bwd, on global
// coordinates without compensation; four float64 sums travel around the ring.  Sums are added with float64
// atomics, as in k_sym_bwd.
template <int T>
__global__ __launch_bounds__(kSymThreads) void k_sym64_bwd(const double4* __restrict__ recF,
                                                           const double4* __restrict__ recG,
                                                           const int4* __restrict__ cyc,
                                                           const int32_t* __restrict__ meta, int P,
                                                           double* __restrict__ gsum, double* __restrict__ vsum) {
  constexpr int CB = kRows * T;
  __shared__ int4 s_ti[CB];                          // (vesicle or -1, count, first point, 0)
  __shared__ double4 s_rec[2][kChunk64][2 * kRing];  // source cycles (x, y, F_x, F_y), twice
  __shared__ double2 s_reg[2][kChunk64][2 * kRing];  // source g, twice
  __shared__ double s_col[2][kSymWaves][kChunk64][4][kRing];
  __shared__ double2 ltab[kLogTab64];

  const int ncyc = meta[0];
  const int nb = meta[2];
  if (nb <= 0) return;
  int bx, by;
  if (!sym_unit(nb, bx, by)) return;
  const bool diag = bx == by;
  const int tc0 = bx * CB, tc1 = min(ncyc, tc0 + CB);
  const int sc0 = by * CB, sc1 = min(ncyc, sc0 + CB);

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, p = lane & 15;
  const int row = tid >> 4;
  for (int e = tid; e < kLogTab64; e += kSymThreads) ltab[e] = log_tab_entry_n<kLogTab64>(e);
  for (int t = tid; t < CB; t += kSymThreads) {
    const int c = tc0 + t;
    if (c < tc1) {
      const int4 cy = cyc[c];
      s_ti[t] = make_int4(cy.z, cy.y, cy.x, 0);
    } else {
      s_ti[t] = make_int4(-1, 0, 0, 0);
    }
  }
  __syncthreads();

  double4 tf[T];
  double2 tg[T];
  int4 ti[T];
#pragma unroll
  for (int k = 0; k < T; ++k) {
    ti[k] = s_ti[k * kRows + row];
    const bool in = ti[k].x >= 0 && p < ti[k].y;
    tf[k] = in ? recF[ti[k].z + p] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double4 g4 = in ? recG[ti[k].z + p] : make_double4(0.0, 0.0, 0.0, 0.0);
    tg[k] = make_double2(g4.z, g4.w);
  }
  // per target slot k: position (or a far point), F and g (zero when inactive), -1/2 g, the segment's
  // partials (log and rr parts of v, H) and the unit's sums
  double dx[T], dy[T], fix[T], fiy[T], gix[T], giy[T], ghx[T], ghy[T];
  double lvx[T], lvy[T], rvx[T], rvy[T], gax[T], gay[T], avx[T], avy[T], agx[T], agy[T];
  int actm = 0;
#pragma unroll
  for (int k = 0; k < T; ++k) {
    dx[k] = dy[k] = fix[k] = fiy[k] = gix[k] = giy[k] = ghx[k] = ghy[k] = 0.0;
    lvx[k] = lvy[k] = rvx[k] = rvy[k] = gax[k] = gay[k] = avx[k] = avy[k] = agx[k] = agy[k] = 0.0;
  }

  auto setup = [&](int B) {
    actm = 0;
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const bool act = ti[k].x >= 0 && ti[k].x != B && (!diag || ti[k].x < B) && p < ti[k].y;
      actm |= act ? (1 << k) : 0;
      dx[k] = act ? tf[k].x : kFar64;
      dy[k] = act ? tf[k].y : 0.0;
      fix[k] = act ? tf[k].z : 0.0;
      fiy[k] = act ? tf[k].w : 0.0;
      gix[k] = act ? tg[k].x : 0.0;
      giy[k] = act ? tg[k].y : 0.0;
      ghx[k] = -0.5 * gix[k];
      ghy[k] = -0.5 * giy[k];
      lvx[k] = lvy[k] = rvx[k] = rvy[k] = gax[k] = gay[k] = 0.0;
    }
  };

  auto flush = [&]() {
#pragma unroll
    for (int k = 0; k < T; ++k) {
      const bool act = (actm >> k) & 1;
      avx[k] += act ? fma(-0.5, lvx[k], rvx[k]) : 0.0;
      avy[k] += act ? fma(-0.5, lvy[k], rvy[k]) : 0.0;
      agx[k] += act ? gax[k] : 0.0;
      agy[k] += act ? gay[k] : 0.0;
    }
  };

  auto ring = [&](int buf, int cc) {
    const double4* rb = &s_rec[buf][cc][p];
    const double2* gb = &s_reg[buf][cc][p];
    double cvx = 0.0, cvy = 0.0, cgx = 0.0, cgy = 0.0;
#pragma unroll 1
    for (int s = 0; s < kRing; ++s) {
      const double4 sr = rb[s];
      const double2 sg = gb[s];
      double lvcx = 0.0, lvcy = 0.0, lgcx = 0.0, lgcy = 0.0;
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const double rx = dx[k] - sr.x;
        const double ry = dy[k] - sr.y;
        const double q = fma(ry, ry, rx * rx);
        const double L = log_reduced_n<kLogTab64>(q, ltab);
        const double rho = recip(q);
        const double ux = rx * rho, uy = ry * rho;
        const double p3 = fma(uy, sg.y, ux * sg.x);        // (r . g_j)/q
        const double p2 = fma(uy, giy[k], ux * gix[k]);    // (r . g_i)/q
        const double p1 = fma(uy, sr.w, ux * sr.z);        // (r . F_j)/q
        const double p4 = fma(uy, fiy[k], ux * fix[k]);    // (r . F_i)/q
        lvx[k] = fma(L, sg.x, lvx[k]);
        lvy[k] = fma(L, sg.y, lvy[k]);
        rvx[k] = fma(p3, rx, rvx[k]);
        rvy[k] = fma(p3, ry, rvy[k]);
        // H = -(rho (g_i . F_j + F_i . g_j) + 2 (p1 p2 + p3 p4)) r + g_i p1 + F_j p2 + F_i p3 + g_j p4
        const double ab = fma(gix[k], sr.z, fma(giy[k], sr.w, fma(fix[k], sg.x, fiy[k] * sg.y)));
        const double m = fma(2.0, fma(p1, p2, p3 * p4), rho * ab);
        const double hx = fma(sg.x, p4, fma(fix[k], p3, fma(sr.z, p2, fma(gix[k], p1, -m * rx))));
        const double hy = fma(sg.y, p4, fma(fiy[k], p3, fma(sr.w, p2, fma(giy[k], p1, -m * ry))));
        gax[k] += hx;
        gay[k] += hy;
        if (k == 0) {
          lvcx = L * ghx[k];
          lvcy = L * ghy[k];
          lgcx = -hx;
          lgcy = -hy;
        } else {
          lvcx = fma(L, ghx[k], lvcx);
          lvcy = fma(L, ghy[k], lvcy);
          lgcx -= hx;
          lgcy -= hy;
        }
        lvcx = fma(p2, rx, lvcx);
        lvcy = fma(p2, ry, lvcy);
      }
      cvx = ring_next64(cvx) + lvcx;
      cvy = ring_next64(cvy) + lvcy;
      cgx = ring_next64(cgx) + lgcx;
      cgy = ring_next64(cgy) + lgcy;
    }
    // add the four rows of the wavefront (both halves of each double swapped alike): v, then H
    auto rows4 = [&](double a, double b) {
      const unsigned long long ba = dlo(a), bb = dlo(b);
      const auto hl = __builtin_amdgcn_permlane32_swap((unsigned)ba, (unsigned)bb, false, false);
      const auto hh = __builtin_amdgcn_permlane32_swap((unsigned)(ba >> 32), (unsigned)(bb >> 32), false, false);
      const double z = dfrom(hl[0], hh[0]) + dfrom(hl[1], hh[1]);
      const unsigned long long bz = dlo(z);
      const auto gl = __builtin_amdgcn_permlane16_swap((unsigned)bz, (unsigned)bz, false, false);
      const auto gh = __builtin_amdgcn_permlane16_swap((unsigned)(bz >> 32), (unsigned)(bz >> 32), false, false);
      return dfrom(gl[0], gh[0]) + dfrom(gl[1], gh[1]);
    };
    const double totv = rows4(cvx, cvy);
    const double totg = rows4(cgx, cgy);
    if ((lane & 16) == 0) {
      const int slot = (p + kRing - 1) & (kRing - 1);
      s_col[buf][wv][cc][lane >> 5][slot] = totv;
      s_col[buf][wv][cc][2 + (lane >> 5)][slot] = totg;
    }
  };

  const int nchunks = (sc1 - sc0 + kChunk64 - 1) / kChunk64;
  const bool stager = tid < kChunk64 * 2 * kRing;
  const int st_cc = tid >> 5, st_q = tid & 31, st_m = st_q & (kRing - 1);
  auto stage_load = [&](int g, double2& gg) {
    double4 r = make_double4(0.0, 0.0, 0.0, 0.0);
    gg = make_double2(0.0, 0.0);
    const int c = sc0 + g * kChunk64 + st_cc;
    if (stager && c < sc1) {
      const int4 cy = cyc[c];
      const int j = cy.x + (st_m < cy.y ? st_m : 0);
      r = recF[j];
      const double4 rg = recG[j];
      if (st_m >= cy.y) {
        r.z = r.w = 0.0;
      } else {
        gg = make_double2(rg.z, rg.w);
      }
    }
    return r;
  };
  auto stage_store = [&](int buf, const double4& r, const double2& gg) {
    if (stager) {
      s_rec[buf][st_cc][st_q] = r;
      s_reg[buf][st_cc][st_q] = gg;
    }
  };
  // column sums of chunk g: v and H added over the wavefronts in a fixed order, one float64 atomic
  // addition per (source, quantity, component)
  auto reduce = [&](int g, int buf) {
    const int cc = tid >> 6, comp = (tid >> 4) & 3, m = tid & (kRing - 1);
    const int c = sc0 + g * kChunk64 + cc;
    if (cc >= kChunk64 || c >= sc1) return;
    const int4 cy = cyc[c];
    if (m >= cy.y) return;
    const double v = ((s_col[buf][0][cc][comp][m] + s_col[buf][1][cc][comp][m]) + s_col[buf][2][cc][comp][m]) +
                     s_col[buf][3][cc][comp][m];
    double* dst = comp < 2 ? vsum : gsum;
    atomicAdd(&dst[(size_t)(comp & 1) * P + cy.x + m], v);
  };

  int curB = -1;
  {
    double2 g0;
    const double4 r0 = stage_load(0, g0);
    stage_store(0, r0, g0);
  }
  __syncthreads();
  for (int g = 0; g < nchunks; ++g) {
    const int buf = g & 1;
    double2 ng;
    const double4 nxt = stage_load(g + 1, ng);
    if (g > 0) reduce(g - 1, buf ^ 1);
    const int cbase = sc0 + g * kChunk64;
    const int ncc = min(kChunk64, sc1 - cbase);
    for (int cc = 0; cc < ncc; ++cc) {
      const int4 cy = cyc[cbase + cc];
      if (cy.z != curB) {
        if (curB >= 0) flush();
        setup(cy.z);
        curB = cy.z;
      }
      ring(buf, cc);
    }
    stage_store(buf ^ 1, nxt, ng);
    __syncthreads();
  }
  if (nchunks > 0) {
    reduce(nchunks - 1, (nchunks - 1) & 1);
    flush();
  }
#pragma unroll
  for (int k = 0; k < T; ++k) {
    if (ti[k].x >= 0 && p < ti[k].y) {
      const int i = ti[k].z + p;
      atomicAdd(&vsum[i], avx[k]);
      atomicAdd(&vsum[(size_t)P + i], avy[k]);
      atomicAdd(&gsum[i], agx[k]);
      atomicAdd(&gsum[(size_t)P + i], agy[k]);
    }
  }
}

__global__ __launch_bounds__(256) void k_zero_f64(double* __restrict__ a, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    a[e] = 0.0;
}

__global__ __launch_bounds__(256) void k_add_f64(double* __restrict__ a, const double* __restrict__ b, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    a[e] += b[e];
}

// dL/dX = c gsum (in place), dL/df = c w v, dL/dw = c f . v
__global__ __launch_bounds__(256) void k_sym_bwd_finish(const double* __restrict__ vsum, const double* __restrict__ f,
                                                        const double* __restrict__ w, int P, double scale,
                                                        double* __restrict__ gX, double* __restrict__ gf,
                                                        double* __restrict__ gw) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < P; j += gridDim.x * blockDim.x) {
    if (gX) {
      gX[j] *= scale;
      gX[P + j] *= scale;
    }
    const double vx = scale * vsum[j], vy = scale * vsum[P + j];
    if (gf) {
      gf[j] = w[j] * vx;
      gf[P + j] = w[j] * vy;
    }
    if (gw) gw[j] = f[j] * vx + f[P + j] * vy;
  }
}

__global__ __launch_bounds__(256) void k_sym_finish(const unsigned long long* __restrict__ acc,
                                                    const int32_t* __restrict__ meta, int P, double scale,
                                                    double* __restrict__ out) {
  const int S = meta[1];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < 2 * (int64_t)P;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = ldexp((double)(long long)acc[e] * scale, -S);
}

}  // namespace

static inline hipStream_t Sx_(void* s) { return reinterpret_cast<hipStream_t>(s); }

int sym_cycles_per_block(int T) { return kRows * T; }

int64_t sym_max_cycles(int P, int M) { return (int64_t)P / kRing + (int64_t)M + 1; }

int64_t sym_max_blocks(int P, int M, int T) {
  const int cb = sym_cycles_per_block(T);
  return (sym_max_cycles(P, M) + cb - 1) / cb;
}

int64_t sym_units(int64_t nb) {
  if (nb <= 0) return 0;
  const int64_t h = nb / 2;
  return (nb & 1) ? nb * (h + 1) : nb * h + h;
}

bool sym_fits(int P, int M, int T) { return sym_units(sym_max_blocks(P, M, T)) <= (int64_t)INT32_MAX; }

hipError_t launch_backward_symmetric(int T, int P, int M, const PreparedView& pvF, const PreparedView& pvG,
                                     const SymmetricView& sv, double* vsum, const double* f, const double* w,
                                     double scale, double* grad_points, double* grad_f, double* grad_w,
                                     void* stream) {
  if (P == 0) return hipSuccess;
  if (!grad_points || !vsum) return hipErrorInvalidValue;
  hipStream_t st = Sx_(stream);
  const int cb = sym_cycles_per_block(T);
  const int ncyc_max = (int)sym_max_cycles(P, M);
  const int nb_max = (int)sym_max_blocks(P, M, T);
  hipLaunchKernelGGL(k_sym_plan, dim3(1), dim3(1024), 0, st, pvF.vrange, pvF.vaux, M, cb, ncyc_max, sv.cyc, sv.meta);
  const int cgrid = (int)std::min<int64_t>((2 * (int64_t)P + 255) / 256, 4096);
  // cycle sums of g (its float64 copy is the f64 array of the g-prepared region)
  hipLaunchKernelGGL(k_sym_cycles, dim3(cgrid), dim3(256), 0, st, sv.cyc, sv.meta, pvG.f64, P, sv.fcyc, sv.acc);
  hipLaunchKernelGGL(k_zero_f64, dim3(cgrid), dim3(256), 0, st, grad_points, 2 * (int64_t)P);
  hipLaunchKernelGGL(k_zero_f64, dim3(cgrid), dim3(256), 0, st, vsum, 2 * (int64_t)P);
  const dim3 grid((unsigned)sym_units(nb_max));
  const float4* recF = static_cast<const float4*>(pvF.rec);
  const float4* recG = static_cast<const float4*>(pvG.rec);
  switch (T) {
#define VESNET_SYMB_CASE(TT)                                                                                   \
  case TT:                                                                                                     \
    hipLaunchKernelGGL(k_sym_bwd<TT>, grid, dim3(kSymThreads), 0, st, pvF.vtab, pvF.vaux, recF, recG, sv.cyc,  \
                       sv.fcyc, sv.meta, P, grad_points, vsum);                                                 \
    break;
    VESNET_SYMB_CASE(1) VESNET_SYMB_CASE(2) VESNET_SYMB_CASE(3) VESNET_SYMB_CASE(4)
#undef VESNET_SYMB_CASE
    default: return hipErrorInvalidValue;
  }
  const int fgrid = (P + 255) / 256 < 16384 ? (P + 255) / 256 : 16384;
  hipLaunchKernelGGL(k_sym_bwd_finish, dim3(fgrid), dim3(256), 0, st, vsum, f, w, P, scale, grad_points, grad_f,
                     grad_w);
  return hipGetLastError();
}

hipError_t launch_backward_symmetric64(int T, int P, int M, const PreparedView& pvF, const PreparedView& pvG,
                                       const SymmetricView& sv, double* vsum, const double* f, const double* w,
                                       double scale, double* grad_points, double* grad_f, double* grad_w,
                                       void* stream) {
  if (P == 0) return hipSuccess;
  if (!grad_points || !vsum) return hipErrorInvalidValue;
  hipStream_t st = Sx_(stream);
  const int cb = sym_cycles_per_block(T);
  const int ncyc_max = (int)sym_max_cycles(P, M);
  const int nb_max = (int)sym_max_blocks(P, M, T);
  hipLaunchKernelGGL(k_sym_plan, dim3(1), dim3(1024), 0, st, pvF.vrange, pvF.vaux, M, cb, ncyc_max, sv.cyc, sv.meta);
  const int cgrid = (int)std::min<int64_t>((2 * (int64_t)P + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_f64, dim3(cgrid), dim3(256), 0, st, grad_points, 2 * (int64_t)P);
  hipLaunchKernelGGL(k_zero_f64, dim3(cgrid), dim3(256), 0, st, vsum, 2 * (int64_t)P);
  const dim3 grid((unsigned)sym_units(nb_max));
  const double4* recF = static_cast<const double4*>(pvF.rec);
  const double4* recG = static_cast<const double4*>(pvG.rec);
  switch (T) {
    case 1: hipLaunchKernelGGL(k_sym64_bwd<1>, grid, dim3(kSymThreads), 0, st, recF, recG, sv.cyc, sv.meta, P,
                               grad_points, vsum); break;
    case 2: hipLaunchKernelGGL(k_sym64_bwd<2>, grid, dim3(kSymThreads), 0, st, recF, recG, sv.cyc, sv.meta, P,
                               grad_points, vsum); break;
    default: return hipErrorInvalidValue;
  }
  const int fgrid = (P + 255) / 256 < 16384 ? (P + 255) / 256 : 16384;
  hipLaunchKernelGGL(k_sym_bwd_finish, dim3(fgrid), dim3(256), 0, st, vsum, f, w, P, scale, grad_points, grad_f,
                     grad_w);
  return hipGetLastError();
}

hipError_t launch_add_f64(double* a, const double* b, int64_t n, void* stream) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_add_f64, dim3(grid), dim3(256), 0, Sx_(stream), a, b, n);
  return hipGetLastError();
}

int64_t symb_max_units(int P, int M, int S, int T) {
  // the blocks of all suspensions number at most (cycles / CB) + S, and n (n + 1) / 2 is superadditive
  return sym_units(sym_max_blocks(P, M, T) + S);
}

// Cached after the first query (every device this library runs on is a gfx950).
int symb_units_per_cu(int T) {
  static std::atomic<int> cache[5] = {};
  if (T < 1 || T > 4) return 1;
  int n = cache[T].load(std::memory_order_relaxed);
  if (n > 0) return n;
  hipError_t e = hipErrorInvalidValue;
  switch (T) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_symb_main<1>, kSymThreads, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_symb_main<2>, kSymThreads, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_symb_main<3>, kSymThreads, 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_symb_main<4>, kSymThreads, 0); break;
  }
  if (e != hipSuccess || n <= 0) return 1;
  cache[T].store(n, std::memory_order_relaxed);
  return n;
}

hipError_t launch_batched_symmetric(int T, int grid, int P, int M, const PreparedView& pv, const SymmetricView& sv,
                                    const SymBatchView& bv, const int32_t* sus_off, const int32_t* off, int S,
                                    const double* mu, double* out, void* stream) {
  if (P == 0 || S == 0) return hipSuccess;
  if (grid < 1) return hipErrorInvalidValue;
  hipStream_t st = Sx_(stream);
  const int cb = sym_cycles_per_block(T);
  const int ncyc_max = (int)sym_max_cycles(P, M);
  hipLaunchKernelGGL(k_symb_plan, dim3(1), dim3(1024), 0, st, pv.vrange, pv.vaux, sus_off, M, P, S, cb, ncyc_max,
                     sv.cyc, bv.stab, bv.ustart, bv.pstart, bv.vr, sv.meta);
  const int cgrid = (int)std::min<int64_t>((2 * (int64_t)P + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sym_cycles, dim3(cgrid), dim3(256), 0, st, sv.cyc, sv.meta, pv.f64, P, sv.fcyc, sv.acc);
  const float4* rec = static_cast<const float4*>(pv.rec);
  switch (T) {
#define VESNET_SYMB_MAIN(TT)                                                                                     \
  case TT:                                                                                                       \
    hipLaunchKernelGGL(k_symb_main<TT>, dim3(grid), dim3(kSymThreads), 0, st, P, pv.vtab, pv.vaux, rec, sv.cyc, \
                       sv.fcyc, bv.stab, bv.ustart, S, sv.meta, sv.acc);                                          \
    break;
    VESNET_SYMB_MAIN(1) VESNET_SYMB_MAIN(2) VESNET_SYMB_MAIN(3) VESNET_SYMB_MAIN(4)
#undef VESNET_SYMB_MAIN
    default: return hipErrorInvalidValue;
  }
  const int64_t n = 2 * (int64_t)P;
  const int fgrid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
  hipLaunchKernelGGL(k_symb_finish, dim3(fgrid), dim3(256), 0, st, sv.acc, bv.stab, bv.pstart, mu, S, P, out);
  return hipGetLastError();
}

hipError_t launch_forward_symmetric64(int T, int P, int M, const PreparedView& pv, const SymmetricView& sv,
                                      double scale, double* out, void* stream) {
  if (P == 0) return hipSuccess;
  hipStream_t st = Sx_(stream);
  const int cb = sym_cycles_per_block(T);
  const int ncyc_max = (int)sym_max_cycles(P, M);
  const int nb_max = (int)sym_max_blocks(P, M, T);
  hipLaunchKernelGGL(k_sym_plan, dim3(1), dim3(1024), 0, st, pv.vrange, pv.vaux, M, cb, ncyc_max, sv.cyc, sv.meta);
  // cycle forces (unused here) and the first 2P accumulator words; the low words are zeroed below
  const int cgrid = (int)std::min<int64_t>((2 * (int64_t)P + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sym_cycles, dim3(cgrid), dim3(256), 0, st, sv.cyc, sv.meta, pv.f64, P, sv.fcyc, sv.acc);
  hipLaunchKernelGGL(k_zero_f64, dim3(cgrid), dim3(256), 0, st, reinterpret_cast<double*>(sv.acc + 2 * (size_t)P),
                     2 * (int64_t)P);
  const dim3 grid((unsigned)sym_units(nb_max));
  const double4* rec = static_cast<const double4*>(pv.rec);
  switch (T) {
    case 1: hipLaunchKernelGGL(k_sym64_main<1>, grid, dim3(kSymThreads), 0, st, P, rec, sv.cyc, sv.meta, sv.acc); break;
    case 2: hipLaunchKernelGGL(k_sym64_main<2>, grid, dim3(kSymThreads), 0, st, P, rec, sv.cyc, sv.meta, sv.acc); break;
    case 3: hipLaunchKernelGGL(k_sym64_main<3>, grid, dim3(kSymThreads), 0, st, P, rec, sv.cyc, sv.meta, sv.acc); break;
    case 4: hipLaunchKernelGGL(k_sym64_main<4>, grid, dim3(kSymThreads), 0, st, P, rec, sv.cyc, sv.meta, sv.acc); break;
    default: return hipErrorInvalidValue;
  }
  const int64_t n = 2 * (int64_t)P;
  const int fgrid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
  hipLaunchKernelGGL(k_sym64_finish, dim3(fgrid), dim3(256), 0, st, sv.acc, sv.meta, P, scale, out);
  return hipGetLastError();
}

hipError_t launch_forward_symmetric(int T, int P, int M, const PreparedView& pv, const SymmetricView& sv,
                                    double scale, double* out, void* stream) {
  if (P == 0) return hipSuccess;
  hipStream_t st = Sx_(stream);
  const int cb = sym_cycles_per_block(T);
  const int ncyc_max = (int)sym_max_cycles(P, M);
  const int nb_max = (int)sym_max_blocks(P, M, T);
  hipLaunchKernelGGL(k_sym_plan, dim3(1), dim3(1024), 0, st, pv.vrange, pv.vaux, M, cb, ncyc_max, sv.cyc, sv.meta);
  const int cgrid = (int)std::min<int64_t>((2 * (int64_t)P + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sym_cycles, dim3(cgrid), dim3(256), 0, st, sv.cyc, sv.meta, pv.f64, P, sv.fcyc, sv.acc);
  const dim3 grid((unsigned)sym_units(nb_max));
  const float4* rec = static_cast<const float4*>(pv.rec);
  switch (T) {
#define VESNET_SYM_CASE(TT)                                                                                    \
  case TT:                                                                                                     \
    hipLaunchKernelGGL(k_sym_main<TT>, grid, dim3(kSymThreads), 0, st, P, pv.vtab, pv.vaux, rec, sv.cyc,      \
                       sv.fcyc, sv.meta, sv.acc);                                                               \
    break;
    VESNET_SYM_CASE(1) VESNET_SYM_CASE(2) VESNET_SYM_CASE(3) VESNET_SYM_CASE(4) VESNET_SYM_CASE(8)
#undef VESNET_SYM_CASE
    default: return hipErrorInvalidValue;
  }
  const int64_t n = 2 * (int64_t)P;
  const int fgrid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
  hipLaunchKernelGGL(k_sym_finish, dim3(fgrid), dim3(256), 0, st, sv.acc, sv.meta, P, scale, out);
  return hipGetLastError();
}

}  // namespace vesnet
