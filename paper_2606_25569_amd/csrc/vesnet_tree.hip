// Treecode far field on gfx950: the far-field sum of eq. (single_layer) at O(P log P) cost.  The
// paper evaluates the sum directly and leaves fast summation out of scope (Section 4.1); this is
// a fast, approximate alternative with its own accuracy contract (order p of the expansions).
//
// With complex numbers z = x + i y, F_j = w_j (f_x + i f_y)_j, u = u_x + i u_y, each Stokeslet term is
//   -F_j ln|z - z_j| + F_j / 2 + (z - z_j) conj(F_j / (z - z_j)) / 2,
// so a box of sources with centre c, zeta_j = z_j - c, acts at w = z - c, t = 1/w, through the
// power moments M_k[q] = sum_j q_j zeta_j^k of three charge sets (F, conj F, conj(zeta) F):
//   -M_0[F] ln|w| + 1/2 sum_{k=1}^p (M_k[F] t^k + conj(M_k[conj F] t^k)) / k + M_0[F] / 2
//   + (w conj(Phi) - conj(Psi)) / 2,   Phi = sum_{k=0}^p M_k[F] t^(k+1),  Psi = sum_k M_k[conj(zeta) F] t^(k+1).
//
// The evaluation merges the conj-F log series and Psi into one series D, and writes w conj(Phi) as
// (w / conj w) conj(E), E = sum_k M_k[F] t^k: three Horner chains per box.
//
// Tree: a uniform quadtree of depth L over the bounding square of the points.  Leaf moments come
// from the points (k_tc_p2m), coarser ones by exact binomial translation (k_tc_m2m).  A target takes,
// at each level l = 2..L, the interaction list of its level-l ancestor (children of the parent's
// 3 x 3 neighbourhood not adjacent to the ancestor) through the expansions, and the 3 x 3 leaves
// around its own directly, skipping its own vesicle; own-vesicle sources outside those leaves,
// which the expansions included, are subtracted exactly.  Everything is FP64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "vesnet_internal.h"

namespace vesnet {

namespace {

constexpr int kTB = 256;       // threads of the point-parallel kernels
constexpr int kBBoxBlocks = 256;
constexpr int kSortMax = 2048;  // larger leaves keep the order of the atomic scatter

struct Geom {
  double x0, y0, side;  // lower-left corner and side of the root square
};

constexpr int kMaxDepth = 10;
constexpr int kMaxOrder = 48;

// Where each level's boxes start: in boxes (counts) and in complex moment entries.
struct Levels {
  unsigned long long box[kMaxDepth + 1];
  unsigned long long mom[kMaxDepth + 1];
};

__device__ __forceinline__ int clamp_i(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * t + c
__device__ __forceinline__ double2 cfma(double2 a, double2 t, double2 c) {
  return make_double2(fma(a.x, t.x, fma(-a.y, t.y, c.x)), fma(a.x, t.y, fma(a.y, t.x, c.y)));
}

// 1 / x for finite x != 0: the hardware estimate refined by two Newton steps (each doubles the correct
// bits; the result is within an ulp or so of the correctly rounded quotient).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
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

// Table of the reduced log below: entry i (mantissa interval [1 + i/64, 1 + (i+1)/64)) holds a 10-bit
// approximation a of 1 / (1 + (i + 0.5) / 64) and -ln a (from log_pos).  One entry per lane.
constexpr int kLogTab = 64;
__device__ __forceinline__ double2 log_tab_entry(int i) {
  const double c = 1.0 + ((double)i + 0.5) / 64.0;
  const double a = rint(512.0 / c) / 512.0;
  return make_double2(a, -log_pos(a));
}

// Natural log of a finite q > 0 with the table: q = m 2^e, m in [1, 2); r = m a - 1 (exact product, one
// rounding), |r| < 0.009, ln m = -ln a + log1p(r), log1p by its series through r^7 (the next term is
// below 5e-18); ln 2 in a high and a low part as in log_pos.  About 20 operations, no division.
__device__ __forceinline__ double log_reduced(double q, const double2* __restrict__ tab) {
  constexpr double kLn2Hi = 6.93147180369123816490e-01;
  constexpr double kLn2Lo = 1.90821492927058770002e-10;
  int e;
  const double m = 2.0 * frexp(q, &e);
  const int i = clamp_i((int)fma(m, 64.0, -64.0), 0, kLogTab - 1);
  const double2 t = tab[i];
  const double r = fma(m, t.x, -1.0);
  double pol = 1.0 / 7.0;
  pol = fma(pol, r, -1.0 / 6.0);
  pol = fma(pol, r, 1.0 / 5.0);
  pol = fma(pol, r, -1.0 / 4.0);
  pol = fma(pol, r, 1.0 / 3.0);
  pol = fma(pol, r, -0.5);
  pol = fma(pol, r, 1.0);
  const double ed = (double)(e - 1);
  return fma(ed, kLn2Hi, fma(ed, kLn2Lo, fma(r, pol, t.y)));
}

// Box centre at a level with n boxes per side (contraction off: the same bits as the plain formula).
__device__ __forceinline__ double2 box_center(const Geom& g, int n, int bx, int by) {
#pragma clang fp contract(off)
  const double wl = g.side / (double)n;
  return make_double2(g.x0 + ((double)bx + 0.5) * wl, g.y0 + ((double)by + 0.5) * wl);
}

// First box of level l >= 2 when levels 2, 3, ... are stored one after another: sum_{m=2}^{l-1} 4^m.
__device__ __forceinline__ size_t level_box_base(int l) { return (((size_t)1 << (2 * l)) - 16) / 3; }

// ---------------------------------------------------------------- tree construction

__global__ __launch_bounds__(kTB) void k_tc_bbox_partial(const double* __restrict__ X, int P,
                                                         double* __restrict__ part) {
  __shared__ double red[4][kTB];
  double xl = INFINITY, xh = -INFINITY, yl = INFINITY, yh = -INFINITY;
  for (int j = blockIdx.x * kTB + threadIdx.x; j < P; j += gridDim.x * kTB) {
    const double x = X[j], y = X[P + j];
    xl = fmin(xl, x);
    xh = fmax(xh, x);
    yl = fmin(yl, y);
    yh = fmax(yh, y);
  }
  red[0][threadIdx.x] = xl;
  red[1][threadIdx.x] = xh;
  red[2][threadIdx.x] = yl;
  red[3][threadIdx.x] = yh;
  __syncthreads();
  for (int s = kTB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
      red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + s]);
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void k_tc_bbox_final(const double* __restrict__ part, int nparts,
                                                      Geom* __restrict__ geom) {
  double xl = INFINITY, xh = -INFINITY, yl = INFINITY, yh = -INFINITY;
  for (int b = threadIdx.x; b < nparts; b += 64) {
    xl = fmin(xl, part[4 * b]);
    xh = fmax(xh, part[4 * b + 1]);
    yl = fmin(yl, part[4 * b + 2]);
    yh = fmax(yh, part[4 * b + 3]);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    xl = fmin(xl, __shfl_xor(xl, m, 64));
    xh = fmax(xh, __shfl_xor(xh, m, 64));
    yl = fmin(yl, __shfl_xor(yl, m, 64));
    yh = fmax(yh, __shfl_xor(yh, m, 64));
  }
  if (threadIdx.x != 0) return;
  {
#pragma clang fp contract(off)
    double side = fmax(xh - xl, yh - yl);
    if (side == 0.0) side = 1.0;
    Geom g;
    g.x0 = 0.5 * (xl + xh) - 0.5 * side;
    g.y0 = 0.5 * (yl + yh) - 0.5 * side;
    g.side = side;
    *geom = g;
  }
}

__global__ __launch_bounds__(kTB) void k_tc_zero(int32_t* __restrict__ a, int n) {
  for (int i = blockIdx.x * kTB + threadIdx.x; i < n; i += gridDim.x * kTB) a[i] = 0;
}

// Leaf of every point, leaf occupancy, vesicle id of every point.
__global__ __launch_bounds__(kTB) void k_tc_leaf(const double* __restrict__ X, int P, const Geom* __restrict__ geom,
                                                 int depth, const int32_t* __restrict__ off, int M,
                                                 int32_t* __restrict__ leafid, int32_t* __restrict__ vid,
                                                 int32_t* __restrict__ counts) {
  const Geom g = *geom;
  const int n = 1 << depth;
  for (int j = blockIdx.x * kTB + threadIdx.x; j < P; j += gridDim.x * kTB) {
    int ix, iy;
    {
#pragma clang fp contract(off)
      const double wl = g.side / (double)n;
      ix = clamp_i((int)floor((X[j] - g.x0) / wl), 0, n - 1);
      iy = clamp_i((int)floor((X[P + j] - g.y0) / wl), 0, n - 1);
    }
    const int leaf = ix * n + iy;
    leafid[j] = leaf;
    atomicAdd(counts + leaf, 1);
    // vesicle of j: the last v with off[v] <= j
    int lo = 0, hi = M;  // off[lo] <= j < off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= j) lo = mid; else hi = mid;
    }
    vid[j] = lo;
  }
}

// Exclusive scans of the leaf occupancies (starts) and of their chunks of 2^cshift targets (wave starts).
__global__ __launch_bounds__(1024) void k_tc_scan(const int32_t* __restrict__ counts, int nleaf,
                                                  int32_t* __restrict__ starts, int32_t* __restrict__ wstart,
                                                  int cshift) {
  __shared__ int32_t sa[1024];
  __shared__ int32_t sb[1024];
  const int t = threadIdx.x;
  const int seg = (nleaf + 1023) / 1024;
  const int b0 = min(t * seg, nleaf), b1 = min(b0 + seg, nleaf);
  int32_t a = 0, b = 0;
  for (int i = b0; i < b1; ++i) {
    a += counts[i];
    b += (counts[i] + (1 << cshift) - 1) >> cshift;
  }
  const int32_t own_a = a, own_b = b;
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the segment sums (Hillis-Steele)
    const int32_t xa = t >= d ? sa[t - d] : 0, xb = t >= d ? sb[t - d] : 0;
    __syncthreads();
    sa[t] += xa;
    sb[t] += xb;
    __syncthreads();
  }
  if (t == 1023) {
    starts[nleaf] = sa[t];
    wstart[nleaf] = sb[t];
  }
  a = sa[t] - own_a;  // exclusive
  b = sb[t] - own_b;
  for (int i = b0; i < b1; ++i) {
    starts[i] = a;
    wstart[i] = b;
    a += counts[i];
    b += (counts[i] + (1 << cshift) - 1) >> cshift;
  }
}

__global__ __launch_bounds__(kTB) void k_tc_scatter(const int32_t* __restrict__ leafid, int P,
                                                    const int32_t* __restrict__ starts, int32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ perm) {
  for (int j = blockIdx.x * kTB + threadIdx.x; j < P; j += gridDim.x * kTB) {
    const int leaf = leafid[j];
    perm[starts[leaf] + atomicAdd(cursor + leaf, 1)] = j;
  }
}

// Points of each leaf in ascending index order (deterministic sums).  One wavefront per leaf: the
// keys (distinct point indices) go to LDS and each is written at its rank, the number of smaller
// keys in the leaf.
__global__ __launch_bounds__(64) void k_tc_sort(const int32_t* __restrict__ starts, int32_t* __restrict__ perm) {
  __shared__ int32_t key[kSortMax];
  const int leaf = blockIdx.x;
  const int s0 = starts[leaf], n = starts[leaf + 1] - s0;
  if (n < 2 || n > kSortMax) return;
  for (int a = threadIdx.x; a < n; a += 64) key[a] = perm[s0 + a];
  __syncthreads();
  for (int a = threadIdx.x; a < n; a += 64) {
    const int32_t k = key[a];
    int rank = 0;
    for (int b = 0; b < n; ++b) rank += key[b] < k;
    perm[s0 + rank] = k;
  }
}

// ---------------------------------------------------------------- moments
//
// Moments of a box: 4 rows of (p + 1) complex numbers: row 0 M_k[F], row 1 M_k[conj F] (divided by k
// for k >= 1 once all translations are done), row 2 M_k[conj(zeta) F], row 3 M_k[F] / k (filled last).

__device__ __forceinline__ double2 cpow_int(double2 z, int k) {
  double2 r = make_double2(1.0, 0.0);
  double2 b = z;
  while (k > 0) {
    if (k & 1) r = cmul(r, b);
    b = cmul(b, b);
    k >>= 1;
  }
  return r;
}

// One wavefront per leaf, lane k = order.  The leaf's points pass through LDS 32 at a time, each with
// its powers zeta^0 .. zeta^p (by repeated multiplication), so lane k reads zeta^k instead of forming it.
constexpr int kP2MChunk = 32;

__global__ __launch_bounds__(64) void k_tc_p2m(const double* __restrict__ X, const double* __restrict__ f,
                                               const double* __restrict__ w, int P, const int32_t* __restrict__ perm,
                                               const int32_t* __restrict__ starts, const Geom* __restrict__ geom,
                                               int depth, int p, double2* __restrict__ mom,
                                               int32_t* __restrict__ bcount) {
  __shared__ double2 pw[kP2MChunk][kMaxOrder + 1];
  __shared__ double2 Fs[kP2MChunk], Zc[kP2MChunk];
  const int leaf = blockIdx.x;
  const int k = threadIdx.x;
  const int n = 1 << depth;
  const int s0 = starts[leaf], s1 = starts[leaf + 1];
  if (k == 0) bcount[leaf] = s1 - s0;
  const double2 c = box_center(*geom, n, leaf / n, leaf % n);
  double2 m0 = make_double2(0.0, 0.0), m1 = m0, m2 = m0;
  for (int c0 = s0; c0 < s1; c0 += kP2MChunk) {
    const int cnt = min(kP2MChunk, s1 - c0);
    __syncthreads();  // the previous chunk is done
    if (k < cnt) {
      const int j = perm[c0 + k];
      const double2 zeta = make_double2(X[j] - c.x, X[P + j] - c.y);
      Fs[k] = make_double2(w[j] * f[j], w[j] * f[P + j]);
      Zc[k] = make_double2(zeta.x, -zeta.y);
      double2 z = make_double2(1.0, 0.0);
      for (int m = 0; m <= p; ++m) {
        pw[k][m] = z;
        z = cmul(z, zeta);
      }
    }
    __syncthreads();
    if (k <= p) {
      for (int q = 0; q < cnt; ++q) {
        const double2 F = Fs[q], zk = pw[q][k];
        const double2 Fz = cmul(F, zk);
        m0.x += Fz.x;
        m0.y += Fz.y;
        const double2 Fcz = cmul(make_double2(F.x, -F.y), zk);
        m1.x += Fcz.x;
        m1.y += Fcz.y;
        const double2 Pz = cmul(Zc[q], Fz);
        m2.x += Pz.x;
        m2.y += Pz.y;
      }
    }
  }
  if (k > p) return;
  double2* mb = mom + (size_t)leaf * 4 * (p + 1);
  mb[k] = m0;
  mb[(p + 1) + k] = m1;
  mb[2 * (p + 1) + k] = m2;
}

// 1 / (m + 1), m = 0..kMaxOrder: the binomial recurrence below multiplies instead of dividing.
__constant__ double kRecip[kMaxOrder + 1] = {
    1.0 / 1,  1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,  1.0 / 6,  1.0 / 7,  1.0 / 8,  1.0 / 9,  1.0 / 10,
    1.0 / 11, 1.0 / 12, 1.0 / 13, 1.0 / 14, 1.0 / 15, 1.0 / 16, 1.0 / 17, 1.0 / 18, 1.0 / 19, 1.0 / 20,
    1.0 / 21, 1.0 / 22, 1.0 / 23, 1.0 / 24, 1.0 / 25, 1.0 / 26, 1.0 / 27, 1.0 / 28, 1.0 / 29, 1.0 / 30,
    1.0 / 31, 1.0 / 32, 1.0 / 33, 1.0 / 34, 1.0 / 35, 1.0 / 36, 1.0 / 37, 1.0 / 38, 1.0 / 39, 1.0 / 40,
    1.0 / 41, 1.0 / 42, 1.0 / 43, 1.0 / 44, 1.0 / 45, 1.0 / 46, 1.0 / 47, 1.0 / 48, 1.0 / 49};

// Parent moments at a level with n boxes per side from the children one level down:
// M'_k = sum_children sum_{m <= k} C(k, m) d^(k-m) M_m, d = child centre - parent centre; the
// conj(zeta) F row gains conj(d) times the translated F row.  One workgroup per parent box, wave q
// translates child q (lane k = order, the child's three rows staged in LDS), and the four results
// are added in child order.  C(k, m + 1) = C(k, m) (k - m) / (m + 1) is an integer below 2^53 for
// k <= 48, so rounding the product with the reciprocal to the nearest integer gives it exactly.
__global__ __launch_bounds__(256) void k_tc_m2m(const Geom* __restrict__ geom, int n, int p,
                                                const double2* __restrict__ child, const int32_t* __restrict__ ccount,
                                                double2* __restrict__ parent, int32_t* __restrict__ pcount) {
  __shared__ double2 cm[4][3 * (kMaxOrder + 1)];
  const int box = blockIdx.x;
  const int q = threadIdx.x >> 6, k = threadIdx.x & 63;
  const int bx = box / n, by = box % n;
  const int stride = 4 * (p + 1);
  const double wc = geom->side / (double)(2 * n);  // child width
  const int cb = (2 * bx + (q >> 1)) * (2 * n) + (2 * by + (q & 1));
  const int cnt = ccount[cb];
  if (cnt > 0)
    for (int e = k; e < 3 * (p + 1); e += 64) cm[q][e] = child[(size_t)cb * stride + e];
  __syncthreads();
  double2 t0 = make_double2(0.0, 0.0), t1 = t0, t2 = t0;
  if (cnt > 0 && k <= p) {
    const double2 d = make_double2(((double)(q >> 1) - 0.5) * wc, ((double)(q & 1) - 0.5) * wc);
    const double dd = d.x * d.x + d.y * d.y;
    const double2 dinv = make_double2(d.x / dd, -d.y / dd);
    double binom = 1.0;           // C(k, m)
    double2 dp = cpow_int(d, k);  // d^(k - m)
    for (int m = 0; m <= k; ++m) {
      const double2 coef = make_double2(binom * dp.x, binom * dp.y);
      t0 = cfma(coef, cm[q][m], t0);
      t1 = cfma(coef, cm[q][(p + 1) + m], t1);
      t2 = cfma(coef, cm[q][2 * (p + 1) + m], t2);
      binom = rint(binom * (double)(k - m) * kRecip[m]);
      dp = cmul(dp, dinv);
    }
    const double2 extra = cmul(make_double2(d.x, -d.y), t0);
    t2.x += extra.x;
    t2.y += extra.y;
  }
  __syncthreads();  // every wave is done reading its child
  if (k <= p) {     // each wave's row of LDS now holds its three results
    cm[q][k] = t0;
    cm[q][(p + 1) + k] = t1;
    cm[q][2 * (p + 1) + k] = t2;
  }
  __syncthreads();
  if (q == 0) {
    int tot = 0;
    for (int c = 0; c < 4; ++c) tot += ccount[(2 * bx + (c >> 1)) * (2 * n) + (2 * by + (c & 1))];
    if (k == 0) pcount[box] = tot;
    if (k <= p) {
      double2 s0 = cm[0][k], s1 = cm[0][(p + 1) + k], s2 = cm[0][2 * (p + 1) + k];
      for (int c = 1; c < 4; ++c) {
        s0.x += cm[c][k].x;
        s0.y += cm[c][k].y;
        s1.x += cm[c][(p + 1) + k].x;
        s1.y += cm[c][(p + 1) + k].y;
        s2.x += cm[c][2 * (p + 1) + k].x;
        s2.y += cm[c][2 * (p + 1) + k].y;
      }
      double2* pm = parent + (size_t)box * stride;
      pm[k] = s0;
      pm[(p + 1) + k] = s1;
      pm[2 * (p + 1) + k] = s2;
    }
  }
}

// After all translations: row 3 = M_k[F] / k (k >= 1) for the log series of F, and row 2 = D_k, the
// coefficients of t^(k+1) in (S[conj F] - Psi) / 2: D_k = (M_{k+1}[conj F] / (k+1) - M_k[conj(zeta) F]) / 2,
// D_p = -M_p[conj(zeta) F] / 2.  The evaluation then needs three series instead of four.
__global__ __launch_bounds__(kTB) void k_tc_finalize(double2* __restrict__ mom, size_t nbox, int p) {
  const size_t stride = 4 * (size_t)(p + 1);
  for (size_t e = (size_t)blockIdx.x * kTB + threadIdx.x; e < nbox * (p + 1); e += (size_t)gridDim.x * kTB) {
    const size_t box = e / (p + 1);
    const int k = (int)(e - box * (p + 1));
    double2* mb = mom + box * stride;
    const double2 a = mb[k];
    mb[3 * (p + 1) + k] = k == 0 ? make_double2(0.0, 0.0) : make_double2(a.x / (double)k, a.y / (double)k);
    const double2 psi = mb[2 * (p + 1) + k];
    double2 d = make_double2(-0.5 * psi.x, -0.5 * psi.y);
    if (k < p) {
      const double2 b = mb[(p + 1) + k + 1];
      const double ik = 0.5 / (double)(k + 1);
      d.x = fma(b.x, ik, d.x);
      d.y = fma(b.y, ik, d.y);
    }
    mb[2 * (p + 1) + k] = d;
  }
}

// ---------------------------------------------------------------- fast multipole translations
//
// Local expansion of a box T (centre c_T, zeta = z - c_T): three rows of (p + 1) complex Taylor
// coefficients A, B, C such that the far field (times 4 pi mu) of everything in the interaction lists
// of T and of its ancestors is
//     u = -A(zeta)/2 - conj(B(zeta))/2 + zeta conj(C(zeta))/2.
// A source box S, d = c_S - c_T, t = 1/d, enters through its multipole series in powers of (z - c_S)^-1:
//   A: log sum of F,  lambda = M_0[F],       a_m = -M_m[F]/m                      (m = 1..p);
//   C: Cauchy sum Phi,                       a_m = M_{m-1}[F]                     (m = 1..p+1);
//   B: log sum of conj F plus Psi,  lambda = M_0[conj F],  a_m = -M_m[conj F]/m + M_{m-1}[conj(zeta) F],
//      plus conj(d) times C (the term that re-centres conj(zeta_j) from c_S to c_T).
// With (z - c_S)^-m = (-t)^m sum_l C(m + l - 1, l) t^l zeta^l and log(z - c_S) = log(-d) - sum_{l>=1} t^l zeta^l / l,
// the coefficient of zeta^l is t^l (sum_m C(m + l - 1, l) (-t)^m a_m - lambda / l), and for l = 0
// lambda ln|d| + sum_m (-t)^m a_m: the imaginary part of log(-d) cancels between A and conj(B) because
// M_0[conj F] = conj(M_0[F]).  Each source box's constant M_0[F]/2 goes into A_0 as -M_0[F].
// A child inherits its parent's expansion re-centred by e = c_child - c_parent:
//   X_l += sum_{m>=l} C(m, l) e^(m-l) X_m  for A, B, C, and B additionally -conj(e) times the shifted C.

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// T[m][l] = C(m + l - 1, l) for m = 0..p+1, l = 0..p (row 0: 1, 0, 0, ...), row stride p + 1, by Pascal's
// rule T[m][l] = T[m-1][l] + T[m][l-1] along anti-diagonals: sums of integers, exact below 2^53.  The
// same table holds C(m, l) = T[m - l + 1][l].  One wavefront, lane = l.
__global__ __launch_bounds__(64) void k_fmm_binom(int p, double* __restrict__ tab) {
  __shared__ double prev[64];
  const int l = threadIdx.x;
  double v = l == 0 ? 1.0 : 0.0;  // T[0][l]
  if (l <= p) tab[l] = v;
  for (int s = 1; s <= 2 * p + 1; ++s) {
    prev[l] = v;  // this lane's latest entry, T[s - 1 - l][l]
    __syncthreads();
    const int m = s - l;
    if (l <= p && m >= 1 && m <= p + 1) {
      v += l > 0 ? prev[l - 1] : 0.0;  // + T[m][l - 1], written by lane l - 1 one step earlier
      tab[m * (p + 1) + l] = v;
    }
    __syncthreads();
  }
}

constexpr int kM2LWaves = 4;  // waves per target box; source box k of the list goes to wave k mod 4

// Dynamic LDS of k_fmm_m2l: the binomial table, then per wave three staging vectors (A, Phi and B
// series) of max(G (p + 2), 64) complex numbers, G = floor(64 / (p + 1)).
__host__ __device__ inline int m2l_groups(int p) { return 64 / (p + 1); }
__host__ __device__ inline int m2l_stage(int p) {
  const int g = m2l_groups(p) * (p + 2);
  return g > 64 ? g : 64;
}
__host__ __device__ inline int m2l_table_doubles(int p) { return ((p + 2) * (p + 1) + 1) / 2 * 2; }  // 16-byte multiple
inline size_t m2l_lds_bytes(int p) {
  return sizeof(double) * (size_t)m2l_table_doubles(p) + sizeof(double2) * (size_t)kM2LWaves * 3 * m2l_stage(p);
}

// Interaction-list contributions to the local expansion of every non-empty box of levels 2..depth (one
// launch for all levels, one workgroup per target box).  Lanes form G groups of p + 1; each group takes
// one source box at a time: lane j of the group scales a_(j+1) by (-t)^(j+1) into LDS, then forms
// sum_m C(m + j - 1, j) (-t)^m a_m for order l = j of the three series.  The partial expansions of all
// groups and waves are added in a fixed order at the end.
__global__ __launch_bounds__(64 * kM2LWaves) void k_fmm_m2l(const Geom* __restrict__ geom, int depth, int p,
                                                           const double2* __restrict__ mom,
                                                           const int32_t* __restrict__ bcount,
                                                           const double* __restrict__ tab, double2* __restrict__ loc) {
  extern __shared__ double smem[];
  const size_t box = blockIdx.x;
  if (bcount[box] == 0) return;  // the whole workgroup
  const int np = p + 1;
  const int G = m2l_groups(p), stage = m2l_stage(p);
  double* T = smem;
  double2* st = reinterpret_cast<double2*>(smem + m2l_table_doubles(p));
  const int nt = (p + 2) * np;
  for (int e = threadIdx.x; e < nt; e += 64 * kM2LWaves) T[e] = tab[e];
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / np, j = lane - g * np;  // group, order within the group; g >= G: idle lane
  double2* sA = st + (size_t)wv * 3 * stage;
  double2* sP = sA + stage;
  double2* sQ = sP + stage;
  int l = 2;
  while (l < depth && box >= level_box_base(l + 1)) ++l;
  const int n = 1 << l;
  const size_t base = level_box_base(l);
  const int b = (int)(box - base);
  const int bx = b / n, by = b - (b / n) * n;
  const double wl = geom->side / (double)n;
  const int stride = 4 * np;
  const double inv_m = 1.0 / (double)(j + 1);          // 1/m, m = j + 1
  const double inv_l = j > 0 ? 1.0 / (double)j : 0.0;  // 1/l, l = j
  double2 accA = make_double2(0.0, 0.0), accB = accA, accC = accA;
  int cand = 0, k = 0;  // next candidate of the 6 x 6 block; non-empty sources seen so far
  for (;;) {
    // this wave's next batch: up to G non-empty sources, group g takes the g-th
    int nb = 0, msx = 0, msy = 0;
    while (nb < G && cand < 36) {
      const int sx = 2 * (bx >> 1) + cand / 6 - 2, sy = 2 * (by >> 1) + cand % 6 - 2;
      ++cand;
      if (sx < 0 || sx >= n || sy < 0 || sy >= n) continue;
      if (abs(sx - bx) <= 1 && abs(sy - by) <= 1) continue;
      if (bcount[base + (size_t)sx * n + sy] == 0) continue;
      if ((k++ & (kM2LWaves - 1)) != wv) continue;
      if (g == nb) {
        msx = sx;
        msy = sy;
      }
      ++nb;
    }
    if (nb == 0) break;
    const bool on = g < nb;
    const double2 d = make_double2((double)(msx - bx) * wl, (double)(msy - by) * wl);
    const double dd = on ? d.x * d.x + d.y * d.y : 1.0;
    const double rdd = recip(dd);
    const double2 mt = make_double2(-d.x * rdd, d.y * rdd);  // -t = -1/d
    const double2 pl = cpow_int(mt, j);                      // (-t)^l, l = j
    const double2 pm = cmul(pl, mt);                         // (-t)^m, m = j + 1
    const double2* ms = mom + (base + (size_t)msx * n + msy) * stride;
    double2* qA = sA + g * (p + 2);
    double2* qP = sP + g * (p + 2);
    double2* qQ = sQ + g * (p + 2);
    if (on) {
      double2 aA = make_double2(0.0, 0.0), aQ = ms[2 * np + j];
      if (j < p) {
        const double2 Fm = ms[j + 1], Cm = ms[np + j + 1];
        aA = make_double2(-Fm.x * inv_m, -Fm.y * inv_m);
        aQ.x = fma(-Cm.x, inv_m, aQ.x);
        aQ.y = fma(-Cm.y, inv_m, aQ.y);
      }
      qA[j + 1] = cmul(aA, pm);
      qP[j + 1] = cmul(ms[j], pm);
      qQ[j + 1] = cmul(aQ, pm);
    }
    wave_sync();
    if (on) {
      double2 xA = make_double2(0.0, 0.0), xP = xA, xQ = xA;
#pragma unroll 2
      for (int m = 1; m <= np; ++m) {
        const double cb = T[m * np + j];
        const double2 va = qA[m], vp = qP[m], vq = qQ[m];
        xA.x = fma(cb, va.x, xA.x);
        xA.y = fma(cb, va.y, xA.y);
        xP.x = fma(cb, vp.x, xP.x);
        xP.y = fma(cb, vp.y, xP.y);
        xQ.x = fma(cb, vq.x, xQ.x);
        xQ.y = fma(cb, vq.y, xQ.y);
      }
      const double2 lamA = ms[0], lamQ = ms[np];
      double2 bA, bP, bQ;
      if (j == 0) {
        const double lnd = 0.5 * log_pos(dd);
        bA = make_double2(fma(lamA.x, lnd, xA.x) - lamA.x, fma(lamA.y, lnd, xA.y) - lamA.y);  // - M_0[F]: constant
        bP = xP;
        bQ = make_double2(fma(lamQ.x, lnd, xQ.x), fma(lamQ.y, lnd, xQ.y));
      } else {
        const double2 tl = (j & 1) ? make_double2(-pl.x, -pl.y) : pl;  // t^l = (-1)^l (-t)^l
        bA = cmul(tl, make_double2(fma(-lamA.x, inv_l, xA.x), fma(-lamA.y, inv_l, xA.y)));
        bP = cmul(tl, xP);
        bQ = cmul(tl, make_double2(fma(-lamQ.x, inv_l, xQ.x), fma(-lamQ.y, inv_l, xQ.y)));
      }
      accA.x += bA.x;
      accA.y += bA.y;
      accC.x += bP.x;
      accC.y += bP.y;
      const double2 sh = cmul(make_double2(d.x, -d.y), bP);  // + conj(d) Phi
      accB.x += bQ.x + sh.x;
      accB.y += bQ.y + sh.y;
    }
    wave_sync();  // the staging is rewritten by the next batch
  }
  // partial expansions of every group of every wave, added in a fixed order
  __syncthreads();
  sA[lane] = accA;
  sP[lane] = accB;
  sQ[lane] = accC;
  __syncthreads();
  if (threadIdx.x < np) {
    const int t = threadIdx.x;
    double2 rA = make_double2(0.0, 0.0), rB = rA, rC = rA;
    for (int w = 0; w < kM2LWaves; ++w) {
      const double2* r = st + (size_t)w * 3 * stage;
      for (int q = 0; q < G; ++q) {
        const double2 a = r[q * np + t], bb = r[stage + q * np + t], c = r[2 * stage + q * np + t];
        rA.x += a.x;
        rA.y += a.y;
        rB.x += bb.x;
        rB.y += bb.y;
        rC.x += c.x;
        rC.y += c.y;
      }
    }
    double2* lb = loc + box * 3 * np;
    lb[t] = rA;
    lb[np + t] = rB;
    lb[2 * np + t] = rC;
  }
}

// Adds the parent's local expansion, re-centred, to every non-empty box of level l (n = 2^l per side).
// One wavefront per box, lane = order, the parent's three rows staged in LDS.
__global__ __launch_bounds__(64) void k_fmm_l2l(const Geom* __restrict__ geom, int n, int p,
                                               const int32_t* __restrict__ bcount, const double* __restrict__ tab,
                                               const double2* __restrict__ parent, double2* __restrict__ child) {
  __shared__ double2 pl[3 * (kMaxOrder + 1)];
  const int box = blockIdx.x;
  if (bcount[box] == 0) return;
  const int k = threadIdx.x;
  const int bx = box / n, by = box % n;
  const int rows = 3 * (p + 1);
  const size_t pbox = (size_t)(bx >> 1) * (n >> 1) + (by >> 1);
  for (int e = k; e < rows; e += 64) pl[e] = parent[pbox * rows + e];
  __syncthreads();
  if (k > p) return;
  const double wl = geom->side / (double)n;
  const double2 e = make_double2(((double)(bx & 1) - 0.5) * wl, ((double)(by & 1) - 0.5) * wl);
  double2 sA = make_double2(0.0, 0.0), sB = sA, sC = sA;
  double2 ej = make_double2(1.0, 0.0);  // e^j
  for (int j = 0; j <= p - k; ++j) {
    const double cb = tab[(j + 1) * (p + 1) + k];  // C(k + j, k)
    const double2 ce = make_double2(cb * ej.x, cb * ej.y);
    sA = cfma(ce, pl[k + j], sA);
    sB = cfma(ce, pl[(p + 1) + k + j], sB);
    sC = cfma(ce, pl[2 * (p + 1) + k + j], sC);
    ej = cmul(ej, e);
  }
  const double2 sh = cmul(make_double2(e.x, -e.y), sC);
  double2* cb_ = child + (size_t)box * rows;
  double2 v = cb_[k];
  cb_[k] = make_double2(v.x + sA.x, v.y + sA.y);
  v = cb_[(p + 1) + k];
  cb_[(p + 1) + k] = make_double2(v.x + sB.x - sh.x, v.y + sB.y - sh.y);
  v = cb_[2 * (p + 1) + k];
  cb_[2 * (p + 1) + k] = make_double2(v.x + sC.x, v.y + sC.y);
}

// ---------------------------------------------------------------- evaluation

__device__ __forceinline__ void direct_term(double zx, double zy, double sx, double sy, double Fx, double Fy,
                                            const double2* __restrict__ ltab, double& ux, double& uy) {
  const double rx = zx - sx, ry = zy - sy;
  const double q = rx * rx + ry * ry;
  const double lg = -0.5 * log_reduced(q, ltab);
  const double s = (rx * Fx + ry * Fy) * recip(q);
  ux = fma(lg, Fx, fma(s, rx, ux));
  uy = fma(lg, Fy, fma(s, ry, uy));
}

// Walk over the interaction lists of a leaf (ix, iy), levels 2..depth, candidates in a fixed order;
// the same in every lane.  Yields the non-empty boxes (level, sx, sy).
struct ListWalk {
  int l, a, b;
};

__device__ __forceinline__ bool next_box(ListWalk& s, int depth, int ix, int iy, const int32_t* __restrict__ bcount,
                                         int& lo, int& sxo, int& syo) {
  while (s.l <= depth) {
    const int l = s.l, nl = 1 << l;
    const int bx = ix >> (depth - l), by = iy >> (depth - l);
    const int sx = 2 * (bx >> 1) + s.a, sy = 2 * (by >> 1) + s.b;
    if (++s.b > 3) {
      s.b = -2;
      if (++s.a > 3) {
        s.a = -2;
        ++s.l;
      }
    }
    if (sx < 0 || sx >= nl || sy < 0 || sy >= nl) continue;
    if (abs(sx - bx) <= 1 && abs(sy - by) <= 1) continue;
    if (bcount[level_box_base(l) + (size_t)sx * nl + sy] == 0) continue;
    lo = l;
    sxo = sx;
    syo = sy;
    return true;
  }
  return false;
}

// Targets per wavefront of the evaluation: the treecode's far part costs the same per wavefront whatever
// its target count, so it takes 64; the fast multipole method's is a short polynomial per target and
// takes 32, twice the wavefronts to hide the direct part's latencies.
template <bool kFmm> constexpr int eval_chunk_shift() { return kFmm ? 5 : 6; }

// One wavefront per (leaf, chunk of kChunk of its points); every lane one target.  The far part is the
// treecode's walk over the interaction lists (kFmm false: mom holds the finalised moments) or the leaf's
// local expansion (kFmm true: loc holds it); the direct part is shared.
template <bool kFmm>
__global__ __launch_bounds__(64) void k_tc_eval(const double* __restrict__ X, const double* __restrict__ f,
                                                const double* __restrict__ w, int P, const int32_t* __restrict__ vid,
                                                const int32_t* __restrict__ perm, const int32_t* __restrict__ starts,
                                                const int32_t* __restrict__ wstart, const Geom* __restrict__ geom,
                                                int depth, int p, const double2* __restrict__ mom,
                                                const double2* __restrict__ loc, const int32_t* __restrict__ bcount,
                                                double scale, double* __restrict__ out) {
  constexpr int kChunk = 1 << eval_chunk_shift<kFmm>();
  const int n = 1 << depth;
  const int nleaf = n * n;
  const int item = blockIdx.x;
  if (item >= wstart[nleaf]) return;
  int lo = 0, hi = nleaf;  // wstart[lo] <= item < wstart[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (wstart[mid] <= item) lo = mid; else hi = mid;
  }
  const int leaf = lo;
  const int s0 = starts[leaf], s1 = starts[leaf + 1];
  // A chunk of at most 32 targets splits the wave into S = 64 / K lane groups (K = the target count
  // rounded up to a power of two): lane = g K + t takes target t, and in the direct part every S-th
  // source from g on; the groups' direct sums are added at the end.  The far part is the same in every
  // group.
  const int lane = threadIdx.x;
  const int base = s0 + (item - wstart[leaf]) * kChunk;
  const int tcnt = min(kChunk, s1 - base);
  int K = 1;
  while (K < tcnt) K <<= 1;
  const int S = 64 / K;
  const int slot = base + (lane & (K - 1));
  const bool active = slot < s1;
  const int i = active ? perm[slot] : perm[s0];
  const double zx = X[i], zy = X[P + i];
  const int vi = vid[i];
  const int ix = leaf / n, iy = leaf % n;
  const Geom g = *geom;
  const int stride = 4 * (p + 1);
  double ux = 0.0, uy = 0.0;
  // per-wavefront staging: the moments of one box, then chunks of 64 direct sources
  __shared__ double2 cf[4 * 64];  // 4 (p + 1) <= 196 entries used; padded for whole-wave copies
  __shared__ double sx_[64], sy_[64], sfx[64], sfy[64];
  __shared__ int32_t sv[64];
  __shared__ double2 ltab[kLogTab];
  ltab[threadIdx.x] = log_tab_entry(threadIdx.x);  // read after the first barrier below

  if constexpr (kFmm) {
    // the leaf's local expansion: u += -A(zeta)/2 - conj(B(zeta))/2 + zeta conj(C(zeta))/2
    if (depth >= 2) {
      const double2* lb = loc + (level_box_base(depth) + (size_t)leaf) * 3 * (p + 1);
      cf[threadIdx.x] = lb[threadIdx.x];  // 3 x 64 >= 3 (kMaxOrder + 1); the array has 192 spare entries
      cf[threadIdx.x + 64] = lb[threadIdx.x + 64];
      cf[threadIdx.x + 128] = lb[threadIdx.x + 128];
      __syncthreads();
      const double2 c = box_center(g, n, ix, iy);
      const double2 zt = make_double2(zx - c.x, zy - c.y);
      double2 A = cf[p], B = cf[2 * p + 1], C = cf[3 * p + 2];
      for (int k = p - 1; k >= 0; --k) {
        A = cfma(A, zt, cf[k]);
        B = cfma(B, zt, cf[(p + 1) + k]);
        C = cfma(C, zt, cf[2 * (p + 1) + k]);
      }
      ux += -0.5 * A.x - 0.5 * B.x + 0.5 * (zt.x * C.x + zt.y * C.y);
      uy += -0.5 * A.y + 0.5 * B.y + 0.5 * (zt.y * C.x - zt.x * C.y);
    }
  } else {
    // expansions of the interaction lists: box by box, the next box's moments loaded into registers
    // while the current one is evaluated from LDS
    // four entries per lane: 4 x 64 >= 4 (kMaxOrder + 1); the moment array has 256 spare entries
    double2 n0 = make_double2(0.0, 0.0), n1 = n0, n2 = n0, n3 = n0;
    ListWalk it = {2, -2, -2};
    int nl_ = 0, nsx = 0, nsy = 0;
    bool have = next_box(it, depth, ix, iy, bcount, nl_, nsx, nsy);
    if (have) {
      const double2* mb = mom + (level_box_base(nl_) + (size_t)nsx * (1 << nl_) + nsy) * stride;
      n0 = mb[threadIdx.x];
      n1 = mb[threadIdx.x + 64];
      n2 = mb[threadIdx.x + 128];
      n3 = mb[threadIdx.x + 192];
    }
    while (have) {
      __syncthreads();  // the previous box is done with cf
      cf[threadIdx.x] = n0;
      cf[threadIdx.x + 64] = n1;
      cf[threadIdx.x + 128] = n2;
      cf[threadIdx.x + 192] = n3;
      __syncthreads();
      const int l = nl_, sx = nsx, sy = nsy;
      have = next_box(it, depth, ix, iy, bcount, nl_, nsx, nsy);
      if (have) {
        const double2* mb = mom + (level_box_base(nl_) + (size_t)nsx * (1 << nl_) + nsy) * stride;
        n0 = mb[threadIdx.x];
        n1 = mb[threadIdx.x + 64];
        n2 = mb[threadIdx.x + 128];
        n3 = mb[threadIdx.x + 192];
      }
      {
        const double2 c = box_center(g, 1 << l, sx, sy);
        const double2 wv = make_double2(zx - c.x, zy - c.y);
        const double w2 = wv.x * wv.x + wv.y * wv.y;
        const double2 t = make_double2(wv.x / w2, -wv.y / w2);
        // Three series in t, highest order first:
        //   S = sum_{k>=1} M_k[F] / k t^k,  D = sum_k D_k t^(k+1),  E = sum_k M_k[F] t^k;
        // the box contributes S/2 + M_0/2 - M_0 ln|w| + conj(D) + (w / conj w) conj(E) / 2.
        double2 aS = make_double2(0.0, 0.0), aD = aS, aE = aS;
        for (int k = p; k >= 1; --k) {
          aS = cfma(aS, t, cf[3 * (p + 1) + k]);
          aD = cfma(aD, t, cf[2 * (p + 1) + k]);
          aE = cfma(aE, t, cf[k]);
        }
        const double2 M0 = cf[0];
        aD = cfma(aD, t, cf[2 * (p + 1)]);
        aE = cfma(aE, t, M0);
        aS = cmul(aS, t);
        aD = cmul(aD, t);
        const double lnw = 0.5 * log_pos(w2);
        const double2 rot = make_double2((wv.x * wv.x - wv.y * wv.y) / w2, 2.0 * wv.x * wv.y / w2);  // w / conj w
        const double2 pe = cmul(rot, make_double2(aE.x, -aE.y));
        ux += 0.5 * aS.x + 0.5 * M0.x - M0.x * lnw + aD.x + 0.5 * pe.x;
        uy += 0.5 * aS.y + 0.5 * M0.y - M0.y * lnw - aD.y + 0.5 * pe.y;
      }
    }
  }
  // 3 x 3 leaves directly, own vesicle skipped
  double dx = 0.0, dy = 0.0;
  for (int jx = max(ix - 1, 0); jx <= min(ix + 1, n - 1); ++jx)
    for (int jy = max(iy - 1, 0); jy <= min(iy + 1, n - 1); ++jy) {
      const int nl = jx * n + jy;
      const int e0 = starts[nl], e1 = starts[nl + 1];
      for (int c0 = e0; c0 < e1; c0 += 64) {
        const int cnt = min(64, e1 - c0);
        __syncthreads();  // the previous chunk is done
        if ((int)threadIdx.x < cnt) {
          const int j = perm[c0 + threadIdx.x];
          sx_[threadIdx.x] = X[j];
          sy_[threadIdx.x] = X[P + j];
          sfx[threadIdx.x] = w[j] * f[j];
          sfy[threadIdx.x] = w[j] * f[P + j];
          sv[threadIdx.x] = vid[j];
        }
        __syncthreads();
        // the next source's data is read while the current one is evaluated
        int q = lane / K;
        const int qq = q < cnt ? q : 0;
        double nx = sx_[qq], ny = sy_[qq], nfx = sfx[qq], nfy = sfy[qq];
        int nv = sv[qq];
        for (; q < cnt; q += S) {
          const double cx = nx, cy = ny, cfx = nfx, cfy = nfy;
          const int cv = nv;
          const int qn = q + S < cnt ? q + S : q;
          nx = sx_[qn];
          ny = sy_[qn];
          nfx = sfx[qn];
          nfy = sfy[qn];
          nv = sv[qn];
          if (cv != vi) direct_term(zx, zy, cx, cy, cfx, cfy, ltab, dx, dy);
        }
      }
    }
  for (int o = K; o < 64; o <<= 1) {  // groups' direct sums, pairwise in a fixed order
    dx += __shfl_down(dx, o);
    dy += __shfl_down(dy, o);
  }
  if (active && lane < K) {
    out[i] = (ux + dx) * scale;
    out[P + i] = (uy + dy) * scale;
  }
}

// Own-vesicle sources outside the 3 x 3 leaves around a target were in the expansions: their direct terms
// are subtracted from the finished velocity.  One wavefront per vesicle, targets 64 at a time, the
// vesicle's points (coordinates, weighted force, leaf) staged in LDS in chunks.  Few sources of a chunk
// are far from a given target, and different ones for different lanes: each lane first lists its far
// sources, then the wave evaluates the lists side by side (as many steps as the longest list).
constexpr int kOwnChunk = 128;

__global__ __launch_bounds__(64) void k_tc_own(const double* __restrict__ X, const double* __restrict__ f,
                                               const double* __restrict__ w, int P, const int32_t* __restrict__ off,
                                               const int32_t* __restrict__ leafid, int depth, double scale,
                                               double* __restrict__ out) {
  __shared__ double sx_[kOwnChunk], sy_[kOwnChunk], sfx[kOwnChunk], sfy[kOwnChunk];
  __shared__ int32_t sl[kOwnChunk];
  __shared__ uint8_t lst[kOwnChunk][64];  // lst[k][lane]: the k-th far source of the lane's target
  __shared__ double2 ltab[kLogTab];
  const int v = blockIdx.x;
  const int v0 = clamp_i(off[v], 0, P), v1 = max(v0, clamp_i(off[v + 1], 0, P));  // offsets never trusted
  if (v1 - v0 < 2) return;
  const int lane = threadIdx.x;
  ltab[lane] = log_tab_entry(lane);  // read after the first barrier below
  const int mask = (1 << depth) - 1;
  for (int t0 = v0; t0 < v1; t0 += 64) {
    const int i = t0 + lane;
    const bool act = i < v1;
    const int ii = act ? i : v0;
    const double zx = X[ii], zy = X[P + ii];
    const int li = leafid[ii];
    const int ix = li >> depth, iy = li & mask;
    double ux = 0.0, uy = 0.0;
    for (int c0 = v0; c0 < v1; c0 += kOwnChunk) {
      const int cnt = min(kOwnChunk, v1 - c0);
      __syncthreads();  // the previous chunk is done
      for (int q = lane; q < cnt; q += 64) {
        const int j = c0 + q;
        sx_[q] = X[j];
        sy_[q] = X[P + j];
        sfx[q] = w[j] * f[j];
        sfy[q] = w[j] * f[P + j];
        sl[q] = leafid[j];
      }
      __syncthreads();
      int nf = 0;
      for (int q = 0; q < cnt; ++q) {
        const int lj = sl[q];
        if (abs((lj >> depth) - ix) > 1 || abs((lj & mask) - iy) > 1) lst[nf++][lane] = (uint8_t)q;  // far
      }
      int most = nf;  // longest list of the wave
      for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
      for (int k = 0; k < most; ++k) {
        if (k < nf) {
          const int q = lst[k][lane];
          direct_term(zx, zy, sx_[q], sy_[q], sfx[q], sfy[q], ltab, ux, uy);
        }
      }
    }
    if (act) {
      out[i] -= ux * scale;
      out[P + i] -= uy * scale;
    }
  }
}

}  // namespace

// Workspace layout shared by the size queries and the launchers; the fast multipole method adds the
// local expansions (3 rows per box) and the binomial table.
struct TreeLayout {
  size_t geom, part, leafid, vid, perm, counts, cursor, starts, wstart, bcount, mom, loc, tab, total;
};

static size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

static TreeLayout tree_layout(int P, int depth, int p, bool fmm) {
  TreeLayout t;
  const size_t nleaf = (size_t)1 << (2 * depth);
  size_t boxes = 0;
  for (int l = 2; l <= depth; ++l) boxes += (size_t)1 << (2 * l);
  const size_t moms = boxes * 4 * (size_t)(p + 1);
  size_t o = 0;
  t.geom = o;       o += align_up(sizeof(double) * 4);
  t.part = o;       o += align_up(sizeof(double) * 4 * kBBoxBlocks);
  t.leafid = o;     o += align_up(sizeof(int32_t) * (size_t)P);
  t.vid = o;        o += align_up(sizeof(int32_t) * (size_t)P);
  t.perm = o;       o += align_up(sizeof(int32_t) * (size_t)P);
  t.counts = o;     o += align_up(sizeof(int32_t) * nleaf);
  t.cursor = o;     o += align_up(sizeof(int32_t) * nleaf);
  t.starts = o;     o += align_up(sizeof(int32_t) * (nleaf + 1));
  t.wstart = o;     o += align_up(sizeof(int32_t) * (nleaf + 1));
  t.bcount = o;     o += align_up(sizeof(int32_t) * (boxes > 0 ? boxes : 1));
  t.mom = o;        o += align_up(sizeof(double2) * (moms + 256));  // 256 spare entries: whole-wave copies
  t.loc = o;
  t.tab = o;
  if (fmm) {
    t.loc = o;      o += align_up(sizeof(double2) * (boxes * 3 * (size_t)(p + 1) + 192));  // 192 spare: as above
    t.tab = o;      o += align_up(sizeof(double) * (size_t)(p + 2) * (p + 1));
  }
  t.total = o;
  return t;
}

size_t treecode_workspace_bytes(int P, int depth, int p) { return tree_layout(P, depth, p, false).total; }
size_t fmm_workspace_bytes(int P, int depth, int p) { return tree_layout(P, depth, p, true).total; }

namespace {

struct TreeRun {
  Geom* geom;
  double* part;
  int32_t *leafid, *vid, *perm, *counts, *cursor, *starts, *wstart, *bcount;
  double2 *mom, *loc;
  double* tab;
  Levels lv;       // first box and first moment entry of every level
  size_t nbox;     // boxes of levels 2..depth
};

TreeRun tree_run(void* ws, const TreeLayout& t, int depth, int p) {
  char* base = static_cast<char*>(ws);
  TreeRun r;
  r.geom = reinterpret_cast<Geom*>(base + t.geom);
  r.part = reinterpret_cast<double*>(base + t.part);
  r.leafid = reinterpret_cast<int32_t*>(base + t.leafid);
  r.vid = reinterpret_cast<int32_t*>(base + t.vid);
  r.perm = reinterpret_cast<int32_t*>(base + t.perm);
  r.counts = reinterpret_cast<int32_t*>(base + t.counts);
  r.cursor = reinterpret_cast<int32_t*>(base + t.cursor);
  r.starts = reinterpret_cast<int32_t*>(base + t.starts);
  r.wstart = reinterpret_cast<int32_t*>(base + t.wstart);
  r.bcount = reinterpret_cast<int32_t*>(base + t.bcount);
  r.mom = reinterpret_cast<double2*>(base + t.mom);
  r.loc = reinterpret_cast<double2*>(base + t.loc);
  r.tab = reinterpret_cast<double*>(base + t.tab);
  r.lv = {};
  size_t acc = 0;
  for (int l = 2; l <= depth; ++l) {  // boxes of level l start at box index sum_{m = 2}^{l-1} 4^m
    r.lv.box[l] = acc;
    r.lv.mom[l] = acc * 4 * (size_t)(p + 1);
    acc += (size_t)1 << (2 * l);
  }
  r.nbox = acc;
  return r;
}

// Tree over the points (root square, leaves, leaf order) and the moments of every box of levels
// 2..depth (leaves from the points, coarser levels by translation).
void launch_upward(const double* X, const double* f, const double* w, const int32_t* off, int M, int P, int p,
                   int depth, int cshift, const TreeRun& r, hipStream_t st) {
  const int nleaf = 1 << (2 * depth);
  const int pb = (P + kTB - 1) / kTB < 4096 ? (P + kTB - 1) / kTB : 4096;
  const int bb = (P + kTB - 1) / kTB < kBBoxBlocks ? (P + kTB - 1) / kTB : kBBoxBlocks;
  hipLaunchKernelGGL(k_tc_bbox_partial, dim3(bb), dim3(kTB), 0, st, X, P, r.part);
  hipLaunchKernelGGL(k_tc_bbox_final, dim3(1), dim3(64), 0, st, r.part, bb, r.geom);
  const int zb = (nleaf + kTB - 1) / kTB < 4096 ? (nleaf + kTB - 1) / kTB : 4096;
  hipLaunchKernelGGL(k_tc_zero, dim3(zb), dim3(kTB), 0, st, r.counts, nleaf);
  hipLaunchKernelGGL(k_tc_zero, dim3(zb), dim3(kTB), 0, st, r.cursor, nleaf);
  hipLaunchKernelGGL(k_tc_leaf, dim3(pb), dim3(kTB), 0, st, X, P, r.geom, depth, off, M, r.leafid, r.vid, r.counts);
  hipLaunchKernelGGL(k_tc_scan, dim3(1), dim3(1024), 0, st, r.counts, nleaf, r.starts, r.wstart, cshift);
  hipLaunchKernelGGL(k_tc_scatter, dim3(pb), dim3(kTB), 0, st, r.leafid, P, r.starts, r.cursor, r.perm);
  hipLaunchKernelGGL(k_tc_sort, dim3(nleaf), dim3(64), 0, st, r.starts, r.perm);
  if (depth < 2) return;
  hipLaunchKernelGGL(k_tc_p2m, dim3(nleaf), dim3(64), 0, st, X, f, w, P, r.perm, r.starts, r.geom, depth, p,
                     r.mom + r.lv.mom[depth], r.bcount + r.lv.box[depth]);
  for (int l = depth - 1; l >= 2; --l) {
    const int n = 1 << l;
    hipLaunchKernelGGL(k_tc_m2m, dim3(n * n), dim3(256), 0, st, r.geom, n, p, r.mom + r.lv.mom[l + 1],
                       r.bcount + r.lv.box[l + 1], r.mom + r.lv.mom[l], r.bcount + r.lv.box[l]);
  }
}

template <bool kFmm>
void launch_eval(const double* X, const double* f, const double* w, const int32_t* off, int M, int P, int p, int depth,
                 double scale, const TreeRun& r, double* out, hipStream_t st) {
  const int nleaf = 1 << (2 * depth);
  constexpr int kChunk = 1 << eval_chunk_shift<kFmm>();
  const int items = nleaf + (P + kChunk - 1) / kChunk;  // bound on sum over leaves of ceil(count / kChunk)
  hipLaunchKernelGGL(k_tc_eval<kFmm>, dim3(items), dim3(64), 0, st, X, f, w, P, r.vid, r.perm, r.starts, r.wstart,
                     r.geom, depth, p, r.mom, r.loc, r.bcount, scale, out);
  // without expansions (depth < 2) every own-vesicle source is in the 3 x 3 leaves
  if (depth >= 2)
    hipLaunchKernelGGL(k_tc_own, dim3(M), dim3(64), 0, st, X, f, w, P, off, r.leafid, depth, scale, out);
}

}  // namespace

// Everything is built on the device; the launches need no host copy and no synchronisation.
hipError_t launch_treecode(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                           double scale, int p, int depth, double* out, void* ws, void* stream) {
  if (P == 0) return hipSuccess;
  if (depth < 0 || depth > kMaxDepth || p < 1 || p > kMaxOrder) return hipErrorInvalidValue;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const TreeRun r = tree_run(ws, tree_layout(P, depth, p, false), depth, p);
  launch_upward(X, f, w, off, M, P, p, depth, eval_chunk_shift<false>(), r, st);
  if (depth >= 2) {
    const size_t work = r.nbox * (p + 1);
    const int gb = (int)((work + kTB - 1) / kTB < 4096 ? (work + kTB - 1) / kTB : 4096);
    hipLaunchKernelGGL(k_tc_finalize, dim3(gb), dim3(kTB), 0, st, r.mom, r.nbox, p);
  }
  launch_eval<false>(X, f, w, off, M, P, p, depth, scale, r, out, st);
  return hipGetLastError();
}

hipError_t launch_fmm(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                      double scale, int p, int depth, double* out, void* ws, void* stream) {
  if (P == 0) return hipSuccess;
  if (depth < 0 || depth > kMaxDepth || p < 1 || p > kMaxOrder) return hipErrorInvalidValue;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const TreeRun r = tree_run(ws, tree_layout(P, depth, p, true), depth, p);
  launch_upward(X, f, w, off, M, P, p, depth, eval_chunk_shift<true>(), r, st);
  if (depth >= 2) {
    hipLaunchKernelGGL(k_fmm_binom, dim3(1), dim3(64), 0, st, p, r.tab);
    hipLaunchKernelGGL(k_fmm_m2l, dim3((unsigned)r.nbox), dim3(64 * kM2LWaves), m2l_lds_bytes(p), st, r.geom, depth, p,
                       r.mom, r.bcount, r.tab, r.loc);
    const size_t rows = 3 * (size_t)(p + 1);
    for (int l = 3; l <= depth; ++l) {
      const int n = 1 << l;
      hipLaunchKernelGGL(k_fmm_l2l, dim3(n * n), dim3(64), 0, st, r.geom, n, p, r.bcount + r.lv.box[l], r.tab,
                         r.loc + r.lv.box[l - 1] * rows, r.loc + r.lv.box[l] * rows);
    }
  }
  launch_eval<true>(X, f, w, off, M, P, p, depth, scale, r, out, st);
  return hipGetLastError();
}

}  // namespace vesnet
