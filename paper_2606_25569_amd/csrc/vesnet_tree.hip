// Tree far fields on gfx950: the far-field sum of eq. (single_layer) at O(P log P) (treecode) and O(P)
// (fast multipole method) cost.  The paper evaluates the sum directly, names the fast multipole method as
// the route to O(M) cost and leaves fast summation out of scope (Section 4.1); both methods here are fast,
// approximate alternatives with their own accuracy contract (order p of the expansions).
//
// With complex numbers z = x + i y, F_j = w_j (f_x + i f_y)_j, u = u_x + i u_y, each Stokeslet term is
//   -F_j ln|z - z_j| + F_j / 2 + (z - z_j) conj(F_j / (z - z_j)) / 2,
// so a box of sources with centre c, zeta_j = z_j - c, acts at w = z - c, t = 1/w, through the
// power moments M_k[q] = sum_j q_j zeta_j^k of three charge sets (F, conj F, conj(zeta) F):
//   -M_0[F] ln|w| + 1/2 sum_{k=1}^p (M_k[F] t^k + conj(M_k[conj F] t^k)) / k + M_0[F] / 2
//   + (w conj(Phi) - conj(Psi)) / 2,   Phi = sum_{k=0}^p M_k[F] t^(k+1),  Psi = sum_k M_k[conj(zeta) F] t^(k+1).
//
// Tree: a uniform quadtree of depth L over the bounding square of the points.  Leaf moments come from
// the points (k_tc_p2m), coarser ones by exact binomial translation (k_tc_m2m).  A target takes, at each
// level l = 2..L, the interaction list of its level-l ancestor (children of the parent's 3 x 3
// neighbourhood not adjacent to the ancestor) through the expansions, and the 3 x 3 leaves around its own
// directly, skipping its own vesicle; own-vesicle sources outside those leaves, which the expansions
// included, are subtracted exactly (k_tc_own).  Everything is FP64.
//
// Treecode: every target evaluates the series of every box of its lists (k_tc_eval<false>); the
// evaluation merges the conj-F log series and Psi into one series D, and writes w conj(Phi) as
// (w / conj w) conj(E), E = sum_k M_k[F] t^k: three Horner chains per box.
// Fast multipole method: each box's series becomes a Taylor polynomial of degree p about the centre of
// every box whose list holds it (k_fmm_m2l, on the matrix cores), the polynomials of a leaf's ancestors
// are re-centred onto the leaf (k_fmm_l2l), and every target evaluates its leaf's polynomial
// (k_tc_eval<true>).
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

// Box centre at a level with n boxes per side (contraction off: the same bits as the plain formula).
__device__ __forceinline__ double2 box_center(const Geom& g, int n, int bx, int by) {
#pragma clang fp contract(off)
  const double wl = g.side / (double)n;
  return make_double2(g.x0 + ((double)bx + 0.5) * wl, g.y0 + ((double)by + 0.5) * wl);
}

// First box of level l >= 2 when levels 2, 3, ... are stored one after another: sum_{m=2}^{l-1} 4^m.
__device__ __forceinline__ size_t level_box_base(int l) { return (((size_t)1 << (2 * l)) - 16) / 3; }

// ---------------------------------------------------------------- tree construction

// Binomial table T[m][l] = C(m + l - 1, l) for m = 1..p+1, l = 0..p, zero elsewhere, over rows m = 0..kTabM-1
// and columns l = 0..63 (stride kTabL): the whole zero-padded range the matrix-core tiles read.  Row 0 holds
// 1, 0, 0, ... while it is built (the start of the recurrence) and zeros once done.  Pascal's rule
// T[m][l] = T[m-1][l] + T[m][l-1] runs along anti-diagonals: sums of integers, exact below 2^53.  The same
// table holds C(m, l) = T[m - l + 1][l].  Run by the one wavefront (lane = l) of the bounding-box kernel.
constexpr int kTabL = 64;
constexpr int kTabM = 4 * ((kMaxOrder + 1 + 3) / 4) + 1;  // m up to 4 ceil((p + 1) / 4)

__device__ void build_binomials(int p, double* __restrict__ tab) {
  __shared__ double prev[64];
  const int l = threadIdx.x;
  for (int m = 0; m < kTabM; ++m) tab[m * kTabL + l] = 0.0;
  double v = l == 0 ? 1.0 : 0.0;  // T[0][l]
  for (int s = 1; s <= 2 * p + 1; ++s) {
    prev[l] = v;  // this lane's latest entry, T[s - 1 - l][l]
    __syncthreads();
    const int m = s - l;
    if (l <= p && m >= 1 && m <= p + 1) {
      v += l > 0 ? prev[l - 1] : 0.0;  // + T[m][l - 1], written by lane l - 1 one step earlier
      tab[m * kTabL + l] = v;
    }
    __syncthreads();
  }
}


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

// Also builds the binomial table of the fast multipole method when tab is not null.
__global__ __launch_bounds__(64) void k_tc_bbox_final(const double* __restrict__ part, int nparts,
                                                      Geom* __restrict__ geom, int p, double* __restrict__ tab) {
  if (tab != nullptr) build_binomials(p, tab);
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

__global__ __launch_bounds__(kTB) void k_tc_zero(int32_t* __restrict__ a, int32_t* __restrict__ b, int n) {
  for (int i = blockIdx.x * kTB + threadIdx.x; i < n; i += gridDim.x * kTB) {
    a[i] = 0;
    b[i] = 0;
  }
}

// Within a wavefront, the lanes whose key equals the first pending lane's form a group: one atomic adds the
// group's size to counter[key] and returns the group's base, and each lane takes base + its rank among the
// group's lanes.  Consecutive points mostly share a leaf, so a wavefront needs a few atomics instead of 64.
__device__ __forceinline__ int wave_group_add(bool ok, int key, int32_t* __restrict__ counter) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(ok);
  int pos = 0;
  while (todo) {
    const int leader = __ffsll(todo) - 1;
    const int lk = __shfl(key, leader);
    const unsigned long long same = __ballot(ok && key == lk);  // not yet placed: earlier groups had other keys
    int base = 0;
    if (lane == leader) base = atomicAdd(counter + lk, __popcll(same));
    base = __shfl(base, leader);
    if ((same >> lane) & 1ull) pos = base + __popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  return pos;
}

// Leaf of every point and leaf occupancy.
__global__ __launch_bounds__(kTB) void k_tc_leaf(const double* __restrict__ X, int P, const Geom* __restrict__ geom,
                                                 int depth, int32_t* __restrict__ leafid, int32_t* __restrict__ counts) {
  const Geom g = *geom;
  const int n = 1 << depth;
  for (int j0 = blockIdx.x * kTB; j0 < P; j0 += gridDim.x * kTB) {  // the same trip count for every lane
    const int j = j0 + (int)threadIdx.x;
    const bool ok = j < P;
    int leaf = 0;
    if (ok) {
      int ix, iy;
      {
#pragma clang fp contract(off)
        const double wl = g.side / (double)n;
        ix = clamp_i((int)floor((X[j] - g.x0) / wl), 0, n - 1);
        iy = clamp_i((int)floor((X[P + j] - g.y0) / wl), 0, n - 1);
      }
      leaf = ix * n + iy;
      leafid[j] = leaf;
    }
    wave_group_add(ok, leaf, counts);
  }
}

// Vesicle id of every point: one workgroup per vesicle writes its index over its range (offsets clamped).
// With h2 given, also the squared near-field radius h_v^2 of every vesicle, h_v = sum_j w_j / N_v (the
// mean arclength spacing, summed in a fixed order), and bit 1 of *flag when h_v exceeds the leaf width
// (then a point within h_v of a target may lie outside its 3 x 3 leaves).
__global__ __launch_bounds__(kTB) void k_tc_vid(const int32_t* __restrict__ off, int P, int32_t* __restrict__ vid,
                                                const double* __restrict__ w, const Geom* __restrict__ geom,
                                                int depth, double* __restrict__ h2, int32_t* __restrict__ flag) {
  const int v = blockIdx.x;
  const int v0 = clamp_i(off[v], 0, P), v1 = max(v0, clamp_i(off[v + 1], 0, P));
  for (int j = v0 + (int)threadIdx.x; j < v1; j += kTB) vid[j] = v;
  if (h2 == nullptr) return;
  __shared__ double red[kTB];
  double a = 0.0;
  for (int j = v0 + (int)threadIdx.x; j < v1; j += kTB) a += w[j];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = kTB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double h = v1 > v0 ? red[0] / (double)(v1 - v0) : 0.0;
    h2[v] = h * h;
    if (h > geom->side / (double)(1 << depth)) atomicOr(flag, 2);
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
  for (int j0 = blockIdx.x * kTB; j0 < P; j0 += gridDim.x * kTB) {  // the same trip count for every lane
    const int j = j0 + (int)threadIdx.x;
    const bool ok = j < P;
    const int leaf = ok ? leafid[j] : 0;
    const int pos = wave_group_add(ok, leaf, cursor);
    if (ok) perm[starts[leaf] + pos] = j;
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
  extern __shared__ double2 p2m_lds[];  // powers [kP2MChunk][p + 1], then F and conj(zeta) of the chunk
  double2* Fs = p2m_lds + kP2MChunk * (p + 1);
  double2* Zc = Fs + kP2MChunk;
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
        p2m_lds[k * (p + 1) + m] = z;
        z = cmul(z, zeta);
      }
    }
    __syncthreads();
    if (k <= p) {
      for (int q = 0; q < cnt; ++q) {
        const double2 F = Fs[q], zk = p2m_lds[q * (p + 1) + k];
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

typedef double double4v __attribute__((ext_vector_type(4)));

// Dynamic LDS of k_fmm_m2l for order p, KS = ceil((p + 1) / 4) steps of four m and RT = ceil((p + 1) / 16)
// tiles of 16 orders: the binomial tile T[m - 1][l] (4 KS x 16 RT), the source list, the scaled coefficients
// X[v][m - 1][s] of a batch (3 series x 4 KS x 8 sources, complex; also the final exchange of 3 x 64 sums),
// the powers (-t_s)^l (8 sources x 4 KS, complex), and per source lambda_A, lambda_B (complex) and ln|d|.
// (Splitting a box's batches over several waves, or taking one series at a time to save registers, both
// measured slower: the first is limited by LDS occupancy, the second loses independent MFMA chains.)
constexpr int kM2LBatch = 8;  // source boxes per batch: 8 complex columns fill one 16-column tile
__host__ __device__ inline int m2l_ksteps(int p) { return (p + 1 + 3) / 4; }
__host__ __device__ inline int m2l_rtiles(int p) { return (p + 1 + 15) / 16; }
__host__ __device__ inline int m2l_tsize(int p) { return (4 * m2l_ksteps(p) * 16 * m2l_rtiles(p) + 1) / 2; }  // double2
__host__ __device__ inline int m2l_xsize(int p) {  // in double2
  const int mm = 4 * m2l_ksteps(p);
  return 3 * mm * kM2LBatch > 3 * 64 ? 3 * mm * kM2LBatch : 3 * 64;
}
inline size_t m2l_lds_bytes(int p) {
  const int mm = 4 * m2l_ksteps(p);
  return sizeof(double2) * ((size_t)m2l_tsize(p) + 36 + m2l_xsize(p) + (size_t)kM2LBatch * mm + 2 * kM2LBatch +
                            kM2LBatch / 2);
}

// Interaction-list contributions to the local expansion of every non-empty box of levels 2..depth (one
// launch for all levels, one wavefront per target box), on the matrix cores.  For a source box s at
// d_s = c_s - c_T, t_s = 1/d_s, and each series v (A, Phi, and B with the conj(d) Phi term folded in,
// conj(d_s) being a constant factor per source), the coefficient of zeta^l is
//   t_s^l (sum_{m=1}^{p+1} C(m + l - 1, l) X_v[m][s] - lambda_v / l),   X_v[m][s] = a_v(m) (-t_s)^m,
// (l = 0: sum_m X_v[m][s] + lambda_v ln|d_s|).  The sums over m are the product D = X^T T with
// X^T: (16 columns: 8 sources x re, im) x m and T: m x l, in 16 x 16 x 4 FP64 steps: the columns of a tile
// are one series of eight sources, source c's real part in row (c mod 4) + 8 (c / 4) and its imaginary part
// four rows below, so that every lane (l = lane mod 16, q = lane / 16) receives both parts of sources q and
// q + 4 for its order l and scales them itself.  Sources go eight at a time, in the fixed candidate order;
// at the end the sums of the four lanes of every order are added in q order.  RT = ceil((p + 1) / 16).
template <int RT>
__global__ __launch_bounds__(64) void k_fmm_m2l(const Geom* __restrict__ geom, int depth, int p,
                                                           const double2* __restrict__ mom,
                                                           const int32_t* __restrict__ bcount,
                                                           const double* __restrict__ tab, double2* __restrict__ loc) {
  extern __shared__ double2 sm[];
  const size_t box = blockIdx.x;
  if (bcount[box] == 0) return;
  const int lane = threadIdx.x;
  const int np = p + 1;
  const int KS = m2l_ksteps(p), MM = 4 * KS;
  constexpr int TL = 16 * RT;                                    // orders per table row
  double* Tt = reinterpret_cast<double*>(sm);                    // [MM][TL]
  int32_t* lst = reinterpret_cast<int32_t*>(sm + m2l_tsize(p));  // [36][2]: source box coordinates
  double2* X = sm + m2l_tsize(p) + 36;                           // [3][MM][8]
  double2* pw = X + m2l_xsize(p);                                // [8][MM]: (-t_s)^l
  double2* lam = pw + kM2LBatch * MM;                            // [8][2]: lambda_A, lambda_B
  double* lnd = reinterpret_cast<double*>(lam + 2 * kM2LBatch);  // [8]
  for (int e = threadIdx.x; e < MM * TL; e += blockDim.x) Tt[e] = tab[(size_t)(e / TL + 1) * kTabL + e % TL];
  int l2 = 2;
  while (l2 < depth && box >= level_box_base(l2 + 1)) ++l2;
  const int n = 1 << l2;
  const size_t base = level_box_base(l2);
  const int b = (int)(box - base);
  const int bx = b / n, by = b - (b / n) * n;
  const double wl = geom->side / (double)n;
  const int stride = 4 * np;
  // the interaction list's non-empty boxes in the fixed candidate order: lane c examines candidate c
  int ns;
  {
    const int sx = 2 * (bx >> 1) + lane / 6 - 2, sy = 2 * (by >> 1) + lane % 6 - 2;
    bool ok = lane < 36 && sx >= 0 && sx < n && sy >= 0 && sy < n && (abs(sx - bx) > 1 || abs(sy - by) > 1);
    if (ok) ok = bcount[base + (size_t)sx * n + sy] != 0;
    const unsigned long long mask = __ballot(ok);
    ns = __popcll(mask);
    if (ok) {
      const int rank = __popcll(mask & ((1ull << lane) - 1ull));
      lst[2 * rank] = sx;
      lst[2 * rank + 1] = sy;
    }
  }
  wave_sync();  // table and list ready
  const int j = lane & 15, q = lane >> 4;  // result lanes: order j (+ 16 rt), sources q and q + 4
  const int ai = lane & 15, ak = lane >> 4;  // operand lanes: column / order ai, step row ak
  const int acol = (ai & 3) + 4 * (ai >> 3), apart = (ai >> 2) & 1;  // column ai: source acol, re or im
  double2 acc[3][RT];
  double inv_l[RT];  // 1/l for the lane's orders l = j + 16 rt (0 for l = 0 or beyond p)
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int l = j + 16 * rt;
    inv_l[rt] = (l >= 1 && l <= p) ? kRecip[l - 1] : 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v) acc[v][rt] = make_double2(0.0, 0.0);
  }
  for (int b0 = 0; b0 < ns; b0 += kM2LBatch) {
    const int nb = min(kM2LBatch, ns - b0);
    // scaling: lane takes source s = lane mod 8 and m = 1 + lane / 8, then every eighth m
    {
      const int s = lane & 7;
      const bool valid = s < nb;
      const int sx = valid ? lst[2 * (b0 + s)] : bx + 2, sy = valid ? lst[2 * (b0 + s) + 1] : by;
      const double2 d = make_double2((double)(sx - bx) * wl, (double)(sy - by) * wl);
      const double dd = d.x * d.x + d.y * d.y;
      const double rdd = recip(dd);
      const double2 mt = make_double2(-d.x * rdd, d.y * rdd);  // -t
      const double2* ms = mom + (base + (size_t)(valid ? sx : 0) * n + (valid ? sy : 0)) * stride;
      const int m0 = 1 + (lane >> 3);
      // every moment load first, at indices clamped into the rows (values outside are discarded), so
      // that they are all in flight together
      double2 Fm1[2 * RT], Fm[2 * RT], Cm[2 * RT], Pm1[2 * RT];
#pragma unroll
      for (int it = 0; it < 2 * RT; ++it) {
        const int mc = min(m0 + 8 * it, np), mp = min(mc, p);
        Fm1[it] = ms[mc - 1];
        Fm[it] = ms[mp];
        Cm[it] = ms[np + mp];
        Pm1[it] = ms[2 * np + mc - 1];
      }
      const double2 t2 = cmul(mt, mt), t4 = cmul(t2, t2), step = cmul(t4, t4);  // (-t)^2, ^4, ^8
      const int e0 = m0 - 1;                                                     // 0..7
      double2 pl = (e0 & 1) ? mt : make_double2(1.0, 0.0);                      // (-t)^(m-1)
      if (e0 & 2) pl = cmul(pl, t2);
      if (e0 & 4) pl = cmul(pl, t4);
#pragma unroll
      for (int it = 0; it < 2 * RT; ++it) {  // m = m0 + 8 it; MM <= 16 RT
        const int m = m0 + 8 * it;
        if (m <= MM) {
          pw[s * MM + (m - 1)] = valid ? pl : make_double2(0.0, 0.0);
          const bool use = valid && m <= np;
          const double2 pm = cmul(pl, mt);  // (-t)^m
          const double im = m <= p ? kRecip[m - 1] : 0.0;  // the A and conj-F series stop at order p
          const double2 aA = make_double2(-Fm[it].x * im, -Fm[it].y * im);
          const double2 aQ = make_double2(fma(-Cm[it].x, im, Pm1[it].x), fma(-Cm[it].y, im, Pm1[it].y));
          const double2 sh = cmul(make_double2(d.x, -d.y), Fm1[it]);  // conj(d) Phi folded into B
          const double2 zero = make_double2(0.0, 0.0);
          X[(0 * MM + (m - 1)) * kM2LBatch + s] = use ? cmul(aA, pm) : zero;
          X[(1 * MM + (m - 1)) * kM2LBatch + s] = use ? cmul(Fm1[it], pm) : zero;
          X[(2 * MM + (m - 1)) * kM2LBatch + s] = use ? cmul(make_double2(aQ.x + sh.x, aQ.y + sh.y), pm) : zero;
        }
        pl = cmul(pl, step);
      }
      if (lane < kM2LBatch) {  // lane = s, m0 = 1: the first load of the loop above read M_0[F]
        const double2 lq = ms[np];
        lam[2 * s] = valid ? Fm1[0] : make_double2(0.0, 0.0);
        lam[2 * s + 1] = valid ? lq : make_double2(0.0, 0.0);
        lnd[s] = valid ? 0.5 * log_pos(dd) : 0.0;
      }
    }
    wave_sync();
    // D[v][rt] = sum over m of the batch's columns times the binomials, three series and RT order tiles
    // issued together at every step
    const double* Xd = reinterpret_cast<const double*>(X);
    double4v D[3][RT];
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) D[v][rt] = (double4v){0.0, 0.0, 0.0, 0.0};
    for (int ks = 0; ks < KS; ++ks) {
      const int mi = 4 * ks + ak;  // m - 1
      double av[3], bv[RT];
#pragma unroll
      for (int v = 0; v < 3; ++v) av[v] = Xd[2 * ((v * MM + mi) * kM2LBatch + acol) + apart];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) bv[rt] = Tt[mi * TL + ai + 16 * rt];
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) D[v][rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[v], bv[rt], D[v][rt], 0, 0, 0);
    }
    // scale: every lane owns orders l = j + 16 rt and sources q, q + 4; t^l, 1/l, the lambdas and ln|d|
    // are shared by the three series
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int s = q + 4 * h;
      const double2 lamA = lam[2 * s], lamB = lam[2 * s + 1];
      const double ld = lnd[s];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int l = j + 16 * rt;
        if (l > p) continue;
        const double2 pwl = pw[s * MM + l];
        const double sg = (l & 1) ? -1.0 : 1.0;  // t^l = (-1)^l (-t)^l
        const double2 tl = l == 0 ? make_double2(1.0, 0.0) : make_double2(sg * pwl.x, sg * pwl.y);
        const double il = inv_l[rt];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          const double2 y = make_double2(D[v][rt][2 * h], D[v][rt][2 * h + 1]);
          const double2 lv = v == 0 ? lamA : (v == 2 ? lamB : make_double2(0.0, 0.0));
          // l = 0: y + lambda ln|d| (and, for A, the source's constant M_0[F] / 2 as -M_0[F]);
          // l >= 1: t^l (y - lambda / l)
          const double2 c0 = make_double2(fma(lv.x, l == 0 ? ld : -il, y.x), fma(lv.y, l == 0 ? ld : -il, y.y));
          double2 bv2 = cmul(tl, c0);
          if (v == 0 && l == 0) {
            bv2.x -= lv.x;
            bv2.y -= lv.y;
          }
          acc[v][rt].x += bv2.x;
          acc[v][rt].y += bv2.y;
        }
      }
    }
    wave_sync();  // the staging is rewritten by the next batch
  }
  // the sums of the four lanes of every order, added in q order; X is reused for the exchange
  double2* lb = loc + box * 3 * np;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int v = 0; v < 3; ++v) X[v * 64 + lane] = acc[v][rt];
    wave_sync();
    const int l = lane + 16 * rt;
    if (lane < 16 && l <= p) {
      for (int v = 0; v < 3; ++v) {
        double2 r = X[v * 64 + lane];
        for (int qq = 1; qq < 4; ++qq) {
          r.x += X[v * 64 + lane + 16 * qq].x;
          r.y += X[v * 64 + lane + 16 * qq].y;
        }
        lb[(v == 0 ? 0 : (v == 1 ? 2 : 1)) * np + l] = r;  // series A, Phi, B -> rows A, B, C
      }
    }
    wave_sync();
  }
}

// Completes the local expansion of every non-empty leaf: its own interaction-list part plus the part of
// each ancestor (levels 2..depth-1), re-centred from the ancestor's centre straight to the leaf's (the
// re-centring of a polynomial is exact, so one shift per ancestor equals the chain through the levels).
// With e = c_leaf - c_anc: X_k += sum_{m>=k} C(m, k) e^(m-k) X_m for A, B, C, and B also -conj(e) times the
// shifted C.  One wavefront per leaf, all ancestors' rows staged in LDS together; lane = (half h, order k):
// for p + 1 <= 32 the two halves of the wavefront take alternate ancestors and their sums are added at the
// end, otherwise one half does all.  The binomials follow their recurrence (C(48, 24) < 2^53: rounding the
// product with the reciprocal to the nearest integer gives each one exactly).
__global__ __launch_bounds__(64) void k_fmm_l2l(const Geom* __restrict__ geom, int depth, int p,
                                               const int32_t* __restrict__ bcount, double2* __restrict__ loc) {
  extern __shared__ double2 anc[];  // [depth - 2][3 (p + 1)], then 3 x 32 for the halves' exchange
  const int n = 1 << depth;
  const int leaf = blockIdx.x;
  const size_t lbox = level_box_base(depth) + (size_t)leaf;
  if (bcount[lbox] == 0) return;
  const int lane = threadIdx.x;
  const int bx = leaf / n, by = leaf % n;
  const int rows = 3 * (p + 1);
  const double wL = geom->side / (double)n;
  const int nanc = depth - 2;
  for (int e = lane; e < nanc * rows; e += 64) {
    const int l = 2 + e / rows, sh = depth - l;
    const size_t abox = level_box_base(l) + (size_t)(bx >> sh) * (1 << l) + (by >> sh);
    anc[e] = loc[abox * rows + e % rows];
  }
  __syncthreads();
  const bool split = p + 1 <= 32;
  const int h = split ? lane >> 5 : 0, k = split ? lane & 31 : lane;
  const int hstep = split ? 2 : 1;
  double2 sA = make_double2(0.0, 0.0), sB = sA, sC = sA;
  if (k <= p && (split || lane <= p)) {
    for (int a = h; a < nanc; a += hstep) {
      const int l = 2 + a, sh = depth - l;
      const int ax = bx >> sh, ay = by >> sh;
      const double2* pl = anc + a * rows;
      // leaf centre - ancestor centre = ((b + 1/2) - (a + 1/2) 2^sh) wL per coordinate: exact before the product
      const double2 e = make_double2(((double)bx + 0.5 - ((double)ax + 0.5) * (double)(1 << sh)) * wL,
                                     ((double)by + 0.5 - ((double)ay + 0.5) * (double)(1 << sh)) * wL);
      double2 tA = make_double2(0.0, 0.0), tB = tA, tC = tA;
      double2 ej = make_double2(1.0, 0.0);  // e^j
      double cb = 1.0;                      // C(k + j, k): integers below 2^53, each step exact after rounding
      for (int j = 0; j <= p - k; ++j) {
        const double2 ce = make_double2(cb * ej.x, cb * ej.y);
        tA = cfma(ce, pl[k + j], tA);
        tB = cfma(ce, pl[(p + 1) + k + j], tB);
        tC = cfma(ce, pl[2 * (p + 1) + k + j], tC);
        ej = cmul(ej, e);
        cb = rint(cb * (double)(k + j + 1) * kRecip[j]);  // C(k + j + 1, k) = C(k + j, k) (k + j + 1) / (j + 1)
      }
      const double2 shc = cmul(make_double2(e.x, -e.y), tC);
      sA.x += tA.x;
      sA.y += tA.y;
      sB.x += tB.x - shc.x;
      sB.y += tB.y - shc.y;
      sC.x += tC.x;
      sC.y += tC.y;
    }
  }
  double2* xch = anc + nanc * rows;
  if (split) {  // the second half's sums join the first half's
    if (h == 1) {
      xch[k] = sA;
      xch[32 + k] = sB;
      xch[64 + k] = sC;
    }
    __syncthreads();
    if (h == 1) return;
    if (k <= p) {
      sA.x += xch[k].x;
      sA.y += xch[k].y;
      sB.x += xch[32 + k].x;
      sB.y += xch[32 + k].y;
      sC.x += xch[64 + k].x;
      sC.y += xch[64 + k].y;
    }
  }
  if (k > p) return;
  double2* cb_ = loc + lbox * rows;
  double2 v = cb_[k];
  cb_[k] = make_double2(v.x + sA.x, v.y + sA.y);
  v = cb_[(p + 1) + k];
  cb_[(p + 1) + k] = make_double2(v.x + sB.x, v.y + sB.y);
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
// takes 16, four times the wavefronts to hide the direct part's latencies (at 2000 x 128, order 30:
// 0.58 ms against 0.63 ms at 32 and 0.60 ms at 8 targets).
template <bool kFmm> constexpr int eval_chunk_shift() { return kFmm ? 4 : 6; }

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
// are subtracted from the finished velocity.  One workgroup of two wavefronts per vesicle, targets 128 at a
// time, the vesicle's points (coordinates, weighted force, leaf) staged in LDS in chunks.  Few sources of a
// chunk are far from a given target, and different ones for different lanes: each lane first lists its far
// sources, then each wavefront evaluates its lanes' lists side by side (as many steps as its longest list).
constexpr int kOwnChunk = 128;
constexpr int kOwnThreads = 128;

__global__ __launch_bounds__(kOwnThreads) void k_tc_own(const double* __restrict__ X, const double* __restrict__ f,
                                                        const double* __restrict__ w, int P,
                                                        const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ leafid, int depth, double scale,
                                                        double* __restrict__ out) {
  __shared__ double sx_[kOwnChunk], sy_[kOwnChunk], sfx[kOwnChunk], sfy[kOwnChunk];
  __shared__ int32_t sl[kOwnChunk];
  __shared__ uint8_t lst[kOwnChunk][kOwnThreads];  // lst[k][thread]: the k-th far source of its target
  __shared__ double2 ltab[kLogTab];
  __shared__ int bb[kOwnThreads / 64][4];  // per wavefront: min and max leaf column and row of the chunk
  const int v = blockIdx.x;
  const int v0 = clamp_i(off[v], 0, P), v1 = max(v0, clamp_i(off[v + 1], 0, P));  // offsets never trusted
  if (v1 - v0 < 2) return;
  const int t = threadIdx.x;
  if (t < kLogTab) ltab[t] = log_tab_entry(t);  // read after the first barrier below
  const int mask = (1 << depth) - 1;
  for (int t0 = v0; t0 < v1; t0 += kOwnThreads) {
    const int i = t0 + t;
    const bool act = i < v1;
    const int ii = act ? i : v0;
    const double zx = X[ii], zy = X[P + ii];
    const int li = leafid[ii];
    const int ix = li >> depth, iy = li & mask;
    double ux = 0.0, uy = 0.0;
    for (int c0 = v0; c0 < v1; c0 += kOwnChunk) {
      const int cnt = min(kOwnChunk, v1 - c0);
      __syncthreads();  // the previous chunk is done
      for (int q = t; q < cnt; q += kOwnThreads) {
        const int j = c0 + q;
        sx_[q] = X[j];
        sy_[q] = X[P + j];
        sfx[q] = w[j] * f[j];
        sfy[q] = w[j] * f[P + j];
        sl[q] = leafid[j];
      }
      // the chunk's leaf bounding box: a target whose 3 x 3 leaves cover it has no far source here
      int mnx = 1 << 30, mxx = -1, mny = 1 << 30, mxy = -1;
      for (int q = t; q < cnt; q += kOwnThreads) {
        const int lj = leafid[c0 + q];
        mnx = min(mnx, lj >> depth);
        mxx = max(mxx, lj >> depth);
        mny = min(mny, lj & mask);
        mxy = max(mxy, lj & mask);
      }
      for (int o = 32; o > 0; o >>= 1) {
        mnx = min(mnx, __shfl_xor(mnx, o));
        mxx = max(mxx, __shfl_xor(mxx, o));
        mny = min(mny, __shfl_xor(mny, o));
        mxy = max(mxy, __shfl_xor(mxy, o));
      }
      if ((t & 63) == 0) {
        bb[t >> 6][0] = mnx;
        bb[t >> 6][1] = mxx;
        bb[t >> 6][2] = mny;
        bb[t >> 6][3] = mxy;
      }
      __syncthreads();
      for (int wv = 0; wv < kOwnThreads / 64; ++wv) {
        mnx = min(mnx, bb[wv][0]);
        mxx = max(mxx, bb[wv][1]);
        mny = min(mny, bb[wv][2]);
        mxy = max(mxy, bb[wv][3]);
      }
      const bool covered = ix - 1 <= mnx && mxx <= ix + 1 && iy - 1 <= mny && mxy <= iy + 1;
      int nf = 0;
      if (!covered) {
#pragma unroll 8
        for (int q = 0; q < cnt; ++q) {
          const int lj = sl[q];
          if (abs((lj >> depth) - ix) > 1 || abs((lj & mask) - iy) > 1) lst[nf++][t] = (uint8_t)q;  // far
        }
      }
      int most = nf;  // longest list of the wavefront
      for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
      for (int k = 0; k < most; ++k) {
        if (k < nf) {
          const int q = lst[k][t];
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

// Near-field masking of Algorithm 4 on the fast multipole result: vesicle v (not the target's own) is near
// target i when min_j |x_i - x_j| <= h_v (the rule of the direct masked sum, decided here in FP64 on
// squared distances).  With every h_v at most the leaf width, all such points lie in the 3 x 3 leaves around
// the target's leaf.  One wavefront per (leaf, chunk of targets: the evaluation's work list) stages those
// leaves' points in LDS, up to kNearStage at a time with every lane's loads issued together (a neighbourhood
// of that many points costs three rounds of memory latency); the 64 / chunk lanes t, t + chunk, ... scan
// interleaved points for target t, each keeping the distinct near vesicles it meets (at most kNearMax, else
// bit 0 of *flag), and lane t merges the sets and sorts them ascending.  One atomic per
// wavefront reserves the pair slots.  The whole wavefront then takes the near vesicles of each target in
// turn, 64 points at a time, and subtracts their exact direct sum at x_i from out[i]: the FMM had included v
// through the direct part or the expansions, and the difference leaves the masked far field with the FMM's
// truncation error.  The lane partials are combined by a butterfly, so the result is deterministic.
constexpr int kNearMax = 16;
constexpr int kNearStage = 6 * 64;  // points of the 3 x 3 leaves staged at once (six per lane)

__device__ __forceinline__ void near_insert(int (&nv)[kNearMax], int& nn, bool& over, int v) {
  bool seen = false;
#pragma unroll
  for (int k = 0; k < kNearMax; ++k) seen |= k < nn && nv[k] == v;
  if (seen) return;
  if (nn == kNearMax) {
    over = true;
    return;
  }
#pragma unroll
  for (int k = 0; k < kNearMax; ++k)
    if (k == nn) nv[k] = v;
  ++nn;
}

__global__ __launch_bounds__(64) void k_fmm_near(const double* __restrict__ X, const double* __restrict__ f,
                                                const double* __restrict__ w, int P, int M,
                                                const int32_t* __restrict__ off,
                                                const int32_t* __restrict__ vid, const int32_t* __restrict__ perm,
                                                const int32_t* __restrict__ starts,
                                                const int32_t* __restrict__ wstart, int depth,
                                                const double* __restrict__ h2, double scale, double* __restrict__ out,
                                                int32_t* __restrict__ pairs, int capacity, int32_t* __restrict__ count,
                                                int32_t* __restrict__ flag) {
  constexpr int kChunk = 1 << eval_chunk_shift<true>();
  constexpr int kGroups = 64 / kChunk;  // lanes per target: group g scans every kGroups-th source from g on
  static_assert(kGroups >= 2 && kGroups * kChunk == 64, "a power-of-two chunk of at most 32 targets");
  __shared__ double sx_[kNearStage], sy_[kNearStage], sh[kNearStage];
  __shared__ int32_t sv[kNearStage];
  __shared__ double2 ltab[kLogTab];
  __shared__ int32_t mlist[kGroups - 1][kChunk][kNearMax + 1];
  __shared__ int32_t mcount[kGroups - 1][kChunk];
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
  const int lane = threadIdx.x;
  const int t = lane & (kChunk - 1), grp = lane / kChunk;
  ltab[lane] = log_tab_entry(lane);  // read after the barriers below
  const int s0 = starts[leaf], s1 = starts[leaf + 1];
  const int slot = s0 + (item - wstart[leaf]) * kChunk + t;
  const bool active = slot < s1;
  const int i = active ? perm[slot] : perm[s0];
  const double zx = X[i], zy = X[P + i];
  const int vi = clamp_i(vid[i], 0, M - 1);
  const int ix = leaf / n, iy = leaf % n;
  int nv[kNearMax];
  int nn = 0;
  bool over = false;
  // point ranges of the 3 x 3 leaves (empty outside the grid) and their running offsets
  int lb[9], cum[10];
  cum[0] = 0;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const int jx = ix + a / 3 - 1, jy = iy + a % 3 - 1;
    const bool in = jx >= 0 && jx < n && jy >= 0 && jy < n;
    const int nl = in ? jx * n + jy : 0;
    lb[a] = in ? starts[nl] : 0;
    cum[a + 1] = cum[a] + (in ? starts[nl + 1] - lb[a] : 0);
  }
  const int nsrc = cum[9];
  for (int b0 = 0; b0 < nsrc; b0 += kNearStage) {
    const int cnt = min(kNearStage, nsrc - b0);
    __syncthreads();  // the previous stage is done
    int jj[kNearStage / 64];
#pragma unroll
    for (int u = 0; u < kNearStage / 64; ++u) {
      const int e = b0 + lane + 64 * u;
      int a = 0;
#pragma unroll
      for (int c = 1; c < 9; ++c) a += e >= cum[c] ? 1 : 0;
      jj[u] = e < nsrc ? perm[lb[a] + e - cum[a]] : -1;
    }
    int vv[kNearStage / 64];
#pragma unroll
    for (int u = 0; u < kNearStage / 64; ++u) {
      if (jj[u] >= 0) {
        const int k = lane + 64 * u;
        sx_[k] = X[jj[u]];
        sy_[k] = X[P + jj[u]];
        vv[u] = clamp_i(vid[jj[u]], 0, M - 1);  // ids index the per-vesicle arrays: never trusted
        sv[k] = vv[u];
      }
    }
#pragma unroll
    for (int u = 0; u < kNearStage / 64; ++u)
      if (jj[u] >= 0) sh[lane + 64 * u] = h2[vv[u]];
    __syncthreads();
    if (!active) continue;
#pragma unroll 4
    for (int q = grp; q < cnt; q += kGroups) {
      const double rx = zx - sx_[q], ry = zy - sy_[q];
      const int vq = sv[q];
      if (!(rx * rx + ry * ry > sh[q]) && vq != vi) near_insert(nv, nn, over, vq);
    }
  }
  // merge the other groups' sets into group 0's
  if (grp > 0) {
#pragma unroll
    for (int k = 0; k < kNearMax; ++k)
      if (k < nn) mlist[grp - 1][t][k] = nv[k];
    mcount[grp - 1][t] = nn;
    nn = 0;
  }
  __syncthreads();
  if (grp == 0) {
    for (int g2 = 0; g2 < kGroups - 1; ++g2) {
      const int m = mcount[g2][t];
      for (int k = 0; k < m; ++k) near_insert(nv, nn, over, mlist[g2][t][k]);
    }
    // ascending vesicle order: the subtraction order, and so the result, does not depend on the scan
#pragma unroll
    for (int a = 1; a < kNearMax; ++a)
#pragma unroll
      for (int b = kNearMax - 1; b >= a; --b)
        if (b < nn && nv[b - 1] > nv[b]) {
          const int tmp = nv[b - 1];
          nv[b - 1] = nv[b];
          nv[b] = tmp;
        }
  }
  if (__ballot(over) != 0 && lane == 0) atomicOr(flag, 1);
  int incl = nn;  // inclusive prefix of the pair counts over the wavefront (zero outside group 0)
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  const int total = __shfl(incl, 63);
  if (total == 0) return;
  int base = 0;
  if (lane == 0) base = atomicAdd(count, total);
  base = __shfl(base, 0);
  if (grp == 0) {
    const int b0 = base + incl - nn;
#pragma unroll
    for (int k = 0; k < kNearMax; ++k)
      if (k < nn) {
        if (b0 + k < capacity) {
          pairs[2 * (b0 + k)] = i;
          pairs[2 * (b0 + k) + 1] = nv[k];
        }
        mlist[0][t][k] = nv[k];
      }
    mcount[0][t] = nn;
  }
  __syncthreads();
  unsigned long long todo = __ballot(grp == 0 && nn > 0);
  while (todo) {
    const int tt = __ffsll(todo) - 1;
    todo &= todo - 1;
    const double tx = __shfl(zx, tt), ty = __shfl(zy, tt);
    const int it = __shfl(i, tt);
    const int m = mcount[0][tt];
    double ux = 0.0, uy = 0.0;
    for (int k = 0; k < m; ++k) {
      const int v = mlist[0][tt][k];
      const int v0 = clamp_i(off[v], 0, P), v1 = max(v0, clamp_i(off[v + 1], 0, P));
      for (int j = v0 + lane; j < v1; j += 64)
        direct_term(tx, ty, X[j], X[P + j], w[j] * f[j], w[j] * f[P + j], ltab, ux, uy);
    }
    for (int o = 32; o > 0; o >>= 1) {
      ux += __shfl_xor(ux, o);
      uy += __shfl_xor(uy, o);
    }
    if (lane == 0) {
      out[it] -= ux * scale;
      out[P + it] -= uy * scale;
    }
  }
}

// The list's status: a negative count when the masking could not be completed (see k_fmm_near and k_tc_vid).
__global__ __launch_bounds__(64) void k_fmm_near_status(const int32_t* __restrict__ flag, int32_t* __restrict__ count) {
  if (threadIdx.x != 0) return;
  const int32_t fl = *flag;
  if (fl & 2) *count = -2;
  else if (fl & 1) *count = -1;
}

}  // namespace

// Workspace layout shared by the size queries and the launchers; the fast multipole method adds the
// local expansions (3 rows per box) and the binomial table.
struct TreeLayout {
  size_t geom, part, leafid, vid, perm, counts, cursor, starts, wstart, bcount, mom, loc, tab, h2, flag, total;
};

static size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

static TreeLayout tree_layout(int P, int depth, int p, bool fmm, int near_M = 0) {
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
    t.tab = o;      o += align_up(sizeof(double) * (size_t)kTabM * kTabL);
  }
  t.h2 = o;
  t.flag = o;
  if (near_M > 0) {  // near-field masking: h_v^2 of every vesicle and a status word
    t.h2 = o;       o += align_up(sizeof(double) * (size_t)near_M);
    t.flag = o;     o += align_up(sizeof(int32_t));
  }
  t.total = o;
  return t;
}

size_t treecode_workspace_bytes(int P, int depth, int p) { return tree_layout(P, depth, p, false).total; }
size_t fmm_workspace_bytes(int P, int depth, int p) { return tree_layout(P, depth, p, true).total; }
size_t fmm_near_workspace_bytes(int P, int M, int depth, int p) { return tree_layout(P, depth, p, true, M).total; }

namespace {

struct TreeRun {
  Geom* geom;
  double* part;
  int32_t *leafid, *vid, *perm, *counts, *cursor, *starts, *wstart, *bcount;
  double2 *mom, *loc;
  double* tab;
  double* h2;
  int32_t* flag;
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
  r.h2 = reinterpret_cast<double*>(base + t.h2);
  r.flag = reinterpret_cast<int32_t*>(base + t.flag);
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
                   int depth, int cshift, bool binomials, bool near, const TreeRun& r, hipStream_t st) {
  const int nleaf = 1 << (2 * depth);
  const int pb = (P + kTB - 1) / kTB < 4096 ? (P + kTB - 1) / kTB : 4096;
  const int bb = (P + kTB - 1) / kTB < kBBoxBlocks ? (P + kTB - 1) / kTB : kBBoxBlocks;
  hipLaunchKernelGGL(k_tc_bbox_partial, dim3(bb), dim3(kTB), 0, st, X, P, r.part);
  hipLaunchKernelGGL(k_tc_bbox_final, dim3(1), dim3(64), 0, st, r.part, bb, r.geom, p, binomials ? r.tab : nullptr);
  const int zb = (nleaf + kTB - 1) / kTB < 4096 ? (nleaf + kTB - 1) / kTB : 4096;
  hipLaunchKernelGGL(k_tc_zero, dim3(zb), dim3(kTB), 0, st, r.counts, r.cursor, nleaf);
  hipLaunchKernelGGL(k_tc_leaf, dim3(pb), dim3(kTB), 0, st, X, P, r.geom, depth, r.leafid, r.counts);
  hipLaunchKernelGGL(k_tc_vid, dim3(M), dim3(kTB), 0, st, off, P, r.vid, w, r.geom, depth, near ? r.h2 : nullptr,
                     r.flag);
  hipLaunchKernelGGL(k_tc_scan, dim3(1), dim3(1024), 0, st, r.counts, nleaf, r.starts, r.wstart, cshift);
  hipLaunchKernelGGL(k_tc_scatter, dim3(pb), dim3(kTB), 0, st, r.leafid, P, r.starts, r.cursor, r.perm);
  hipLaunchKernelGGL(k_tc_sort, dim3(nleaf), dim3(64), 0, st, r.starts, r.perm);
  if (depth < 2) return;
  hipLaunchKernelGGL(k_tc_p2m, dim3(nleaf), dim3(64), sizeof(double2) * (size_t)kP2MChunk * (p + 3), st, X, f, w, P,
                     r.perm, r.starts, r.geom, depth, p,
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
    hipLaunchKernelGGL(k_tc_own, dim3(M), dim3(kOwnThreads), 0, st, X, f, w, P, off, r.leafid, depth, scale, out);
}

}  // namespace

// Everything is built on the device; the launches need no host copy and no synchronisation.
hipError_t launch_treecode(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                           double scale, int p, int depth, double* out, void* ws, void* stream) {
  if (P == 0) return hipSuccess;
  if (depth < 0 || depth > kMaxDepth || p < 1 || p > kMaxOrder) return hipErrorInvalidValue;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const TreeRun r = tree_run(ws, tree_layout(P, depth, p, false), depth, p);
  launch_upward(X, f, w, off, M, P, p, depth, eval_chunk_shift<false>(), false, false, r, st);
  if (depth >= 2) {
    const size_t work = r.nbox * (p + 1);
    const int gb = (int)((work + kTB - 1) / kTB < 4096 ? (work + kTB - 1) / kTB : 4096);
    hipLaunchKernelGGL(k_tc_finalize, dim3(gb), dim3(kTB), 0, st, r.mom, r.nbox, p);
  }
  launch_eval<false>(X, f, w, off, M, P, p, depth, scale, r, out, st);
  return hipGetLastError();
}

static hipError_t run_fmm(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                          double scale, int p, int depth, double* out, void* ws, hipStream_t st, bool near,
                          int32_t* pairs, int capacity, int32_t* count) {
  const TreeRun r = tree_run(ws, tree_layout(P, depth, p, true, near ? M : 0), depth, p);
  if (near) hipLaunchKernelGGL(k_tc_zero, dim3(1), dim3(kTB), 0, st, count, r.flag, 1);
  launch_upward(X, f, w, off, M, P, p, depth, eval_chunk_shift<true>(), depth >= 2, near, r, st);
  if (depth >= 2) {
    const dim3 g((unsigned)r.nbox), bl(64);
    const size_t lds = m2l_lds_bytes(p);
    switch (m2l_rtiles(p)) {
      case 1: hipLaunchKernelGGL(k_fmm_m2l<1>, g, bl, lds, st, r.geom, depth, p, r.mom, r.bcount, r.tab, r.loc); break;
      case 2: hipLaunchKernelGGL(k_fmm_m2l<2>, g, bl, lds, st, r.geom, depth, p, r.mom, r.bcount, r.tab, r.loc); break;
      case 3: hipLaunchKernelGGL(k_fmm_m2l<3>, g, bl, lds, st, r.geom, depth, p, r.mom, r.bcount, r.tab, r.loc); break;
      default: hipLaunchKernelGGL(k_fmm_m2l<4>, g, bl, lds, st, r.geom, depth, p, r.mom, r.bcount, r.tab, r.loc); break;
    }
    if (depth >= 3) {
      const int nleaf = 1 << (2 * depth);
      hipLaunchKernelGGL(k_fmm_l2l, dim3(nleaf), dim3(64), sizeof(double2) * ((size_t)(depth - 2) * 3 * (p + 1) + 96),
                         st, r.geom, depth, p, r.bcount, r.loc);
    }
  }
  launch_eval<true>(X, f, w, off, M, P, p, depth, scale, r, out, st);
  if (near) {
    constexpr int kChunk = 1 << eval_chunk_shift<true>();
    const int nleaf = 1 << (2 * depth);
    const int items = nleaf + (P + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_fmm_near, dim3(items), dim3(64), 0, st, X, f, w, P, M, off, r.vid, r.perm, r.starts, r.wstart,
                       depth, r.h2, scale, out, pairs, capacity, count, r.flag);
    hipLaunchKernelGGL(k_fmm_near_status, dim3(1), dim3(64), 0, st, r.flag, count);
  }
  return hipGetLastError();
}

hipError_t launch_fmm(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                      double scale, int p, int depth, double* out, void* ws, void* stream) {
  if (P == 0) return hipSuccess;
  if (depth < 0 || depth > kMaxDepth || p < 1 || p > kMaxOrder) return hipErrorInvalidValue;
  return run_fmm(X, f, w, off, M, P, scale, p, depth, out, ws, reinterpret_cast<hipStream_t>(stream), false, nullptr,
                 0, nullptr);
}

hipError_t launch_zero_count(int32_t* count, void* stream) {
  hipLaunchKernelGGL(k_tc_zero, dim3(1), dim3(kTB), 0, reinterpret_cast<hipStream_t>(stream), count, count, 1);
  return hipGetLastError();
}

hipError_t launch_fmm_nearmasked(const double* X, const double* f, const double* w, const int32_t* off, int M, int P,
                                 double scale, int p, int depth, double* out, int32_t* pairs, int capacity,
                                 int32_t* count, void* ws, void* stream) {
  if (P == 0) return hipSuccess;
  if (depth < 0 || depth > kMaxDepth || p < 1 || p > kMaxOrder) return hipErrorInvalidValue;
  return run_fmm(X, f, w, off, M, P, scale, p, depth, out, ws, reinterpret_cast<hipStream_t>(stream), true, pairs,
                 capacity, count);
}

}  // namespace vesnet
