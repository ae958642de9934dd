/*
 * Plain FP64 CPU oracle for the far-field Stokeslet single-layer sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * reads this file; it exists so that tests, the smoke check and the
 * benchmark's CPU baseline can check the GPU path against an independent,
 * obviously correct evaluation.  It shares no code with the GPU path.
 *
 * What it computes (Section 2.2, eq. (single_layer) with the Stokeslet of
 * eq. (Stokeslet), discretised by the trapezoid rule of Section 2.2.1, over
 * the vesicles other than the target's own, as in the split of
 * eq. (membrane_velocity) and DirectSingleLayerIntegral of Algorithm 4):
 *
 *   u(x_i) = 1/(4 pi mu) * sum_{j : ves(j) != excl(i)} w_j [ -ln|r| f_j + (r . f_j) r / |r|^2 ],
 *   r = x_i - y_j.
 *
 * Readings of the printed formula: the log term carries a minus sign and the
 * identity matrix (the printed Stokeslet shows "+log|r|" without I; only
 * -ln|r| I gives a divergence-free field whose single layer annihilates the
 * normal, which the pinned tests check).  w_j is the arclength element
 * |X'(alpha_j)| * 2 pi / N of the trapezoid rule, supplied by the caller.
 *
 * Gradients (the paper has none; derived from the sum above).  With
 * c = 1/(4 pi mu), F_j = w_j f_j, g_i = dL/du_i and
 *   phi(r; g, F) = g^T G(r) F = c [ -ln|r| (g.F) + (g.r)(r.F)/|r|^2 ],
 *   grad_r phi   = c [ -(g.F) r/|r|^2 + (g (r.F) + F (g.r))/|r|^2 - 2 (g.r)(r.F) r/|r|^4 ],
 * the outputs are
 *   dL/dx_i = sum_j grad_r phi(r_ij; g_i, F_j)
 *   dL/dy_j = - sum_i grad_r phi(r_ij; g_i, F_j)
 *   v_j     = sum_i G(r_ij) g_i          (the forward operator applied to g)
 *   dL/df_j = w_j v_j,   dL/dw_j = f_j . v_j
 * with the same vesicle exclusion in every sum.
 *
 * Each term is evaluated in double precision with libm log; each output is
 * accumulated in long double in plain index order.  OpenMP runs the outer
 * loop over output points.  A coincident included pair (r = 0) is a
 * precondition violation: the call returns -2 and writes nothing useful.
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

#define VO_PI 3.14159265358979323846

int vo_num_threads(void) { return omp_get_max_threads(); }

/* u at the selected targets sel[0..n_sel) (indices into the target arrays). */
int vo_farfield_at(int64_t n_sel, const int64_t* sel,
                   const double* tx, const double* ty, const int32_t* t_excl,
                   int64_t n_src, const double* sx, const double* sy, const int32_t* s_ves,
                   const double* fx, const double* fy, const double* w, double mu,
                   double* ux, double* uy)
{
    const double c = 1.0 / (4.0 * VO_PI * mu);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(|:bad)
    for (int64_t k = 0; k < n_sel; ++k) {
        const int64_t i = sel[k];
        long double ax = 0.0L, ay = 0.0L;
        for (int64_t j = 0; j < n_src; ++j) {
            if (s_ves[j] == t_excl[i]) continue;
            const double rx = tx[i] - sx[j];
            const double ry = ty[i] - sy[j];
            const double r2 = rx * rx + ry * ry;
            if (r2 == 0.0) { bad = 1; continue; }
            const double lnr = 0.5 * log(r2);
            const double rdotf = rx * fx[j] + ry * fy[j];
            ax += (long double)(w[j] * (-lnr * fx[j] + rdotf * rx / r2));
            ay += (long double)(w[j] * (-lnr * fy[j] + rdotf * ry / r2));
        }
        ux[k] = (double)(c * ax);
        uy[k] = (double)(c * ay);
    }
    return bad ? -2 : 0;
}

/* grad_r phi(r; g, F) without the factor c. */
static void grad_phi(double rx, double ry, double gx, double gy, double Fx, double Fy,
                     double* ox, double* oy)
{
    const double r2 = rx * rx + ry * ry;
    const double gF = gx * Fx + gy * Fy;
    const double gr = gx * rx + gy * ry;
    const double rF = rx * Fx + ry * Fy;
    *ox = -gF * rx / r2 + (gx * rF + Fx * gr) / r2 - 2.0 * gr * rF * rx / (r2 * r2);
    *oy = -gF * ry / r2 + (gy * rF + Fy * gr) / r2 - 2.0 * gr * rF * ry / (r2 * r2);
}

/* dL/dx at the selected targets. g is indexed like the targets. */
int vo_grad_targets_at(int64_t n_sel, const int64_t* sel,
                       const double* tx, const double* ty, const int32_t* t_excl,
                       int64_t n_src, const double* sx, const double* sy, const int32_t* s_ves,
                       const double* fx, const double* fy, const double* w, double mu,
                       const double* gx, const double* gy,
                       double* grad_x, double* grad_y)
{
    const double c = 1.0 / (4.0 * VO_PI * mu);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(|:bad)
    for (int64_t k = 0; k < n_sel; ++k) {
        const int64_t i = sel[k];
        long double ax = 0.0L, ay = 0.0L;
        for (int64_t j = 0; j < n_src; ++j) {
            if (s_ves[j] == t_excl[i]) continue;
            const double rx = tx[i] - sx[j];
            const double ry = ty[i] - sy[j];
            if (rx * rx + ry * ry == 0.0) { bad = 1; continue; }
            double ox, oy;
            grad_phi(rx, ry, gx[i], gy[i], w[j] * fx[j], w[j] * fy[j], &ox, &oy);
            ax += (long double)ox;
            ay += (long double)oy;
        }
        grad_x[k] = (double)(c * ax);
        grad_y[k] = (double)(c * ay);
    }
    return bad ? -2 : 0;
}

/* dL/dy, v, dL/df and dL/dw at the selected sources. g is indexed like the targets. */
int vo_grad_sources_at(int64_t n_sel, const int64_t* sel,
                       int64_t n_tgt, const double* tx, const double* ty, const int32_t* t_excl,
                       const double* sx, const double* sy, const int32_t* s_ves,
                       const double* fx, const double* fy, const double* w, double mu,
                       const double* gx, const double* gy,
                       double* grad_x, double* grad_y, double* vx, double* vy,
                       double* grad_fx, double* grad_fy, double* grad_w)
{
    const double c = 1.0 / (4.0 * VO_PI * mu);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(|:bad)
    for (int64_t k = 0; k < n_sel; ++k) {
        const int64_t j = sel[k];
        const double Fx = w[j] * fx[j], Fy = w[j] * fy[j];
        long double ax = 0.0L, ay = 0.0L, bx = 0.0L, by = 0.0L;
        for (int64_t i = 0; i < n_tgt; ++i) {
            if (s_ves[j] == t_excl[i]) continue;
            const double rx = tx[i] - sx[j];
            const double ry = ty[i] - sy[j];
            const double r2 = rx * rx + ry * ry;
            if (r2 == 0.0) { bad = 1; continue; }
            double ox, oy;
            grad_phi(rx, ry, gx[i], gy[i], Fx, Fy, &ox, &oy);
            ax -= (long double)ox;
            ay -= (long double)oy;
            /* G(r) g_i : the Stokeslet applied to g_i */
            const double lnr = 0.5 * log(r2);
            const double rdotg = rx * gx[i] + ry * gy[i];
            bx += (long double)(-lnr * gx[i] + rdotg * rx / r2);
            by += (long double)(-lnr * gy[i] + rdotg * ry / r2);
        }
        grad_x[k] = (double)(c * ax);
        grad_y[k] = (double)(c * ay);
        const double v_x = (double)(c * bx), v_y = (double)(c * by);
        vx[k] = v_x;
        vy[k] = v_y;
        grad_fx[k] = w[j] * v_x;
        grad_fy[k] = w[j] * v_y;
        grad_w[k] = fx[j] * v_x + fy[j] * v_y;
    }
    return bad ? -2 : 0;
}

/*
 * Near-field masked far field (the masks of Section 4.1; FindNearFieldPoints of
 * Algorithm 4; near-field rule of Section 2.2).  Vesicle v is in the near field
 * of target i when min_{j in v} |x_i - y_j| <= h_v, with h_v = sum_{j in v} w_j / N_v
 * the mean arclength spacing of v.  Such vesicles are dropped like the own one.
 * Source vesicle ids must lie in [0, n_ves).  Near pairs (selected-target position
 * k, vesicle v) are written to pairs[2*c], pairs[2*c+1] for c < capacity in target
 * order, then vesicle order; the return value is the number of near pairs, or -2
 * for a coincident included pair, -3 for a bad vesicle id, -4 if memory ran out.
 */
#include <stdlib.h>

long vo_farfield_nearmasked_at(int64_t n_sel, const int64_t* sel,
                               const double* tx, const double* ty, const int32_t* t_excl,
                               int64_t n_src, const double* sx, const double* sy, const int32_t* s_ves,
                               int32_t n_ves, const double* fx, const double* fy, const double* w, double mu,
                               double* ux, double* uy, int64_t* pairs, int64_t capacity)
{
    const double c = 1.0 / (4.0 * VO_PI * mu);
    for (int64_t j = 0; j < n_src; ++j)
        if (s_ves[j] < 0 || s_ves[j] >= n_ves) return -3;
    double* h = (double*)calloc((size_t)n_ves + 1, sizeof(double));
    int64_t* cnt = (int64_t*)calloc((size_t)n_ves + 1, sizeof(int64_t));
    char* near = (char*)calloc((size_t)n_sel * (size_t)n_ves + 1, 1);
    if (!h || !cnt || !near) { free(h); free(cnt); free(near); return -4; }
    for (int64_t j = 0; j < n_src; ++j) { h[s_ves[j]] += w[j]; cnt[s_ves[j]] += 1; }
    for (int32_t v = 0; v < n_ves; ++v) h[v] = cnt[v] > 0 ? h[v] / (double)cnt[v] : 0.0;
    int bad = 0, oom = 0;
#pragma omp parallel reduction(|:bad) reduction(|:oom)
    {
        long double* ax = (long double*)malloc(((size_t)n_ves + 1) * sizeof(long double));
        long double* ay = (long double*)malloc(((size_t)n_ves + 1) * sizeof(long double));
        double* dmin = (double*)malloc(((size_t)n_ves + 1) * sizeof(double));
        if (!ax || !ay || !dmin) {
            oom = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int64_t k = 0; k < n_sel; ++k) {
                const int64_t i = sel[k];
                for (int32_t v = 0; v < n_ves; ++v) { ax[v] = 0.0L; ay[v] = 0.0L; dmin[v] = INFINITY; }
                for (int64_t j = 0; j < n_src; ++j) {
                    const int32_t v = s_ves[j];
                    if (v == t_excl[i]) continue;
                    const double rx = tx[i] - sx[j];
                    const double ry = ty[i] - sy[j];
                    const double r2 = rx * rx + ry * ry;
                    if (r2 < dmin[v]) dmin[v] = r2;
                    if (r2 == 0.0) { bad = 1; continue; }
                    const double lnr = 0.5 * log(r2);
                    const double rdotf = rx * fx[j] + ry * fy[j];
                    ax[v] += (long double)(w[j] * (-lnr * fx[j] + rdotf * rx / r2));
                    ay[v] += (long double)(w[j] * (-lnr * fy[j] + rdotf * ry / r2));
                }
                long double sxv = 0.0L, syv = 0.0L;
                for (int32_t v = 0; v < n_ves; ++v) {
                    if (v == t_excl[i] || cnt[v] == 0) continue;
                    if (dmin[v] <= h[v] * h[v]) { near[k * (int64_t)n_ves + v] = 1; continue; }
                    sxv += ax[v];
                    syv += ay[v];
                }
                ux[k] = (double)(c * sxv);
                uy[k] = (double)(c * syv);
            }
        }
        free(ax); free(ay); free(dmin);
    }
    long found = 0;
    for (int64_t k = 0; k < n_sel; ++k)
        for (int32_t v = 0; v < n_ves; ++v)
            if (near[k * (int64_t)n_ves + v]) {
                if (found < capacity) { pairs[2 * found] = k; pairs[2 * found + 1] = v; }
                ++found;
            }
    free(h); free(cnt); free(near);
    if (oom) return -4;
    return bad ? -2 : found;
}
