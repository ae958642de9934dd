// Host side of the C-ABI declared in include/vesnet.h: argument validation,
// workspace layout, launch-shape selection, HIP graphs and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "vesnet.h"
#include "vesnet_internal.h"

using namespace vesnet;

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kMaxPoints = 1 << 30;   // 2P indices stay inside int32
constexpr int kMaxSplits = 64;
constexpr double kPi = 3.14159265358979323846;

thread_local char g_err[768] = "";

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return status;
}

int ok() {
  g_err[0] = '\0';
  return VESNET_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(VESNET_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t rec_bytes(int prec) { return prec == P64 ? sizeof(double4) : sizeof(float4); }

// The forward calls' prepared region of the compensated form also holds the float64 weighted
// forces and the per-vesicle |F|_1 sums that the symmetric form needs.
bool fwd_forces(int prec) { return prec == P32C || prec == P64; }

// The precisions with a symmetric form (one evaluation per unordered pair), and the 64-bit accumulator
// words it needs per point and component (float64: a high and a low fixed-point word).
bool has_symmetric(int prec) { return prec == P32C || prec == P64; }
int acc_words(int prec) { return prec == P64 ? 2 : 1; }

size_t prepared_bytes(int32_t P, int32_t M, int prec, bool forces = false) {
  size_t b = align_up((size_t)M * sizeof(int2)) + align_up((size_t)P * sizeof(int32_t)) +
             align_up((size_t)M * sizeof(double4)) + align_up((size_t)M * sizeof(double)) +
             align_up((size_t)P * rec_bytes(prec));
  if (forces) b += align_up((size_t)P * sizeof(double2)) + align_up((size_t)M * sizeof(double2));
  return b;
}

// Carves the prepared region starting at *cursor (already aligned).
PreparedView carve_prepared(char*& cursor, int32_t P, int32_t M, int prec, bool forces = false) {
  PreparedView pv{};
  pv.vrange = reinterpret_cast<int2*>(cursor);
  cursor += align_up((size_t)M * sizeof(int2));
  pv.vid = reinterpret_cast<int32_t*>(cursor);
  cursor += align_up((size_t)P * sizeof(int32_t));
  pv.vtab = reinterpret_cast<double4*>(cursor);
  cursor += align_up((size_t)M * sizeof(double4));
  pv.hlen = reinterpret_cast<double*>(cursor);
  cursor += align_up((size_t)M * sizeof(double));
  pv.rec = cursor;
  cursor += align_up((size_t)P * rec_bytes(prec));
  if (forces) {
    pv.f64 = reinterpret_cast<double2*>(cursor);
    cursor += align_up((size_t)P * sizeof(double2));
    pv.vaux = reinterpret_cast<double2*>(cursor);
    cursor += align_up((size_t)M * sizeof(double2));
  }
  return pv;
}

// The symmetric form's region: cycle table, plan values, cycle net forces, fixed-point sums.
size_t symmetric_bytes(int32_t P, int32_t M, int words = 1) {
  return align_up((size_t)sym_max_cycles(P, M) * sizeof(int4)) + align_up(4 * sizeof(int32_t)) +
         align_up((size_t)sym_max_cycles(P, M) * sizeof(double2)) +
         align_up((size_t)2 * words * P * sizeof(unsigned long long));
}

SymmetricView carve_symmetric(char*& cursor, int32_t P, int32_t M, int words = 1) {
  SymmetricView sv;
  sv.cyc = reinterpret_cast<int4*>(cursor);
  cursor += align_up((size_t)sym_max_cycles(P, M) * sizeof(int4));
  sv.meta = reinterpret_cast<int32_t*>(cursor);
  cursor += align_up(4 * sizeof(int32_t));
  sv.fcyc = reinterpret_cast<double2*>(cursor);
  cursor += align_up((size_t)sym_max_cycles(P, M) * sizeof(double2));
  sv.acc = reinterpret_cast<unsigned long long*>(cursor);
  cursor += align_up((size_t)2 * words * P * sizeof(unsigned long long));
  return sv;
}

char* aligned_base(void* ws) {
  uintptr_t p = reinterpret_cast<uintptr_t>(ws);
  return reinterpret_cast<char*>((p + kAlign - 1) / kAlign * kAlign);
}

bool valid_precision(int prec) { return prec == VESNET_FP64 || prec == VESNET_FP32_COMPENSATED || prec == VESNET_FP32_NAIVE; }

struct Shape {
  int T, B, splits, bpc, staging, accumulate;
  int pair;  // 0 automatic, 1 direct, 2 symmetric
  int symT;  // targets per thread of the symmetric form (0: too few units for it)
};

// Targets per thread of the symmetric form: the largest of `top`, 2 and 1 that gives at least four units
// per compute unit (a unit is one workgroup of 256 threads on one pair of blocks of 256 T points),
// estimated with vesicles of a multiple of 16 points; 0 when even 1 gives fewer (direct form).  `top` is
// the fastest measured on the 2000 x 128 suspension: 3 for the compensated forward (14.9 ms against
// 15.7 ms at 2, 17.1 ms at 4 and 17.7 ms at 1) and adjoint (31.3 ms against 32.2 ms at 2 and 36.6 ms at
// 4), 4 for the float64 forward (41.7 ms against 42.3 ms at 3 and 43.4 ms at 2).
int sym_default_T(int32_t P, int top) {
  for (int T : {top, 2, 1}) {
    const int64_t cyc = (int64_t)P / 16;
    const int cb = sym_cycles_per_block(T);
    if (sym_units((cyc + cb - 1) / cb) >= 1024) return T;
  }
  return 0;
}

// The default launch shape is the one the autotuner picks on the 2000 x 128 suspension
// (T = 1, 256 threads, LDS staging, VALU accumulation) with enough source chunks for
// about 64 waves per SIMD over the launch (at least 16 chunks would be needed at 256k
// targets), which keeps the tail of the last wave round short.
Shape default_shape(int32_t P, int32_t M, int prec) {
  Shape s;
  s.T = 1;
  s.B = 256;
  s.bpc = 4;
  s.staging = 2;
  s.accumulate = 1;
  const int64_t waves = ((int64_t)P + 64 * s.T - 1) / (64 * s.T);
  const int64_t want = 65536;
  int splits = 1;
  while (waves * splits < want && splits < 16) splits *= 2;
  s.splits = std::max(1, std::min<int>(splits, std::max(1, M)));
  s.pair = 0;
  s.symT = has_symmetric(prec) ? sym_default_T(P, prec == P32C ? 3 : 4) : 0;
  return s;
}

int resolve_shape(const vesnet_tile_config* cfg, int32_t P, int32_t M, int prec, Shape* out) {
  Shape s = default_shape(P, M, prec);
  if (cfg) {
    if (cfg->targets_per_thread) s.T = cfg->targets_per_thread;
    if (cfg->block_threads) s.B = cfg->block_threads;
    if (cfg->source_splits) s.splits = cfg->source_splits;
    if (cfg->blocks_per_cu) s.bpc = cfg->blocks_per_cu;
    if (cfg->source_staging) s.staging = cfg->source_staging;
    if (cfg->accumulate) s.accumulate = cfg->accumulate;
    if (cfg->pair_form) s.pair = cfg->pair_form;
    // the symmetric form takes the caller's targets_per_thread only when it is asked for explicitly;
    // the automatic choice keeps its own default
    if (cfg->targets_per_thread && cfg->pair_form == 2) s.symT = cfg->targets_per_thread;
  }
  if (s.T != 1 && s.T != 2 && s.T != 4 && !((s.T == 3 || s.T == 8) && s.pair == 2))
    return fail(VESNET_ERR_INVALID_ARGUMENT,
                "targets_per_thread must be 1, 2 or 4 (3 or 8 for the symmetric form; got %d)", s.T);
  if (s.symT < 0 || s.symT > 8 || (s.symT > 4 && s.symT != 8))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "targets_per_thread of the symmetric form must be 1, 2, 3, 4 or 8");
  if (s.B != 64 && s.B != 128 && s.B != 256)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "block_threads must be 64, 128 or 256 (got %d)", s.B);
  if (s.splits < 1 || s.splits > kMaxSplits)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "source_splits must be in [1, %d] (got %d)", kMaxSplits, s.splits);
  if (s.bpc < 1 || s.bpc > 16)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "blocks_per_cu must be in [1, 16] (got %d)", s.bpc);
  if (s.staging != 1 && s.staging != 2)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "source_staging must be 1 or 2 (got %d)", s.staging);
  if (s.accumulate != 1 && s.accumulate != 2)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "accumulate must be 1 or 2 (got %d)", s.accumulate);
  if (s.accumulate == 2 && prec != VESNET_FP32_COMPENSATED)
    return fail(VESNET_ERR_UNSUPPORTED, "matrix-core accumulation exists for the compensated form only");
  if (s.pair < 0 || s.pair > 2)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "pair_form must be 0, 1 or 2 (got %d)", s.pair);
  if (s.pair == 2 && !has_symmetric(prec))
    return fail(VESNET_ERR_UNSUPPORTED, "the symmetric pair form exists for the compensated and float64 forms only");
  if (s.pair == 2 && prec == P64 && s.symT > 4)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "targets_per_thread of the float64 symmetric form must be 1, 2, 3 or 4");
  if (s.pair == 2 && s.accumulate == 2)
    return fail(VESNET_ERR_UNSUPPORTED, "the symmetric pair form accumulates on the VALU only");
  if (s.pair == 2 && s.symT == 0) s.symT = 1;
  if (s.symT && !sym_fits(P, M, s.symT)) {
    if (s.pair == 2)
      return fail(VESNET_ERR_UNSUPPORTED, "too many points for the symmetric form at %d targets per thread (its "
                  "units exceed one launch); use more targets per thread or the direct form", s.symT);
    s.symT = sym_fits(P, M, 4) ? 4 : prec != P64 && sym_fits(P, M, 8) ? 8 : 0;
  }
  *out = s;
  return VESNET_OK;
}

// Forward workspace: prepared region, then the direct form's split partials and the symmetric
// form's region (both when the form is chosen per call).
size_t forward_bytes(int32_t P, int32_t M, int prec, const Shape& s) {
  size_t b = kAlign + prepared_bytes(P, M, prec, fwd_forces(prec));
  if (s.pair != 2 && s.splits > 1) b += align_up((size_t)2 * s.splits * P * sizeof(double));
  if (has_symmetric(prec) && s.pair != 1) b += symmetric_bytes(P, M, acc_words(prec));
  return b;
}

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  if (!a || !b || an == 0 || bn == 0) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bn && pb < pa + an;
}

int check_sizes(int32_t P, int32_t M) {
  if (P < 0 || M < 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "negative size (n_points=%d, n_vesicles=%d)", P, M);
  if (P > kMaxPoints) return fail(VESNET_ERR_INVALID_ARGUMENT, "n_points=%d exceeds the limit %d", P, kMaxPoints);
  if (P > 0 && M == 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "n_points=%d but no vesicles", P);
  return VESNET_OK;
}

int check_mu(double mu) {
  if (!(std::isfinite(mu) && mu > 0.0)) return fail(VESNET_ERR_INVALID_ARGUMENT, "mu must be finite and > 0 (got %g)", mu);
  return VESNET_OK;
}

int check_workspace(void* ws, size_t have, size_t need) {
  if (need > 0 && !ws) return fail(VESNET_ERR_WORKSPACE, "workspace is NULL but %zu bytes are needed", need);
  if (have < need) return fail(VESNET_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", have, need);
  return VESNET_OK;
}

// Checks common to the forward entry points (targets/sources may be NULL when unused).
int check_forward_args(const double* targets, const double* sources, const double* f, const double* w,
                       const int32_t* off, int32_t M, int32_t P, double* out, int prec, void* ws, size_t ws_bytes,
                       bool need_targets, bool need_sources) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if (!valid_precision(prec)) return fail(VESNET_ERR_INVALID_ARGUMENT, "unknown precision %d", prec);
  if (P == 0) return VESNET_OK;
  if (!off) return fail(VESNET_ERR_INVALID_ARGUMENT, "vesicle_offsets is NULL");
  if (need_targets && !targets) return fail(VESNET_ERR_INVALID_ARGUMENT, "targets is NULL");
  if (need_sources && (!sources || !f || !w))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "sources, force_density and arc_weights must be non-NULL");
  if (out) {
    const size_t vb = (size_t)2 * P * sizeof(double);
    if (overlaps(out, vb, targets, vb) || overlaps(out, vb, sources, vb) || overlaps(out, vb, f, vb) ||
        overlaps(out, vb, w, (size_t)P * sizeof(double)) || overlaps(out, vb, ws, ws_bytes) ||
        overlaps(out, vb, off, (size_t)(M + 1) * sizeof(int32_t)))
      return fail(VESNET_ERR_INVALID_ARGUMENT, "out overlaps an input or the workspace");
  }
  return VESNET_OK;
}

}  // namespace

// ============================================================================ general

extern "C" const char* vesnet_version(void) { return "vesnet 0.1.0 (gfx950)"; }

extern "C" const char* vesnet_last_error(void) { return g_err; }

extern "C" int vesnet_check_offsets(const int32_t* off, int32_t M, int32_t P) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if (!off) return fail(VESNET_ERR_INVALID_ARGUMENT, "offsets is NULL");
  if (off[0] != 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "offsets[0] = %d, expected 0", off[0]);
  for (int32_t v = 0; v < M; ++v)
    if (off[v + 1] < off[v])
      return fail(VESNET_ERR_INVALID_ARGUMENT, "offsets decrease at vesicle %d (%d > %d)", v, off[v], off[v + 1]);
  if (off[M] != P) return fail(VESNET_ERR_INVALID_ARGUMENT, "offsets[M] = %d, expected n_points = %d", off[M], P);
  return ok();
}

extern "C" int vesnet_default_tile_config(int32_t P, int32_t M, int prec, vesnet_tile_config* cfg) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if (!valid_precision(prec)) return fail(VESNET_ERR_INVALID_ARGUMENT, "unknown precision %d", prec);
  if (!cfg) return fail(VESNET_ERR_INVALID_ARGUMENT, "cfg is NULL");
  Shape s = default_shape(P, M, prec);
  cfg->targets_per_thread = s.T;
  cfg->block_threads = s.B;
  cfg->source_splits = s.splits;
  cfg->blocks_per_cu = s.bpc;
  cfg->source_staging = s.staging;
  cfg->accumulate = s.accumulate;
  cfg->pair_form = s.pair;
  return ok();
}

// ============================================================================ forward

extern "C" size_t vesnet_farfield_workspace_bytes(int32_t P, int32_t M, int prec, const vesnet_tile_config* cfg) {
  if (check_sizes(P, M) || !valid_precision(prec)) return 0;
  Shape s;
  if (resolve_shape(cfg, P, M, prec, &s)) return 0;
  return forward_bytes(P, M, prec, s);
}

extern "C" int vesnet_farfield_prepare(const double* sources, const double* f, const double* w, const int32_t* off,
                                       int32_t M, int32_t P, int prec, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_forward_args(nullptr, sources, f, w, off, M, P, nullptr, prec, ws, ws_bytes, false, true);
  if (rc) return rc;
  if (P == 0) return ok();
  const size_t need = kAlign + prepared_bytes(P, M, prec, fwd_forces(prec));
  if ((rc = check_workspace(ws, ws_bytes, need))) return rc;
  char* cur = aligned_base(ws);
  PreparedView pv = carve_prepared(cur, P, M, prec, fwd_forces(prec));
  hipError_t e = launch_prepare(prec, sources, f, w, off, M, P, pv, stream);
  if (e != hipSuccess) return hip_fail(e, "prepare launch");
  return ok();
}

namespace {

// Evaluation from a prepared workspace with a resolved shape; symmetric selects the form that
// evaluates each unordered pair once (targets must be the prepared sources).
int evaluate_resolved(const double* targets, int32_t M, int32_t P, double mu, double* out, int prec, const Shape& s,
                      bool symmetric, void* ws, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = check_workspace(ws, ws_bytes, forward_bytes(P, M, prec, s)))) return rc;
  char* cur = aligned_base(ws);
  PreparedView pv = carve_prepared(cur, P, M, prec, fwd_forces(prec));
  const double scale = 1.0 / (4.0 * kPi * mu);
  hipError_t e;
  if (symmetric) {
    if (s.pair != 2 && s.splits > 1) cur += align_up((size_t)2 * s.splits * P * sizeof(double));
    SymmetricView sv = carve_symmetric(cur, P, M, acc_words(prec));
    e = prec == P64 ? launch_forward_symmetric64(s.symT, P, M, pv, sv, scale, out, stream)
                    : launch_forward_symmetric(s.symT, P, M, pv, sv, scale, out, stream);
    if (e != hipSuccess) return hip_fail(e, "symmetric forward launch");
  } else {
    double* partial = s.splits > 1 ? reinterpret_cast<double*>(cur) : nullptr;
    e = launch_forward(prec, s.T, s.B, s.staging == 2, s.accumulate == 2, s.splits, targets, P, M, pv, scale, out,
                       partial, stream);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
  }
  return ok();
}

}  // namespace

extern "C" int vesnet_farfield_evaluate(const double* targets, const int32_t* off, int32_t M, int32_t P, double mu,
                                        double* out, int prec, const vesnet_tile_config* cfg, void* ws,
                                        size_t ws_bytes, void* stream) {
  int rc = check_forward_args(targets, nullptr, nullptr, nullptr, off, M, P, out, prec, ws, ws_bytes, true, false);
  if (rc) return rc;
  if ((rc = check_mu(mu))) return rc;
  if (P == 0) return ok();
  if (!out) return fail(VESNET_ERR_INVALID_ARGUMENT, "out is NULL");
  Shape s;
  if ((rc = resolve_shape(cfg, P, M, prec, &s))) return rc;
  return evaluate_resolved(targets, M, P, mu, out, prec, s, s.pair == 2, ws, ws_bytes, stream);
}

extern "C" int vesnet_farfield_stokeslet(const double* targets, const double* sources, const double* f,
                                         const double* w, const int32_t* off, int32_t M, int32_t P, double mu,
                                         double* out, int prec, const vesnet_tile_config* cfg, void* ws,
                                         size_t ws_bytes, void* stream) {
  int rc = check_forward_args(targets, sources, f, w, off, M, P, out, prec, ws, ws_bytes, true, true);
  if (rc) return rc;
  if ((rc = check_mu(mu))) return rc;
  if (P == 0) return ok();
  if (!out) return fail(VESNET_ERR_INVALID_ARGUMENT, "out is NULL");
  Shape s;
  if ((rc = resolve_shape(cfg, P, M, prec, &s))) return rc;
  if (s.pair == 2 && targets != sources)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "the symmetric pair form needs targets == sources (one point array)");
  const bool symmetric =
      s.pair == 2 || (s.pair == 0 && targets == sources && has_symmetric(prec) && s.accumulate == 1 && s.symT > 0);
  if ((rc = check_workspace(ws, ws_bytes, forward_bytes(P, M, prec, s)))) return rc;
  if ((rc = vesnet_farfield_prepare(sources, f, w, off, M, P, prec, ws, ws_bytes, stream))) return rc;
  return evaluate_resolved(targets, M, P, mu, out, prec, s, symmetric, ws, ws_bytes, stream);
}

// ============================================================================ membrane force

extern "C" int vesnet_elastic_force(const double* X, const double* sigma, double kappa_b, const int32_t* off,
                                    int32_t M, int32_t P, double* f, double* w, void* stream) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if (!std::isfinite(kappa_b)) return fail(VESNET_ERR_INVALID_ARGUMENT, "kappa_b must be finite (got %g)", kappa_b);
  if (P == 0) return ok();
  if (!X || !off || !f || !w) return fail(VESNET_ERR_INVALID_ARGUMENT, "X, offsets, force and weights must be non-NULL");
  const size_t vb = (size_t)2 * P * sizeof(double), sb = (size_t)P * sizeof(double);
  if (overlaps(f, vb, X, vb) || overlaps(f, vb, sigma, sb) || overlaps(f, vb, w, sb) || overlaps(w, sb, X, vb) ||
      overlaps(w, sb, sigma, sb) || overlaps(f, vb, off, (size_t)(M + 1) * sizeof(int32_t)) ||
      overlaps(w, sb, off, (size_t)(M + 1) * sizeof(int32_t)))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "outputs overlap an input or each other");
  hipError_t e = launch_elastic(X, sigma, kappa_b, off, M, P, f, w, stream);
  if (e != hipSuccess) return hip_fail(e, "elastic force launch");
  return ok();
}

// ============================================================================ near-field interpolation

namespace {

constexpr int32_t kRbfMaxPoints = 200;         // 5 x 200 nodes per vesicle
constexpr int kRbfMaxSlots = 2048;             // eight one-wavefront fits per compute unit
constexpr size_t kRbfSlotBudget = (size_t)1 << 30;  // recommended workspace at most 1 GiB

int rbf_slots(int32_t M, int32_t max_points) {
  const size_t per = rbf_slot_doubles(max_points) * sizeof(double);
  size_t k = kRbfSlotBudget / per;
  if (k < 1) k = 1;
  if (k > (size_t)kRbfMaxSlots) k = kRbfMaxSlots;
  return M < (int32_t)k ? (int)M : (int)k;
}

int check_width(double eps) {
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(VESNET_ERR_INVALID_ARGUMENT, "width must be > 0 and finite (got %g)", eps);
  return VESNET_OK;
}

}  // namespace

extern "C" int vesnet_near_layers(const double* X, const double* w, const int32_t* off, int32_t M, int32_t P,
                                  double* layers, void* stream) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if (P == 0) return ok();
  if (!X || !w || !off || !layers) return fail(VESNET_ERR_INVALID_ARGUMENT, "X, weights, offsets and layers must be non-NULL");
  const size_t vb = (size_t)2 * P * sizeof(double), lb = (size_t)10 * P * sizeof(double);
  if (overlaps(layers, lb, X, vb) || overlaps(layers, lb, w, (size_t)P * sizeof(double)) ||
      overlaps(layers, lb, off, (size_t)(M + 1) * sizeof(int32_t)))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "layers overlap an input");
  hipError_t e = launch_near_layers(X, w, off, M, P, layers, stream);
  if (e != hipSuccess) return hip_fail(e, "near layers launch");
  return ok();
}

extern "C" size_t vesnet_rbf_workspace_bytes(int32_t max_points, int32_t M) {
  if (max_points < 1 || max_points > kRbfMaxPoints || M < 1) return 0;
  return (size_t)rbf_slots(M, max_points) * rbf_slot_doubles(max_points) * sizeof(double);
}

extern "C" int vesnet_rbf_fit(const double* layers, const double* vel, const double* w, const int32_t* off, int32_t M,
                              int32_t P, int32_t max_points, double width, double* coeffs, void* ws, size_t ws_bytes,
                              void* stream) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if ((rc = check_width(width))) return rc;
  if (P == 0) return ok();
  if (max_points < 1 || max_points > kRbfMaxPoints)
    return fail(VESNET_ERR_UNSUPPORTED, "max_points = %d outside 1..%d", max_points, kRbfMaxPoints);
  if (!layers || !vel || !w || !off || !coeffs)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "layers, velocities, weights, offsets and coeffs must be non-NULL");
  const size_t slot = rbf_slot_doubles(max_points) * sizeof(double);
  if (!ws || ws_bytes < slot)
    return fail(VESNET_ERR_WORKSPACE, "workspace of %zu bytes is below one slot (%zu bytes)", ws_bytes, slot);
  const size_t lb = (size_t)10 * P * sizeof(double);
  if (overlaps(coeffs, lb, layers, lb) || overlaps(coeffs, lb, vel, lb) ||
      overlaps(coeffs, lb, w, (size_t)P * sizeof(double)) || overlaps(coeffs, lb, off, (size_t)(M + 1) * sizeof(int32_t)) ||
      overlaps(coeffs, lb, ws, ws_bytes) || overlaps(ws, ws_bytes, layers, lb) || overlaps(ws, ws_bytes, vel, lb))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "coeffs or workspace overlap another array");
  size_t slots = ws_bytes / slot;
  if (slots > (size_t)kRbfMaxSlots) slots = kRbfMaxSlots;
  if (slots > (size_t)M) slots = (size_t)M;
  hipError_t e = launch_rbf_fit(layers, vel, w, off, M, P, max_points, width, coeffs, static_cast<double*>(ws),
                                (int)slots, stream);
  if (e != hipSuccess) return hip_fail(e, "rbf fit launch");
  return ok();
}

extern "C" int vesnet_rbf_eval_near(const double* layers, const double* coeffs, const double* w, const int32_t* off,
                                    int32_t M, int32_t P, double width, const double* targets, int32_t n_targets,
                                    const int32_t* near_pairs, const int32_t* near_count, int32_t near_capacity,
                                    double* out, void* stream) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if ((rc = check_width(width))) return rc;
  if (n_targets < 0 || n_targets > kMaxPoints) return fail(VESNET_ERR_INVALID_ARGUMENT, "n_targets = %d", n_targets);
  if (near_capacity < 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "near_capacity = %d < 0", near_capacity);
  if (P == 0 || n_targets == 0 || near_capacity == 0) return ok();
  if (!layers || !coeffs || !w || !off || !targets || !near_pairs || !near_count || !out)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "a required pointer is NULL");
  const size_t ob = (size_t)2 * n_targets * sizeof(double), lb = (size_t)10 * P * sizeof(double);
  if (overlaps(out, ob, layers, lb) || overlaps(out, ob, coeffs, lb) || overlaps(out, ob, targets, ob) ||
      overlaps(out, ob, w, (size_t)P * sizeof(double)) || overlaps(out, ob, near_pairs, (size_t)2 * near_capacity * sizeof(int32_t)) ||
      overlaps(out, ob, near_count, sizeof(int32_t)) || overlaps(out, ob, off, (size_t)(M + 1) * sizeof(int32_t)))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "out overlaps an input");
  hipError_t e = launch_rbf_eval_near(layers, coeffs, w, off, M, P, width, targets, n_targets, near_pairs, near_count,
                                      near_capacity, out, stream);
  if (e != hipSuccess) return hip_fail(e, "rbf evaluation launch");
  return ok();
}

// ============================================================================ treecode far field

namespace {
constexpr int32_t kTreeMaxOrder = 48;
constexpr int32_t kTreeMaxDepth = 10;
}  // namespace

extern "C" int32_t vesnet_treecode_default_depth(int32_t P) {
  int32_t L = 0;
  while (L < kTreeMaxDepth && (int64_t)P > (int64_t)64 << (2 * L)) ++L;
  return L;
}

extern "C" size_t vesnet_treecode_workspace_bytes(int32_t P, int32_t depth, int32_t order) {
  if (P < 0 || P > kMaxPoints || depth < 0 || depth > kTreeMaxDepth || order < 1 || order > kTreeMaxOrder) return 0;
  return treecode_workspace_bytes(P, depth, order);
}

extern "C" int vesnet_farfield_treecode(const double* X, const double* f, const double* w, const int32_t* off, int32_t M,
                                        int32_t P, double mu, int32_t order, int32_t depth, double* out, void* ws,
                                        size_t ws_bytes, void* stream) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if ((rc = check_mu(mu))) return rc;
  if (order < 1 || order > kTreeMaxOrder)
    return fail(VESNET_ERR_UNSUPPORTED, "order = %d outside 1..%d", order, kTreeMaxOrder);
  if (depth < 0 || depth > kTreeMaxDepth)
    return fail(VESNET_ERR_UNSUPPORTED, "depth = %d outside 0..%d", depth, kTreeMaxDepth);
  if (P == 0) return ok();
  if (!X || !f || !w || !off || !out) return fail(VESNET_ERR_INVALID_ARGUMENT, "a required pointer is NULL");
  if ((rc = check_workspace(ws, ws_bytes, treecode_workspace_bytes(P, depth, order)))) return rc;
  const size_t vb = (size_t)2 * P * sizeof(double);
  if (overlaps(out, vb, X, vb) || overlaps(out, vb, f, vb) || overlaps(out, vb, w, (size_t)P * sizeof(double)) ||
      overlaps(out, vb, off, (size_t)(M + 1) * sizeof(int32_t)) || overlaps(out, vb, ws, ws_bytes) ||
      overlaps(ws, ws_bytes, X, vb) || overlaps(ws, ws_bytes, f, vb) || overlaps(ws, ws_bytes, w, (size_t)P * sizeof(double)))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "out or workspace overlap another array");
  hipError_t e = launch_treecode(X, f, w, off, M, P, 1.0 / (4.0 * kPi * mu), order, depth, out, ws, stream);
  if (e != hipSuccess) return hip_fail(e, "treecode launch");
  return ok();
}

extern "C" int32_t vesnet_fmm_default_depth(int32_t P, int32_t order) {
  // leaves of about 64 points, or 128 above order 32, where M2L (p^2 per box pair) outweighs the direct part
  const int64_t cap = order > 32 ? 128 : 64;
  int32_t L = 0;
  while (L < kTreeMaxDepth && (int64_t)P > cap << (2 * L)) ++L;
  return L;
}

extern "C" size_t vesnet_fmm_workspace_bytes(int32_t P, int32_t depth, int32_t order) {
  if (P < 0 || P > kMaxPoints || depth < 0 || depth > kTreeMaxDepth || order < 1 || order > kTreeMaxOrder) return 0;
  return fmm_workspace_bytes(P, depth, order);
}

extern "C" int vesnet_farfield_fmm(const double* X, const double* f, const double* w, const int32_t* off, int32_t M,
                                   int32_t P, double mu, int32_t order, int32_t depth, double* out, void* ws,
                                   size_t ws_bytes, void* stream) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if ((rc = check_mu(mu))) return rc;
  if (order < 1 || order > kTreeMaxOrder)
    return fail(VESNET_ERR_UNSUPPORTED, "order = %d outside 1..%d", order, kTreeMaxOrder);
  if (depth < 0 || depth > kTreeMaxDepth)
    return fail(VESNET_ERR_UNSUPPORTED, "depth = %d outside 0..%d", depth, kTreeMaxDepth);
  if (P == 0) return ok();
  if (!X || !f || !w || !off || !out) return fail(VESNET_ERR_INVALID_ARGUMENT, "a required pointer is NULL");
  if ((rc = check_workspace(ws, ws_bytes, fmm_workspace_bytes(P, depth, order)))) return rc;
  const size_t vb = (size_t)2 * P * sizeof(double);
  if (overlaps(out, vb, X, vb) || overlaps(out, vb, f, vb) || overlaps(out, vb, w, (size_t)P * sizeof(double)) ||
      overlaps(out, vb, off, (size_t)(M + 1) * sizeof(int32_t)) || overlaps(out, vb, ws, ws_bytes) ||
      overlaps(ws, ws_bytes, X, vb) || overlaps(ws, ws_bytes, f, vb) || overlaps(ws, ws_bytes, w, (size_t)P * sizeof(double)))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "out or workspace overlap another array");
  hipError_t e = launch_fmm(X, f, w, off, M, P, 1.0 / (4.0 * kPi * mu), order, depth, out, ws, stream);
  if (e != hipSuccess) return hip_fail(e, "fast multipole launch");
  return ok();
}

extern "C" size_t vesnet_fmm_nearmasked_workspace_bytes(int32_t P, int32_t M, int32_t depth, int32_t order) {
  if (P < 0 || P > kMaxPoints || M < 0 || depth < 0 || depth > kTreeMaxDepth || order < 1 || order > kTreeMaxOrder)
    return 0;
  return fmm_near_workspace_bytes(P, M > 0 ? M : 1, depth, order);
}

extern "C" int vesnet_farfield_fmm_nearmasked(const double* X, const double* f, const double* w, const int32_t* off,
                                              int32_t M, int32_t P, double mu, int32_t order, int32_t depth,
                                              double* out, int32_t* near_pairs, int32_t near_capacity,
                                              int32_t* near_count, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_sizes(P, M);
  if (rc) return rc;
  if ((rc = check_mu(mu))) return rc;
  if (order < 1 || order > kTreeMaxOrder)
    return fail(VESNET_ERR_UNSUPPORTED, "order = %d outside 1..%d", order, kTreeMaxOrder);
  if (depth < 0 || depth > kTreeMaxDepth)
    return fail(VESNET_ERR_UNSUPPORTED, "depth = %d outside 0..%d", depth, kTreeMaxDepth);
  if (!near_count) return fail(VESNET_ERR_INVALID_ARGUMENT, "near_count is NULL");
  if (near_capacity < 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "near_capacity = %d < 0", near_capacity);
  if (near_capacity > 0 && !near_pairs)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "near_pairs is NULL but near_capacity = %d", near_capacity);
  if (P == 0) {
    hipError_t e = launch_zero_count(near_count, stream);
    return e == hipSuccess ? ok() : hip_fail(e, "near count clear");
  }
  if (!X || !f || !w || !off || !out) return fail(VESNET_ERR_INVALID_ARGUMENT, "a required pointer is NULL");
  if ((rc = check_workspace(ws, ws_bytes, fmm_near_workspace_bytes(P, M, depth, order)))) return rc;
  const size_t vb = (size_t)2 * P * sizeof(double);
  const size_t pb = (size_t)2 * near_capacity * sizeof(int32_t);
  if (overlaps(out, vb, X, vb) || overlaps(out, vb, f, vb) || overlaps(out, vb, w, (size_t)P * sizeof(double)) ||
      overlaps(out, vb, off, (size_t)(M + 1) * sizeof(int32_t)) || overlaps(out, vb, ws, ws_bytes) ||
      overlaps(ws, ws_bytes, X, vb) || overlaps(ws, ws_bytes, f, vb) || overlaps(ws, ws_bytes, w, (size_t)P * sizeof(double)))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "out or workspace overlap another array");
  if (overlaps(near_pairs, pb, out, vb) || overlaps(near_pairs, pb, ws, ws_bytes) ||
      overlaps(near_count, sizeof(int32_t), out, vb) || overlaps(near_count, sizeof(int32_t), ws, ws_bytes) ||
      overlaps(near_count, sizeof(int32_t), near_pairs, pb) || overlaps(near_pairs, pb, X, vb) ||
      overlaps(near_pairs, pb, f, vb))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "near-field outputs overlap other arrays");
  hipError_t e = launch_fmm_nearmasked(X, f, w, off, M, P, 1.0 / (4.0 * kPi * mu), order, depth, out, near_pairs,
                                       near_capacity, near_count, ws, stream);
  if (e != hipSuccess) return hip_fail(e, "fast multipole near-masked launch");
  return ok();
}

// ============================================================================ near-field masked

extern "C" int vesnet_farfield_stokeslet_nearmasked(const double* targets, const double* sources, const double* f,
                                                    const double* w, const int32_t* off, int32_t M, int32_t P,
                                                    double mu, double* out, int32_t* near_pairs,
                                                    int32_t near_capacity, int32_t* near_count, int prec,
                                                    const vesnet_tile_config* cfg, void* ws, size_t ws_bytes,
                                                    void* stream) {
  int rc = check_forward_args(targets, sources, f, w, off, M, P, out, prec, ws, ws_bytes, true, true);
  if (rc) return rc;
  if ((rc = check_mu(mu))) return rc;
  if (!near_count) return fail(VESNET_ERR_INVALID_ARGUMENT, "near_count is NULL");
  if (near_capacity < 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "near_capacity = %d < 0", near_capacity);
  if (near_capacity > 0 && !near_pairs)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "near_pairs is NULL but near_capacity = %d", near_capacity);
  if (P > 0 && !out) return fail(VESNET_ERR_INVALID_ARGUMENT, "out is NULL");
  const size_t vb = (size_t)2 * P * sizeof(double);
  const size_t pb = (size_t)2 * near_capacity * sizeof(int32_t);
  if (overlaps(near_pairs, pb, out, vb) || overlaps(near_pairs, pb, ws, ws_bytes) ||
      overlaps(near_count, sizeof(int32_t), out, vb) || overlaps(near_count, sizeof(int32_t), ws, ws_bytes) ||
      overlaps(near_count, sizeof(int32_t), near_pairs, pb) || overlaps(near_pairs, pb, targets, vb) ||
      overlaps(near_pairs, pb, sources, vb) || overlaps(near_pairs, pb, f, vb))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "near-field outputs overlap other arrays");
  Shape s;
  if ((rc = resolve_shape(cfg, P, M, prec, &s))) return rc;
  if (s.T > 2) s.T = 2;
  if (P > 0 && (rc = check_workspace(ws, ws_bytes, forward_bytes(P, M, prec, s)))) return rc;
  PreparedView pv{};
  double* partial = nullptr;
  if (P > 0) {
    if ((rc = vesnet_farfield_prepare(sources, f, w, off, M, P, prec, ws, ws_bytes, stream))) return rc;
    char* cur = aligned_base(ws);
    pv = carve_prepared(cur, P, M, prec, fwd_forces(prec));
    partial = s.splits > 1 ? reinterpret_cast<double*>(cur) : nullptr;
  }
  const double scale = 1.0 / (4.0 * kPi * mu);
  hipError_t e = launch_forward_near(prec, s.T, s.staging == 2, s.splits, targets, P, M, pv, scale, out, partial,
                                     near_count, near_pairs, near_capacity, stream);
  if (e != hipSuccess) return hip_fail(e, "near-masked forward launch");
  return ok();
}

// ============================================================================ batched

namespace {

size_t plan_bytes(int32_t S) { return align_up((size_t)(4 * (size_t)S + 2) * sizeof(int32_t)); }

// The batched symmetric form's tables: per-suspension (cycles, blocks, exponent), first units and points.
size_t symb_bytes(int32_t S) {
  return align_up((size_t)S * sizeof(int4)) + 2 * align_up((size_t)(S + 1) * sizeof(int32_t)) +
         align_up((size_t)S * sizeof(int2));
}

SymBatchView carve_symb(char*& cur, int32_t S) {
  SymBatchView bv;
  bv.stab = reinterpret_cast<int4*>(cur);
  cur += align_up((size_t)S * sizeof(int4));
  bv.ustart = reinterpret_cast<int32_t*>(cur);
  cur += align_up((size_t)(S + 1) * sizeof(int32_t));
  bv.pstart = reinterpret_cast<int32_t*>(cur);
  cur += align_up((size_t)(S + 1) * sizeof(int32_t));
  bv.vr = reinterpret_cast<int2*>(cur);
  cur += align_up((size_t)S * sizeof(int2));
  return bv;
}

PlanView carve_plan(char*& cur, int32_t S) {
  PlanView pl;
  int32_t* p = reinterpret_cast<int32_t*>(cur);
  pl.psz = p;
  pl.nitems = p + S;
  pl.order = p + 2 * S;
  pl.item_start = p + 3 * S;
  pl.counter = p + 4 * S + 1;
  cur += plan_bytes(S);
  return pl;
}

int num_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

int check_batched_args(const double* targets, const double* sources, const double* f, const double* w,
                       const int32_t* off, int32_t M, int32_t P, const int32_t* sus_off, int32_t S, const double* mu,
                       double* out, int prec, void* ws, size_t ws_bytes) {
  int rc = check_forward_args(targets, sources, f, w, off, M, P, out, prec, ws, ws_bytes, true, true);
  if (rc) return rc;
  if (S < 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "n_suspensions = %d < 0", S);
  if (P > 0 && S == 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "points given but no suspensions");
  if (P > 0 && (!sus_off || !mu)) return fail(VESNET_ERR_INVALID_ARGUMENT, "suspension_offsets and mu must be non-NULL");
  if (P > 0 && !out) return fail(VESNET_ERR_INVALID_ARGUMENT, "out is NULL");
  if (out && overlaps(out, (size_t)2 * P * sizeof(double), mu, (size_t)S * sizeof(double)))
    return fail(VESNET_ERR_INVALID_ARGUMENT, "out overlaps mu");
  return VESNET_OK;
}

// The batched call takes the symmetric form when the precision is compensated, targets and sources are
// one array and the call does not ask for the direct form (or matrix-core accumulation).
bool batched_symmetric(const double* targets, const double* sources, int prec, const Shape& s) {
  return prec == P32C && targets == sources && s.accumulate == 1 && s.pair != 1;
}

// Targets per thread and workgroups of the batched symmetric form: the caller's targets_per_thread when
// pair_form 2 asks for it (1, 2, 3 or 4), else the single-suspension default for the total point count;
// blocks_per_cu when the caller sets it, else as many units as one compute unit holds.
int batched_symmetric_shape(const vesnet_tile_config* cfg, int32_t P, int32_t M, int32_t S, const Shape& s,
                            int* T, int* grid) {
  int t = s.symT ? s.symT : 1;
  if (t == 8) t = 4;
  if (cfg && cfg->pair_form == 2 && cfg->targets_per_thread) t = cfg->targets_per_thread;
  if (t < 1 || t > 4)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "targets_per_thread of the batched symmetric form must be 1, 2, 3 or 4");
  while (t < 4 && symb_max_units(P, M, S, t) > (int64_t)INT32_MAX) ++t;
  if (symb_max_units(P, M, S, t) > (int64_t)INT32_MAX)
    return fail(VESNET_ERR_UNSUPPORTED, "too many points for the batched symmetric form; use pair_form 1");
  const int bpc = cfg && cfg->blocks_per_cu ? cfg->blocks_per_cu : symb_units_per_cu(t);
  *T = t;
  *grid = num_cus() * bpc;
  return VESNET_OK;
}

int enqueue_batched(const double* targets, const double* sources, const double* f, const double* w,
                    const int32_t* off, int32_t M, int32_t P, const int32_t* sus_off, int32_t S, const double* mu,
                    double* out, int prec, const Shape& s, const vesnet_tile_config* cfg, void* ws, void* stream) {
  char* cur = aligned_base(ws);
  PreparedView pv = carve_prepared(cur, P, M, prec, fwd_forces(prec));
  PlanView pl = carve_plan(cur, S);
  hipError_t e = launch_prepare(prec, sources, f, w, off, M, P, pv, stream);
  if (e != hipSuccess) return hip_fail(e, "prepare launch");
  if (batched_symmetric(targets, sources, prec, s)) {
    int T = 0, grid = 0;
    int rc = batched_symmetric_shape(cfg, P, M, S, s, &T, &grid);
    if (rc) return rc;
    SymmetricView sv = carve_symmetric(cur, P, M);
    SymBatchView bv = carve_symb(cur, S);
    e = launch_batched_symmetric(T, grid, P, M, pv, sv, bv, sus_off, off, S, mu, out, stream);
    if (e != hipSuccess) return hip_fail(e, "batched symmetric launch");
    return VESNET_OK;
  }
  e = launch_plan(sus_off, S, M, pv, s.T * s.B, pl, stream);
  if (e != hipSuccess) return hip_fail(e, "plan launch");
  const int grid = num_cus() * s.bpc;
  e = launch_batched(prec, s.T, s.B, s.staging == 2, grid, targets, P, M, pv, sus_off, mu, S, pl, out, stream);
  if (e != hipSuccess) return hip_fail(e, "batched launch");
  return VESNET_OK;
}

}  // namespace

extern "C" size_t vesnet_batched_workspace_bytes(int32_t P, int32_t M, int32_t S, int prec) {
  if (check_sizes(P, M) || !valid_precision(prec) || S < 0) return 0;
  size_t b = kAlign + prepared_bytes(P, M, prec, fwd_forces(prec)) + plan_bytes(S);
  if (prec == P32C) b += symmetric_bytes(P, M) + symb_bytes(S);
  return b;
}

extern "C" int vesnet_farfield_stokeslet_batched(const double* targets, const double* sources, const double* f,
                                                 const double* w, const int32_t* off, int32_t M, int32_t P,
                                                 const int32_t* sus_off, int32_t S, const double* mu, double* out,
                                                 int prec, const vesnet_tile_config* cfg, void* ws, size_t ws_bytes,
                                                 void* stream) {
  int rc = check_batched_args(targets, sources, f, w, off, M, P, sus_off, S, mu, out, prec, ws, ws_bytes);
  if (rc) return rc;
  if (P == 0) return ok();
  Shape s;
  if ((rc = resolve_shape(cfg, P, M, prec, &s))) return rc;
  if ((rc = check_workspace(ws, ws_bytes, vesnet_batched_workspace_bytes(P, M, S, prec)))) return rc;
  if ((rc = enqueue_batched(targets, sources, f, w, off, M, P, sus_off, S, mu, out, prec, s, cfg, ws, stream)))
    return rc;
  return ok();
}

struct vesnet_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" int vesnet_graph_create_batched(const double* targets, const double* sources, const double* f,
                                           const double* w, const int32_t* off, int32_t M, int32_t P,
                                           const int32_t* sus_off, int32_t S, const double* mu, double* out,
                                           int prec, const vesnet_tile_config* cfg, void* ws, size_t ws_bytes,
                                           vesnet_graph** graph) {
  if (!graph) return fail(VESNET_ERR_INVALID_ARGUMENT, "graph is NULL");
  *graph = nullptr;
  int rc = check_batched_args(targets, sources, f, w, off, M, P, sus_off, S, mu, out, prec, ws, ws_bytes);
  if (rc) return rc;
  if (P == 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "nothing to capture (n_points = 0)");
  Shape s;
  if ((rc = resolve_shape(cfg, P, M, prec, &s))) return rc;
  if ((rc = check_workspace(ws, ws_bytes, vesnet_batched_workspace_bytes(P, M, S, prec)))) return rc;
  if (batched_symmetric(targets, sources, prec, s)) {
    // resolve the symmetric shape (and its occupancy query) before the capture begins
    int T = 0, grid = 0;
    if ((rc = batched_symmetric_shape(cfg, P, M, S, s, &T, &grid))) return rc;
  }
  hipStream_t st = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(st);
    return hip_fail(e, "hipStreamBeginCapture");
  }
  rc = enqueue_batched(targets, sources, f, w, off, M, P, sus_off, S, mu, out, prec, s, cfg, ws, st);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(st);
    return rc;
  }
  if (e2 != hipSuccess) {
    (void)hipStreamDestroy(st);
    return hip_fail(e2, "hipStreamEndCapture");
  }
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(st);
    return hip_fail(e, "hipGraphInstantiate");
  }
  (void)hipStreamDestroy(st);
  vesnet_graph* h = new vesnet_graph{g, ex};
  *graph = h;
  return ok();
}

extern "C" int vesnet_graph_launch(vesnet_graph* graph, void* stream) {
  if (!graph) return fail(VESNET_ERR_INVALID_ARGUMENT, "graph is NULL");
  hipError_t e = hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ok();
}

extern "C" int vesnet_graph_destroy(vesnet_graph* graph) {
  if (!graph) return ok();
  (void)hipGraphExecDestroy(graph->exec);
  (void)hipGraphDestroy(graph->graph);
  delete graph;
  return ok();
}

// ============================================================================ adjoint

namespace {

// Backward launch shape: the forward default (one point per thread, 256 threads, LDS
// staging, enough source chunks to give every SIMD many waves).
Shape backward_shape(int32_t P, int32_t M, int prec) {
  Shape s = default_shape(P, M, prec);
  s.T = 1;
  s.B = 256;
  return s;
}

size_t backward_bytes(int32_t P, int32_t M, int prec) {
  const Shape s = backward_shape(P, M, prec);
  size_t b = kAlign + 2 * prepared_bytes(P, M, prec);
  if (s.splits > 1) b += align_up((size_t)6 * s.splits * P * sizeof(double));
  return b;
}

}  // namespace

extern "C" size_t vesnet_backward_workspace_bytes(int32_t P, int32_t M, int prec) {
  if (check_sizes(P, M) || (prec != VESNET_FP64 && prec != VESNET_FP32_COMPENSATED)) return 0;
  return backward_bytes(P, M, prec);
}

extern "C" int vesnet_farfield_stokeslet_backward(const double* targets, const double* sources, const double* f,
                                                  const double* w, const int32_t* off, int32_t M, int32_t P,
                                                  double mu, const double* gout, double* grad_t, double* grad_s,
                                                  double* grad_f, double* grad_w, int prec, void* ws,
                                                  size_t ws_bytes, void* stream) {
  int rc = check_forward_args(targets, sources, f, w, off, M, P, nullptr, prec, ws, ws_bytes, true, true);
  if (rc) return rc;
  if (prec == VESNET_FP32_NAIVE)
    return fail(VESNET_ERR_UNSUPPORTED, "the backward pass supports VESNET_FP64 and VESNET_FP32_COMPENSATED only");
  if ((rc = check_mu(mu))) return rc;
  if (P == 0) return ok();
  if (!gout) return fail(VESNET_ERR_INVALID_ARGUMENT, "grad_out is NULL");
  const size_t vb = (size_t)2 * P * sizeof(double), sb = (size_t)P * sizeof(double);
  const void* ins[] = {targets, sources, f, gout, off, ws};
  const size_t inb[] = {vb, vb, vb, vb, (size_t)(M + 1) * sizeof(int32_t), ws_bytes};
  const void* outs[] = {grad_t, grad_s, grad_f, grad_w};
  const size_t outb[] = {vb, vb, vb, sb};
  for (int a = 0; a < 4; ++a) {
    if (!outs[a]) continue;
    for (int b = 0; b < 6; ++b)
      if (overlaps(outs[a], outb[a], ins[b], inb[b]))
        return fail(VESNET_ERR_INVALID_ARGUMENT, "gradient output %d overlaps an input or the workspace", a);
    if (overlaps(outs[a], outb[a], w, sb))
      return fail(VESNET_ERR_INVALID_ARGUMENT, "gradient output %d overlaps arc_weights", a);
    for (int b = a + 1; b < 4; ++b)
      if (overlaps(outs[a], outb[a], outs[b], outb[b]))
        return fail(VESNET_ERR_INVALID_ARGUMENT, "gradient outputs %d and %d overlap", a, b);
  }
  if (!grad_t && !grad_s && !grad_f && !grad_w) return ok();
  if ((rc = check_workspace(ws, ws_bytes, vesnet_backward_workspace_bytes(P, M, prec)))) return rc;
  char* cur = aligned_base(ws);
  PreparedView pvS = carve_prepared(cur, P, M, prec);
  PreparedView pvT = carve_prepared(cur, P, M, prec);
  const Shape sh = backward_shape(P, M, prec);
  double* part_t = nullptr;
  double* part_s = nullptr;
  if (sh.splits > 1) {
    part_t = reinterpret_cast<double*>(cur);
    part_s = part_t + (size_t)2 * sh.splits * P;
  }
  hipError_t e = hipSuccess;
  if (grad_t) e = launch_prepare(prec, sources, f, w, off, M, P, pvS, stream);
  if (e == hipSuccess && (grad_s || grad_f || grad_w)) e = launch_prepare(prec, targets, gout, nullptr, off, M, P, pvT, stream);
  if (e != hipSuccess) return hip_fail(e, "backward prepare launch");
  const double scale = 1.0 / (4.0 * kPi * mu);
  e = launch_backward(prec, sh.T, sh.splits, targets, sources, f, w, gout, P, M, pvS, pvT, scale, grad_t, grad_s,
                      grad_f, grad_w, part_t, part_s, stream);
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return ok();
}

// Adjoint for one point array (targets = sources = points, positions differentiated in both roles).
namespace {

// Targets per thread of the symmetric adjoint: the forward's rule, one when the problem is small,
// four when the units of the smaller choice would not fit one launch; 0 when none fits (the gathers).
int sym_bwd_T(int32_t P, int32_t M) {
  const int T = sym_default_T(P, 3);
  if (sym_fits(P, M, T ? T : 1)) return T ? T : 1;
  return sym_fits(P, M, 4) ? 4 : 0;
}

// Targets per thread of the float64 symmetric adjoint: two where they give at least four units per compute
// unit (200 VGPRs, two wavefronts per SIMD: 69.4 ms against 74.6 ms at one on 2000 x 128, equal at
// 512 x 64), else one (126 VGPRs); two when the units of one would not fit a launch; 0: the gathers.
int sym64_bwd_T(int32_t P, int32_t M) {
  const int T = sym_default_T(P, 2);
  if (sym_fits(P, M, T ? T : 1)) return T ? T : 1;
  return sym_fits(P, M, 2) ? 2 : 0;
}

int points_bwd_T(int32_t P, int32_t M, int prec) {
  return prec == VESNET_FP32_COMPENSATED ? sym_bwd_T(P, M) : prec == VESNET_FP64 ? sym64_bwd_T(P, M) : 0;
}

// The symmetric pass (FP32-compensated and FP64): two prepared regions with forces, the cycle tables
// and a [2][P] buffer for the position gradient when the caller does not ask for it; otherwise the
// gathers' workspace and a [2][P] buffer for the source-role gradient.
size_t backward_points_bytes(int32_t P, int32_t M, int prec) {
  const size_t vec = align_up((size_t)2 * P * sizeof(double));
  if (points_bwd_T(P, M, prec))
    return kAlign + 2 * prepared_bytes(P, M, prec, true) + symmetric_bytes(P, M) + vec;
  return backward_bytes(P, M, prec) + vec;
}

}  // namespace

extern "C" size_t vesnet_backward_points_workspace_bytes(int32_t P, int32_t M, int prec) {
  if (check_sizes(P, M) || (prec != VESNET_FP64 && prec != VESNET_FP32_COMPENSATED)) return 0;
  return backward_points_bytes(P, M, prec);
}

extern "C" int vesnet_farfield_stokeslet_backward_points(const double* points, const double* f, const double* w,
                                                         const int32_t* off, int32_t M, int32_t P, double mu,
                                                         const double* gout, double* grad_points, double* grad_f,
                                                         double* grad_w, int prec, void* ws, size_t ws_bytes,
                                                         void* stream) {
  int rc = check_forward_args(points, points, f, w, off, M, P, nullptr, prec, ws, ws_bytes, true, true);
  if (rc) return rc;
  if (prec == VESNET_FP32_NAIVE)
    return fail(VESNET_ERR_UNSUPPORTED, "the backward pass supports VESNET_FP64 and VESNET_FP32_COMPENSATED only");
  if ((rc = check_mu(mu))) return rc;
  if (P == 0) return ok();
  if (!gout) return fail(VESNET_ERR_INVALID_ARGUMENT, "grad_out is NULL");
  const size_t vb = (size_t)2 * P * sizeof(double), sb = (size_t)P * sizeof(double);
  const void* ins[] = {points, f, gout, off, ws, w};
  const size_t inb[] = {vb, vb, vb, (size_t)(M + 1) * sizeof(int32_t), ws_bytes, sb};
  const void* outs[] = {grad_points, grad_f, grad_w};
  const size_t outb[] = {vb, vb, sb};
  for (int a = 0; a < 3; ++a) {
    if (!outs[a]) continue;
    for (int b = 0; b < 6; ++b)
      if (overlaps(outs[a], outb[a], ins[b], inb[b]))
        return fail(VESNET_ERR_INVALID_ARGUMENT, "gradient output %d overlaps an input or the workspace", a);
    for (int b = a + 1; b < 3; ++b)
      if (overlaps(outs[a], outb[a], outs[b], outb[b]))
        return fail(VESNET_ERR_INVALID_ARGUMENT, "gradient outputs %d and %d overlap", a, b);
  }
  if (!grad_points && !grad_f && !grad_w) return ok();
  if ((rc = check_workspace(ws, ws_bytes, backward_points_bytes(P, M, prec)))) return rc;
  const double scale = 1.0 / (4.0 * kPi * mu);
  char* cur = aligned_base(ws);
  hipError_t e = hipSuccess;
  const int symT = points_bwd_T(P, M, prec);
  if (symT) {
    // one symmetric pass: (points, w f) and (points, g) records, cycles and their sums of g
    PreparedView pvF = carve_prepared(cur, P, M, prec, true);
    PreparedView pvG = carve_prepared(cur, P, M, prec, true);
    SymmetricView sv = carve_symmetric(cur, P, M);
    double* gx = grad_points ? grad_points : reinterpret_cast<double*>(cur);
    e = launch_prepare(prec, points, f, w, off, M, P, pvF, stream);
    if (e == hipSuccess) e = launch_prepare(prec, points, gout, nullptr, off, M, P, pvG, stream);
    if (e != hipSuccess) return hip_fail(e, "backward prepare launch");
    e = prec == VESNET_FP64
            ? launch_backward_symmetric64(symT, P, M, pvF, pvG, sv, reinterpret_cast<double*>(sv.acc), f, w, scale,
                                          gx, grad_f, grad_w, stream)
            : launch_backward_symmetric(symT, P, M, pvF, pvG, sv, reinterpret_cast<double*>(sv.acc), f, w, scale, gx,
                                        grad_f, grad_w, stream);
    if (e != hipSuccess) return hip_fail(e, "symmetric backward launch");
    return ok();
  }
  // two gathers (targets, then sources), whose position gradients are added
  PreparedView pvS = carve_prepared(cur, P, M, prec);
  PreparedView pvT = carve_prepared(cur, P, M, prec);
  const Shape sh = backward_shape(P, M, prec);
  double* part_t = nullptr;
  double* part_s = nullptr;
  if (sh.splits > 1) {
    part_t = reinterpret_cast<double*>(cur);
    part_s = part_t + (size_t)2 * sh.splits * P;
    cur += align_up((size_t)6 * sh.splits * P * sizeof(double));
  }
  double* grad_s = grad_points ? reinterpret_cast<double*>(cur) : nullptr;
  if (grad_points) e = launch_prepare(prec, points, f, w, off, M, P, pvS, stream);
  if (e == hipSuccess) e = launch_prepare(prec, points, gout, nullptr, off, M, P, pvT, stream);
  if (e != hipSuccess) return hip_fail(e, "backward prepare launch");
  e = launch_backward(prec, sh.T, sh.splits, points, points, f, w, gout, P, M, pvS, pvT, scale, grad_points, grad_s,
                      grad_f, grad_w, part_t, part_s, stream);
  if (e == hipSuccess && grad_points) e = launch_add_f64(grad_points, grad_s, (int64_t)2 * P, stream);
  if (e != hipSuccess) return hip_fail(e, "backward launch");
  return ok();
}

// ============================================================================ tuning

extern "C" int vesnet_autotune(const double* targets, const double* sources, const double* f, const double* w,
                               const int32_t* off, int32_t M, int32_t P, int batched, const int32_t* sus_off,
                               int32_t S, const double* mu_dev, double mu_host, double* out, int prec, int repeats,
                               void* ws, size_t ws_bytes, void* stream, vesnet_tile_config* best, float* best_ms) {
  if (!best) return fail(VESNET_ERR_INVALID_ARGUMENT, "best is NULL");
  int rc;
  if (batched) rc = check_batched_args(targets, sources, f, w, off, M, P, sus_off, S, mu_dev, out, prec, ws, ws_bytes);
  else rc = check_forward_args(targets, sources, f, w, off, M, P, out, prec, ws, ws_bytes, true, true);
  if (rc) return rc;
  if (!batched && (rc = check_mu(mu_host))) return rc;
  if (P == 0) return fail(VESNET_ERR_INVALID_ARGUMENT, "nothing to tune (n_points = 0)");
  if (!out) return fail(VESNET_ERR_INVALID_ARGUMENT, "out is NULL");
  if (repeats < 1) repeats = 1;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  // Direct-form shapes (pair_form 1 where the symmetric form could run, so that each candidate is the
  // shape it names) and, for one compensated point array, the symmetric form's targets per thread
  // (batched: also its workgroups per compute unit, 0 = as many as fit).
  const bool sym_ok = (prec == VESNET_FP32_COMPENSATED || (prec == VESNET_FP64 && !batched)) && targets == sources;
  const int direct = sym_ok ? 1 : 0;
  std::vector<vesnet_tile_config> cands;
  for (int acc : {1, 2}) {
    if (acc == 2 && (batched || prec != VESNET_FP32_COMPENSATED)) continue;
    for (int stg : {1, 2})
      for (int T : {1, 2, 4})
        for (int B : {64, 128, 256}) {
          if (batched) {
            for (int bpc : {1, 2, 4, 8}) cands.push_back({T, B, 1, bpc, stg, acc, direct});
          } else {
            for (int sp : {1, 2, 4, 8, 16}) {
              if (sp > std::max(1, M)) continue;
              const Shape sh{T, B, sp, 1, stg, acc, direct};
              if (forward_bytes(P, M, prec, sh) > ws_bytes) continue;
              cands.push_back({T, B, sp, 1, stg, acc, direct});
            }
          }
        }
  }
  if (sym_ok) {
    for (int T : {1, 2, 3, 4, 8}) {
      if (batched) {
        if (T == 8) continue;
        for (int bpc : {0, 2, 4, 8}) cands.push_back({T, 0, 0, bpc, 0, 1, 2});
      } else {
        if (prec == VESNET_FP64 && T > 4) continue;
        if (!sym_fits(P, M, T)) continue;
        const Shape sh{T, 256, 1, 1, 2, 1, 2, T};
        if (forward_bytes(P, M, prec, sh) > ws_bytes) continue;
        cands.push_back({T, 0, 0, 0, 0, 1, 2});
      }
    }
  }
  if (batched && (rc = check_workspace(ws, ws_bytes, vesnet_batched_workspace_bytes(P, M, S, prec)))) return rc;
  if (cands.empty()) return fail(VESNET_ERR_WORKSPACE, "workspace too small for any launch shape");

  if (!batched) {
    if ((rc = vesnet_farfield_prepare(sources, f, w, off, M, P, prec, ws, ws_bytes, stream))) return rc;
  }
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  float best_t = 1e30f;
  vesnet_tile_config best_c = cands[0];
  rc = VESNET_OK;
  for (const auto& c : cands) {
    auto run = [&]() -> int {
      if (batched)
        return vesnet_farfield_stokeslet_batched(targets, sources, f, w, off, M, P, sus_off, S, mu_dev, out, prec, &c,
                                                 ws, ws_bytes, stream);
      return vesnet_farfield_evaluate(targets, off, M, P, mu_host, out, prec, &c, ws, ws_bytes, stream);
    };
    if ((rc = run())) break;  // warm-up
    float tmin = 1e30f;
    for (int r = 0; r < repeats && rc == VESNET_OK; ++r) {
      (void)hipEventRecord(e0, st);
      rc = run();
      (void)hipEventRecord(e1, st);
      if (rc) break;
      e = hipEventSynchronize(e1);
      if (e != hipSuccess) { rc = hip_fail(e, "hipEventSynchronize"); break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      tmin = std::min(tmin, ms);
    }
    if (rc) break;
    if (tmin < best_t) {
      best_t = tmin;
      best_c = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  *best = best_c;
  if (best_ms) *best_ms = best_t;
  return ok();
}

// ============================================================================ no allocation

namespace {

// The scratch memory of vesnet_farfield_stokeslet_noalloc: a device array of this library, one
// copy per GPU (loaded with the library's code object on each device).  Host code never passes
// its name to a kernel: the name is a host-side stand-in, and each device's address comes from
// hipGetSymbolAddress on that device.
static __device__ __align__(256) unsigned char scratch[VESNET_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of the scratch array (looked up once per device).
int scratch_on_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(VESNET_ERR_UNSUPPORTED, "device %d is beyond the %d devices the scratch table holds", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the scratch array");
    if (!p) return fail(VESNET_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return VESNET_OK;
}

}  // namespace

extern "C" int vesnet_farfield_stokeslet_noalloc(const double* targets, const double* sources, const double* f,
                                                 const double* w, const int32_t* off, int32_t M, int32_t P, double mu,
                                                 double* out, int prec, const vesnet_tile_config* cfg, void* stream) {
  int rc = check_forward_args(targets, sources, f, w, off, M, P, out, prec, nullptr, 0, true, true);
  if (rc) return rc;
  if ((rc = check_mu(mu))) return rc;
  if (P == 0) return ok();
  if (!out) return fail(VESNET_ERR_INVALID_ARGUMENT, "out is NULL");
  Shape s;
  if ((rc = resolve_shape(cfg, P, M, prec, &s))) return rc;
  if (s.pair == 2 && targets != sources)
    return fail(VESNET_ERR_INVALID_ARGUMENT, "the symmetric pair form needs targets == sources (one point array)");
  const bool symmetric =
      s.pair == 2 || (s.pair == 0 && targets == sources && has_symmetric(prec) && s.accumulate == 1 && s.symT > 0);
  // the workspace of the chosen form only; the direct form's split partials shrink until it fits
  // unless the caller fixed source_splits
  s.pair = symmetric ? 2 : 1;
  const size_t cap = VESNET_NOALLOC_SCRATCH_BYTES;
  size_t need = forward_bytes(P, M, prec, s);
  if (!(cfg && cfg->source_splits))
    while (need > cap && s.splits > 1) {
      s.splits /= 2;
      need = forward_bytes(P, M, prec, s);
    }
  if (need > cap)
    return fail(VESNET_ERR_WORKSPACE,
                "n_points=%d, n_vesicles=%d need %zu bytes of scratch; the no-allocation entry point has %zu "
                "(use vesnet_farfield_stokeslet with a workspace)",
                P, M, need, cap);
  void* ws = nullptr;
  if ((rc = scratch_on_current_device(&ws))) return rc;
  if ((rc = vesnet_farfield_prepare(sources, f, w, off, M, P, prec, ws, cap, stream))) return rc;
  return evaluate_resolved(targets, M, P, mu, out, prec, s, symmetric, ws, cap, stream);
}
