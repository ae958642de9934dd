/*
 * vesnet.h - far-field Stokeslet single-layer sum on AMD Instinct MI355X (gfx950).
 *
 * The operation (Section 2.2, eq. (single_layer) with the 2D Stokeslet of
 * eq. (Stokeslet); trapezoid rule for far-field targets, Section 2.2.1; the
 * far-field velocity U_far of eq. (membrane_velocity), which is what
 * DirectSingleLayerIntegral returns in Algorithm 4):
 *
 *   out_i = 1/(4 pi mu) * sum_{j : ves(j) != ves(i)} w_j [ -ln|r| f_j + ((r . f_j)/|r|^2) r ],
 *   r = targets_i - sources_j.
 *
 * The Stokeslet is printed in the paper with "+log|r|" and no identity
 * matrix; this library computes -ln|r| I + r r^T/|r|^2, the divergence-free
 * fundamental solution.  w_j is the trapezoid weight |X'(alpha_j)| 2 pi/N of
 * point j (the arclength element ds of eq. (single_layer)).  Each target
 * skips every source of its own vesicle (self-interaction is handled
 * separately in the paper).  The result overwrites out; near-field and
 * background velocities are the caller's to add.
 *
 * Conventions shared by every entry point
 *  - Arrays of 2D vectors are planar structure-of-arrays [2][P] float64:
 *    x components at [0, P), y components at [P, 2P).
 *  - targets and sources share one vesicle partition: int32
 *    vesicle_offsets[M+1] with offsets[0] = 0, offsets[M] = P, non-decreasing;
 *    vesicle v owns points offsets[v] .. offsets[v+1]-1 of both arrays.
 *  - Every pointer argument marked "device" is device memory owned by the
 *    caller; the library never allocates, frees or retains it.  Device
 *    offsets cannot be read by the host without a synchronisation, so the
 *    kernels clamp them into [0, P]: malformed offsets give wrong numbers
 *    but never out-of-bounds accesses.  vesnet_check_offsets validates a
 *    host copy.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are asynchronous and enqueue kernels only; no call synchronises except
 *    vesnet_autotune and vesnet_graph_create_batched.
 *  - Every call returns a vesnet_status.  Argument errors are detected on the
 *    host before anything is enqueued; vesnet_last_error() then describes
 *    the failure (thread-local, valid until the next call on the thread).
 *  - Coincident points of different vesicles make the sum undefined (log of
 *    zero); the output is then unspecified (inf/NaN) and no error is raised.
 *  - Calls on different streams with separate workspaces may run concurrently.
 */
#ifndef VESNET_H
#define VESNET_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define VESNET_API __attribute__((visibility("default")))
#else
#define VESNET_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VESNET_OK = 0,
  VESNET_ERR_INVALID_ARGUMENT = -1, /* bad pointer, size, mu, precision, aliasing, offsets */
  VESNET_ERR_UNSUPPORTED = -2,      /* valid request the library does not implement       */
  VESNET_ERR_WORKSPACE = -3,        /* workspace missing or smaller than required          */
  VESNET_ERR_HIP = -4               /* a HIP runtime call or kernel launch failed          */
} vesnet_status;

typedef enum {
  VESNET_FP64 = 0,              /* every operation in float64                                   */
  VESNET_FP32_COMPENSATED = 1,  /* pairs in float32 on per-vesicle local, rescaled coordinates;
                                   per-source-vesicle partials flushed into float64 together
                                   with the exact float64 log-term correction                     */
  VESNET_FP32_NAIVE = 2         /* everything in float32 on global coordinates (control only)   */
} vesnet_precision;

/* Launch shape of the pair kernels.  A zero field selects the built-in default. */
typedef struct {
  int32_t targets_per_thread; /* 1, 2 or 4 (symmetric form: see pair_form)                    */
  int32_t block_threads;      /* 64, 128 or 256                                               */
  int32_t source_splits;      /* >= 1: source vesicles split into this many chunks, reduced in
                                 a fixed order by a second kernel (bitwise deterministic)      */
  int32_t blocks_per_cu;      /* batched persistent grid: workgroups per compute unit (1..16;
                                 0: 4 for the direct form, as many as fit for the symmetric form) */
  int32_t source_staging;     /* 1: source records read at wave-uniform addresses into SGPRs;
                                 2: records staged through LDS tiles of 1024 and read back with
                                    broadcast LDS loads into VGPRs                               */
  int32_t accumulate;         /* 1: per-pair sums accumulated with VALU FMAs;
                                 2: (compensated forward only) the four accumulations of each pair
                                    issued to the matrix cores as v_mfma_f32_4x4x1f32 products of
                                    per-target values and per-source features (measured slower on
                                    gfx950: each 4x4x1 product takes about five FMA issue slots
                                    and does not overlap the VALU work; kept for comparison)      */
  int32_t pair_form;          /* 0: automatic - vesnet_farfield_stokeslet takes the symmetric form
                                    when targets == sources (the same pointer), the precision is
                                    VESNET_FP32_COMPENSATED or VESNET_FP64, accumulate is 1 and the
                                    problem is large enough (at least four units per compute
                                    unit); every other call takes the direct form;
                                 1: direct form - one gather per target over all source vesicles;
                                 2: symmetric form (compensated and float64) - each unordered pair
                                    of points of different vesicles is evaluated once and serves
                                    both (the Stokeslet is even), halving the logarithms and
                                    reciprocals; the targets must be the points the workspace was
                                    prepared with (vesnet_farfield_stokeslet requires targets ==
                                    sources).  targets_per_thread (compensated 1, 2, 3, 4 or 8,
                                    default 3; float64 1, 2, 3 or 4, default 4; the default drops to 2,
                                    then 1, for problems too small for four units per compute
                                    unit) sets its blocks of 256 T points (one
                                    256-thread workgroup per pair of blocks); block_threads,
                                    source_splits and source_staging are unused.  The automatic
                                    choice always uses the default.  Its partial sums are added as
                                    64-bit fixed-point integers (float64: a high and a low word,
                                    40 bits finer), so the result is bitwise reproducible.         */
} vesnet_tile_config;

/* Library version string and the thread-local description of the last error. */
VESNET_API const char* vesnet_version(void);
VESNET_API const char* vesnet_last_error(void);

/* Host check of a host copy of the partition: offsets[0] = 0, offsets[M] = P,
   non-decreasing, M >= 0 (M = 0 requires P = 0).  Returns VESNET_OK or
   VESNET_ERR_INVALID_ARGUMENT. */
VESNET_API int vesnet_check_offsets(const int32_t* offsets_host, int32_t n_vesicles, int32_t n_points);

/* The launch shape used when cfg is NULL or has zero fields. */
VESNET_API int vesnet_default_tile_config(int32_t n_points, int32_t n_vesicles, int precision, vesnet_tile_config* cfg);

/* ------------------------------------------------------------------ forward */

/* Bytes of device workspace the forward calls need (256-byte aligned base). */
VESNET_API size_t vesnet_farfield_workspace_bytes(int32_t n_points, int32_t n_vesicles, int precision,
                                       const vesnet_tile_config* cfg);

/* Step 1 of the forward: per-vesicle preprocessing into the workspace.
   For each vesicle: reference point c_v (mean of its source points, float64)
   and net weighted force F_v = sum_j w_j f_j (float64); for each source point
   the record the pair kernel streams (local coordinates y_j - c_v and
   w_j f_j in float32 for the compensated form, global float32 for the naive
   form, global float64 for FP64), and the vesicle id of every point.
     sources, force_density : device [2][P] float64
     arc_weights            : device [P] float64
     vesicle_offsets        : device [M+1] int32 */
VESNET_API int vesnet_farfield_prepare(const double* sources, const double* force_density, const double* arc_weights,
                            const int32_t* vesicle_offsets, int32_t n_vesicles, int32_t n_points,
                            int precision, void* workspace, size_t workspace_bytes, void* stream);

/* Step 2 of the forward: the pair sum at every target from a prepared
   workspace (same partition, precision and cfg as used for the workspace size).
     targets : device [2][P] float64, read only
     out     : device [2][P] float64, overwritten; must not overlap any input
     mu      : viscosity, finite and > 0 */
VESNET_API int vesnet_farfield_evaluate(const double* targets, const int32_t* vesicle_offsets, int32_t n_vesicles,
                             int32_t n_points, double mu, double* out, int precision,
                             const vesnet_tile_config* cfg, void* workspace, size_t workspace_bytes,
                             void* stream);

/* prepare + evaluate. */
VESNET_API int vesnet_farfield_stokeslet(const double* targets, const double* sources, const double* force_density,
                              const double* arc_weights, const int32_t* vesicle_offsets, int32_t n_vesicles,
                              int32_t n_points, double mu, double* out, int precision,
                              const vesnet_tile_config* cfg, void* workspace, size_t workspace_bytes,
                              void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc): vesnet_farfield_stokeslet without a workspace argument.  Its workspace is
   a device array inside the library, VESNET_NOALLOC_SCRATCH_BYTES (64 MiB) on each GPU, held from
   the library's load on that GPU until the process ends; the call itself allocates nothing.
   Its address on the current device is looked up on the first call on that device (the stream
   must belong to the current device).
     - Arguments, layouts, launch shapes, forms and results as vesnet_farfield_stokeslet, except
       that when cfg leaves source_splits at 0 the direct form's split count is halved until the
       workspace fits.
     - Sizes whose workspace exceeds the array are refused with VESNET_ERR_WORKSPACE before
       anything is enqueued.  The symmetric form (float32-compensated, targets == sources) needs
       about 54 bytes per point and 96 per vesicle: about 1.1 million points fit.
     - Every call on one GPU uses that GPU's one array: calls that overlap on a GPU (on different
       streams, or from different threads without ordering) race and give wrong results.  Every
       part that must start at zero is cleared by a kernel of the call itself. */
#define VESNET_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
VESNET_API int vesnet_farfield_stokeslet_noalloc(const double* targets, const double* sources,
                                                 const double* force_density, const double* arc_weights,
                                                 const int32_t* vesicle_offsets, int32_t n_vesicles,
                                                 int32_t n_points, double mu, double* out, int precision,
                                                 const vesnet_tile_config* cfg, void* stream);

/* ------------------------------------------------------------------ membrane force */

/* The step before the sum, on the device: the elastic force density of
   eq. (elastic_force), f = -kappa_b X_ssss + (sigma X_s)_s, and the trapezoid
   weights w = |X_alpha| 2 pi / N, with spectral arclength derivatives
   d/ds = (1/|X_alpha|) d/dalpha (Section 2.2.1).  Each vesicle's N points are
   read as the samples alpha_k = 2 pi k / N of a periodic curve; d/dalpha is exact
   on their band-limited interpolant (the even-N Nyquist mode has zero
   derivative).  Computed in float64.
     X              : device [2][P] float64 membrane points
     sigma          : device [P] float64 tension, or NULL for zero tension
     force_density  : device [2][P] float64, overwritten (the sum's force_density)
     arc_weights    : device [P] float64, overwritten (the sum's arc_weights)
   Vesicles of more than 1024 points get NaN outputs; vesicles of fewer than 3
   points have no tangent and give NaN as well. */
VESNET_API int vesnet_elastic_force(const double* X, const double* sigma, double kappa_b,
                                    const int32_t* vesicle_offsets, int32_t n_vesicles, int32_t n_points,
                                    double* force_density, double* arc_weights, void* stream);

/* ------------------------------------------------------------------ near field */

/* The far field as the paper's direct evaluation masks it (Section 4.1) and the
   near-field detection FindNearFieldPoints of Algorithm 4: vesicle v is in the
   near field of target i when the distance from the target to v's points,
   min_j |targets_i - sources_j|, is at most the arclength spacing of v (the
   near-field rule of Section 2.2), taken as h_v = sum_j w_j / N_v.  Near
   vesicles are dropped from out like the own vesicle, and every near pair
   (target index, vesicle index) is stored into near_pairs[2k], near_pairs[2k+1]
   in unspecified order.  *near_count (device int32) is overwritten with the
   number of near pairs found; when it exceeds near_capacity only the first
   near_capacity pairs were stored and the call should be repeated with a larger
   list.  The distance test runs in the precision of the pair loop (float32 on
   the rescaled coordinates for the compensated form), so a pair whose distance
   lies within about 1e-7 relative of h_v may be classified either way.
     near_pairs : device int32 [near_capacity][2] (may be NULL if capacity is 0)
     near_count : device int32 [1]
   Other arguments as vesnet_farfield_stokeslet; targets_per_thread is capped at 2. */
VESNET_API int vesnet_farfield_stokeslet_nearmasked(const double* targets, const double* sources,
                                                    const double* force_density, const double* arc_weights,
                                                    const int32_t* vesicle_offsets, int32_t n_vesicles,
                                                    int32_t n_points, double mu, double* out, int32_t* near_pairs,
                                                    int32_t near_capacity, int32_t* near_count, int precision,
                                                    const vesnet_tile_config* cfg, void* workspace,
                                                    size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ near-field interpolation */

/* CreateNearLayers of Algorithm 4 (Section 3.3): around each vesicle, five layers of target
   points, its N_v membrane points moved along the outward unit normal by d_l = (l - 2) h_v / 2,
   l = 0..4 (that is -h, -h/2, 0, h/2, h), with h_v = sum_j w_j / N_v the mean arclength spacing.
   The tangent is X_alpha / |X_alpha| with the spectral derivative of vesnet_elastic_force; the
   outward side follows from the sign of the enclosed signed area, so the points may run either
   way round.  Computed in float64.
     X          : device [2][P] float64 membrane points
     arc_weights: device [P] float64 w
     layers     : device [2][5P] float64, overwritten; node a = l N_v + k of vesicle v is stored
                  at index 5 offsets[v] + a (x row, then y row at offset 5P)
   Vesicles of more than 1024 or fewer than 3 points get NaN layers. */
VESNET_API int vesnet_near_layers(const double* X, const double* arc_weights, const int32_t* vesicle_offsets,
                                  int32_t n_vesicles, int32_t n_points, double* layers, void* stream);

/* Workspace of vesnet_rbf_fit: one slot of packed 32 x 32 float64 tiles per concurrently
   factored vesicle (one wavefront each; at most 2048 slots, and at most 1 GiB recommended).
   max_points bounds N_v (1 .. 200); returns 0 when max_points or n_vesicles is out of range.  A
   smaller workspace of at least one slot also works, with fewer vesicles factored at once. */
VESNET_API size_t vesnet_rbf_workspace_bytes(int32_t max_points, int32_t n_vesicles);

/* Gaussian radial basis interpolation of the layer velocities (Section 3.3): for each vesicle
   the coefficients c of  s(x) = sum_a exp(-|x - x_a|^2 / (width h_v)^2) c_a  that reproduce the
   velocities at its 5 N_v layer nodes, from K c = u with the symmetric positive definite Gaussian
   matrix K, by Cholesky factorisation K = L L^T in float64 (the paper's batched Cholesky).  K is
   ill-conditioned for wide Gaussians (condition about 2e8 at width 1 and N_v = 32): the values
   of s are accurate to about that condition number times the float64 epsilon, the individual
   coefficients may be much less so.  A vesicle whose K is not numerically positive definite, or
   with N_v above max_points, gets NaN coefficients.
     layers, layer_velocity : device [2][5P] float64 in the layout of vesnet_near_layers
     width                  : Gaussian width in units of h_v (> 0; the paper gives no value)
     coeffs                 : device [2][5P] float64, overwritten
     workspace              : device, at least one slot (see vesnet_rbf_workspace_bytes) */
VESNET_API int vesnet_rbf_fit(const double* layers, const double* layer_velocity, const double* arc_weights,
                              const int32_t* vesicle_offsets, int32_t n_vesicles, int32_t n_points, int32_t max_points,
                              double width, double* coeffs, void* workspace, size_t workspace_bytes, void* stream);

/* interpolateInNearField of Algorithm 4: for each near pair k < min(*near_count, near_capacity),
   (i, v) = (near_pairs[2k], near_pairs[2k+1]) as vesnet_farfield_stokeslet_nearmasked writes
   them, adds vesicle v's interpolant at targets[:, i] into out[:, i].  Pairs whose indices fall
   outside the problem are skipped.  The additions are atomic: a target near several vesicles
   receives their contributions in an unspecified order (last-bit differences between runs).
     targets : device [2][n_targets] float64
     out     : device [2][n_targets] float64, accumulated into (u_far + u_near of Algorithm 4)
   Other arguments as vesnet_rbf_fit. */
VESNET_API int vesnet_rbf_eval_near(const double* layers, const double* coeffs, const double* arc_weights,
                                    const int32_t* vesicle_offsets, int32_t n_vesicles, int32_t n_points, double width,
                                    const double* targets, int32_t n_targets, const int32_t* near_pairs,
                                    const int32_t* near_count, int32_t near_capacity, double* out, void* stream);

/* ------------------------------------------------------------------ treecode far field */

/* A fast, approximate evaluation of the far-field sum for targets = sources = points (the paper
   evaluates the sum directly and leaves fast summation, e.g. the fast multipole method, out of
   scope: Section 4.1).  A uniform quadtree of the given depth covers the bounding square of the
   points; sources in boxes of a target's interaction lists (levels 2..depth) act through power-
   moment expansions truncated after the given order, sources in the 3 x 3 leaves around the
   target's leaf act directly, and the target's own vesicle is excluded (exactly, also where the
   expansions included it).  Cost O(P log P); everything in float64.
   Accuracy: for a box of radius rho seen from distance R, the dropped terms are below
   sum_box |w f| x^(order+1) (1/((order+1)(1-x)) + (1+x)/(2(1-x))) / (4 pi mu), x = rho/R <= 0.55;
   this bound is the contract.  Measured on the 2000 x 128 suspension at depth 6 (2,000 seeded
   targets against the exact sum): 8.7e-9 relative to max|u| at order 20, 3.2e-12 at order 30,
   1.3e-14 at order 40; order 45 reaches rounding.
   Results are deterministic unless a leaf holds more than 2048 points (then its summation order
   follows an atomic scatter).
     points, force_density : device [2][P] float64; arc_weights device [P] float64
     order                 : 1 .. 48;  depth: 0 .. 10 (vesnet_treecode_default_depth: leaves of
                             at most about 64 points)
     out                   : device [2][P] float64, overwritten with u_far
     workspace             : device, vesnet_treecode_workspace_bytes(P, depth, order) bytes */
VESNET_API int32_t vesnet_treecode_default_depth(int32_t n_points);
VESNET_API size_t vesnet_treecode_workspace_bytes(int32_t n_points, int32_t depth, int32_t order);
VESNET_API int vesnet_farfield_treecode(const double* points, const double* force_density, const double* arc_weights,
                                        const int32_t* vesicle_offsets, int32_t n_vesicles, int32_t n_points,
                                        double mu, int32_t order, int32_t depth, double* out, void* workspace,
                                        size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ fast multipole far field */

/* The fast multipole method the paper names as the route to O(M) cost and leaves out of scope
   (Section 4.1), on the treecode's tree, interaction lists, direct part and own-vesicle exclusion:
   instead of evaluating every far box's truncated multipole series at every target, each box's
   series is converted once into a Taylor polynomial of the same order about the centre of every
   box whose interaction list holds it, the polynomials are re-centred down the tree, and each target
   evaluates only its leaf's polynomial.  The far work becomes O(boxes x order^2) instead of
   O(points x boxes per list x order).  Accuracy: the treecode's bound plus the Taylor truncation of
   each translated series (the contract); measured at the same order 2 to 4 times the treecode's
   error (2000 x 128, depth 6: 2.0e-8 at order 20, 1.1e-11 at order 30, 1.2e-14 at order 40 relative
   to max|u|); everything in float64.
   Deterministic under the same condition as the treecode.
     arguments, layouts, ownership and errors as vesnet_farfield_treecode;
     workspace : device, vesnet_fmm_workspace_bytes(P, depth, order) bytes (the treecode's plus
                 3 (order+1) complex numbers per box and a binomial table) */
/* Default depth of the fast multipole method: leaves of at most about 64 points up to order 32 and 128
   above, where the M2L work (order^2 per pair of boxes) outweighs the direct part (measured best on the
   2000 x 128 and 8000 x 64 suspensions at orders 30 and 40). */
VESNET_API int32_t vesnet_fmm_default_depth(int32_t n_points, int32_t order);
VESNET_API size_t vesnet_fmm_workspace_bytes(int32_t n_points, int32_t depth, int32_t order);
VESNET_API int vesnet_farfield_fmm(const double* points, const double* force_density, const double* arc_weights,
                                   const int32_t* vesicle_offsets, int32_t n_vesicles, int32_t n_points, double mu,
                                   int32_t order, int32_t depth, double* out, void* workspace, size_t workspace_bytes,
                                   void* stream);

/* The fast multipole far field with the near-field masking of Algorithm 4: as
   vesnet_farfield_stokeslet_nearmasked, vesicle v (not the target's own) is near target i when
   min_j |x_i - x_j| <= h_v = sum_j w_j / N_v, decided here in float64 on squared distances.  Every
   near pair (i, v) is stored into near_pairs[2k], near_pairs[2k+1] in unspecified order, and v's
   exact direct sum at x_i is subtracted from the fast multipole result, so that out is the masked
   far field with the fast multipole method's truncation error.  The result does not depend on the
   order of the list.
   Near vesicles are found in the 3 x 3 leaves around the target's leaf, which holds every point
   within h_v while h_v <= side / 2^depth (side: the larger extent of the points).
   *near_count (device int32) receives:
     >= 0: the number of near pairs; when it exceeds near_capacity, only the first near_capacity
           were stored, but out is masked completely;
     -1:   a target had more than 16 near vesicles (out is not masked completely);
     -2:   some h_v exceeds the leaf width (use a smaller depth; out is not masked completely).
     near_pairs : device int32 [near_capacity][2] (may be NULL if capacity is 0)
     workspace  : device, vesnet_fmm_nearmasked_workspace_bytes(P, M, depth, order) bytes
   Other arguments as vesnet_farfield_fmm. */
VESNET_API size_t vesnet_fmm_nearmasked_workspace_bytes(int32_t n_points, int32_t n_vesicles, int32_t depth,
                                                        int32_t order);
VESNET_API int vesnet_farfield_fmm_nearmasked(const double* points, const double* force_density,
                                              const double* arc_weights, const int32_t* vesicle_offsets,
                                              int32_t n_vesicles, int32_t n_points, double mu, int32_t order,
                                              int32_t depth, double* out, int32_t* near_pairs, int32_t near_capacity,
                                              int32_t* near_count, void* workspace, size_t workspace_bytes,
                                              void* stream);

/* ------------------------------------------------------------------ batched */

/* S independent suspensions concatenated point-wise and vesicle-wise.
   Suspension s owns vesicles suspension_offsets[s] .. suspension_offsets[s+1]-1
   (device int32 [S+1], suspension_offsets[0] = 0, [S] = V) and has viscosity
   mu[s] (device float64 [S], each > 0).  No interaction crosses suspensions.
   Each suspension's result is the single call's (vesnet_farfield_stokeslet) on
   its own points; the call needs no host-side copy of the tables (they are
   read on the device, so the call can be captured once and replayed).
   Two forms, chosen as in the single call (cfg->pair_form):
   * symmetric (VESNET_FP32_COMPENSATED, targets == sources, pair_form 0 or 2):
     the single call's symmetric form for every suspension in one persistent
     launch.  A plan kernel cuts each suspension into blocks of 256 T points
     (T = targets_per_thread: 1, 2, 3 or 4 when pair_form is 2, else the single
     call's default for the total point count) that never reach into another
     suspension; the unordered pairs of a suspension's blocks are its units,
     numbered suspension by suspension and split into eight contiguous queues,
     one per XCD, drained through counters in the workspace by
     blocks_per_cu workgroups per compute unit (0: as many as fit).  Every
     suspension's output equals that of a single symmetric call with the same
     T bit for bit (the fixed-point sums do not depend on the order).
   * direct (every other call, or pair_form 1): work items (suspension, block
     of targets) ordered largest suspension first on the device and handed
     out through a counter in the workspace.
   Errors: VESNET_ERR_UNSUPPORTED when the symmetric form's units could exceed
   one launch (about 2^31; use pair_form 1), else as the single call. */
VESNET_API size_t vesnet_batched_workspace_bytes(int32_t n_points, int32_t n_vesicles, int32_t n_suspensions, int precision);

VESNET_API int vesnet_farfield_stokeslet_batched(const double* targets, const double* sources, const double* force_density,
                                      const double* arc_weights, const int32_t* vesicle_offsets,
                                      int32_t n_vesicles, int32_t n_points, const int32_t* suspension_offsets,
                                      int32_t n_suspensions, const double* mu, double* out, int precision,
                                      const vesnet_tile_config* cfg, void* workspace, size_t workspace_bytes,
                                      void* stream);

/* The same batched call captured once into a HIP graph (the capture runs on
   a private stream and synchronises it); replay with vesnet_graph_launch.
   All pointers are baked into the graph and must stay valid until destroy. */
typedef struct vesnet_graph vesnet_graph;
VESNET_API int vesnet_graph_create_batched(const double* targets, const double* sources, const double* force_density,
                                const double* arc_weights, const int32_t* vesicle_offsets, int32_t n_vesicles,
                                int32_t n_points, const int32_t* suspension_offsets, int32_t n_suspensions,
                                const double* mu, double* out, int precision, const vesnet_tile_config* cfg,
                                void* workspace, size_t workspace_bytes, vesnet_graph** graph);
VESNET_API int vesnet_graph_launch(vesnet_graph* graph, void* stream);
VESNET_API int vesnet_graph_destroy(vesnet_graph* graph);

/* ------------------------------------------------------------------ adjoint */

/* Reverse mode of the forward sum (the paper has none; derived from it).
   With c = 1/(4 pi mu), F_j = w_j f_j, g_i = grad_out_i = dL/dout_i and
   phi(r; g, F) = g^T G(r) F:
     grad_targets_i = sum_j grad_r phi(r_ij; g_i, F_j)
     grad_sources_j = - sum_i grad_r phi(r_ij; g_i, F_j)
     grad_force_j   = w_j v_j,  grad_weights_j = f_j . v_j,  v_j = sum_i G(r_ij) g_i
   (sums over pairs in different vesicles).  When targets and sources are the
   same array, dL/dX = grad_targets + grad_sources.
     grad_out                     : device [2][P] float64
     grad_targets, grad_sources,
     grad_force                   : device [2][P] float64 or NULL (skipped)
     grad_weights                 : device [P] float64 or NULL
   Outputs are overwritten and must not overlap inputs or each other.
   precision: VESNET_FP64 or VESNET_FP32_COMPENSATED. */
VESNET_API size_t vesnet_backward_workspace_bytes(int32_t n_points, int32_t n_vesicles, int precision);

VESNET_API int vesnet_farfield_stokeslet_backward(const double* targets, const double* sources, const double* force_density,
                                       const double* arc_weights, const int32_t* vesicle_offsets,
                                       int32_t n_vesicles, int32_t n_points, double mu, const double* grad_out,
                                       double* grad_targets, double* grad_sources, double* grad_force,
                                       double* grad_weights, int precision, void* workspace,
                                       size_t workspace_bytes, void* stream);

/* The same adjoint for one point array that serves as targets and sources
   (u_i = sum_{j not in ves(i)} G(X_i - X_j) F_j), with the positions
   differentiated in both roles:
     grad_points_k = sum_{m not in ves(k)} [ grad_r phi(X_k - X_m; g_k, F_m)
                                            + grad_r phi(X_k - X_m; F_k, g_m) ]
   and grad_force, grad_weights as above.  Both terms of one pair (k, m) share
   r, |r|^2, its reciprocal and logarithm, and grad_r phi is odd in r, so each
   unordered pair of points in different vesicles is evaluated once (the
   symmetric forms of the forward: VESNET_FP32_COMPENSATED on rescaled local
   coordinates, VESNET_FP64 on global coordinates), with float64 atomic sums:
   the last bits may differ from call to call.  (Should the units of the
   symmetric form not fit one launch, about 33 million points, the two gathers
   of vesnet_farfield_stokeslet_backward run and their position gradients are
   added.)
     points                       : device [2][P] float64
     grad_out                     : device [2][P] float64
     grad_points, grad_force      : device [2][P] float64 or NULL (skipped)
     grad_weights                 : device [P] float64 or NULL
     workspace                    : device, vesnet_backward_points_workspace_bytes(P, M, precision)
   Outputs are overwritten and must not overlap inputs or each other; errors as
   for vesnet_farfield_stokeslet_backward. */
VESNET_API size_t vesnet_backward_points_workspace_bytes(int32_t n_points, int32_t n_vesicles, int precision);

VESNET_API int vesnet_farfield_stokeslet_backward_points(const double* points, const double* force_density,
                                              const double* arc_weights, const int32_t* vesicle_offsets,
                                              int32_t n_vesicles, int32_t n_points, double mu,
                                              const double* grad_out, double* grad_points, double* grad_force,
                                              double* grad_weights, int precision, void* workspace,
                                              size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------ tuning */

/* Times every supported launch shape on the given (prepared inside) problem
   with HIP events and returns the fastest in *best and its time in *best_ms.
   batched != 0 tunes the batched call (then suspension_offsets, n_suspensions
   and mu_device are used; otherwise mu_host).  The candidates are the direct
   form's shapes (pair_form 1 where the symmetric form could also run) and, for
   one compensated point array, the symmetric form at 1, 2, 4 (and, single
   call, 8) targets per thread (batched: with 0, 2, 4 or 8 workgroups per
   compute unit).  Host-synchronous; the workspace must hold the largest shape
   tried (shapes that do not fit are skipped). */
VESNET_API int vesnet_autotune(const double* targets, const double* sources, const double* force_density,
                    const double* arc_weights, const int32_t* vesicle_offsets, int32_t n_vesicles,
                    int32_t n_points, int batched, const int32_t* suspension_offsets, int32_t n_suspensions,
                    const double* mu_device, double mu_host, double* out, int precision, int repeats,
                    void* workspace, size_t workspace_bytes, void* stream, vesnet_tile_config* best,
                    float* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* VESNET_H */
