/*
 * vegasp.h -- C ABI of the MI355X (gfx950) vegas+ library.
 *
 * The library runs the per-iteration hot path of vegas+ (G. P. Lepage,
 * "Adaptive Multidimensional Integration: VEGAS Enhanced", arXiv:2009.05112)
 * on one GPU: stratified sampling with a counter-based Philox stream, the
 * vegas map with its Jacobian, integrand evaluation, per-hypercube sums,
 * per-increment training data, reallocation of samples across hypercubes and
 * refinement of the map.  Every step runs in the library's own HIP kernels.
 *
 * Conventions
 *  - Every function returns a vp_status and never throws or exits.  On error
 *    vp_last_error() returns a description (thread-local, valid until the next
 *    call on the same thread).
 *  - Pointers documented as "host" point to host memory owned by the caller;
 *    the library copies what it needs before returning.  The library owns all
 *    device memory it allocates; results are copied into caller buffers.
 *  - Handles are not thread-safe, except the vp_server_* calls documented so.
 *  - Work is enqueued on the context's HIP stream; calls documented as
 *    "synchronising" wait for that stream.
 */
#ifndef VEGASP_H
#define VEGASP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VP_OK = 0,
    VP_ERR_INVALID_ARG = 1, /* an argument violates the documented contract        */
    VP_ERR_OOM = 2,         /* device or host allocation failed / over budget       */
    VP_ERR_DEVICE = 3,      /* a HIP runtime call failed                            */
    VP_ERR_NUMERIC = 4,     /* non-finite integrand values were produced            */
    VP_ERR_NOT_READY = 5,   /* a served request has not finished                    */
    VP_ERR_CANCELLED = 6,   /* a served request was cancelled                       */
    VP_ERR_STATE = 7,       /* the call does not fit the object's current state     */
    VP_ERR_INVARIANT = 8    /* a device-side check found a broken invariant         */
} vp_status;

/* Static description of a status; the caller does not free it. */
const char* vp_status_string(vp_status s);
/* Detail of the last failing call on this thread (never NULL). */
const char* vp_last_error(void);

typedef struct vp_ctx vp_ctx;
typedef struct vp_problem vp_problem;
typedef struct vp_server vp_server;

/* A context binds one GPU and one HIP stream.  device: HIP ordinal.
 * hip_stream: a hipStream_t to enqueue on, or NULL for a stream the context
 * creates (default priority) and destroys. */
vp_status vp_ctx_create(int device, void* hip_stream, vp_ctx** out);
vp_status vp_ctx_destroy(vp_ctx* ctx);
/* Number of compute units of the context's device. */
vp_status vp_ctx_info(vp_ctx* ctx, int32_t* n_cu, int64_t* lds_bytes_per_block);

/* Integrands (f(x) as the user defines it; the sampler multiplies by J).
 *  VP_F_GAUSS_MIX:  scale * sum_k amps[k] exp(-coefs[k] |x - c_k|^2),
 *                   c_k = centers[k*dim .. k*dim+dim-1], 1 <= n_terms <= 4
 *  VP_F_CORR_GAUSS: scale * exp(-1/2 |U (x - m)|^2), m = centers[0..dim-1],
 *                   U = chol, dim x dim row-major upper-triangular
 *                   (U^T U is the inverse covariance)
 *  VP_F_EXP_ABS:    scale * sum_k amps[k] exp(-coefs[k] |x - c_k|), n_terms <= 4
 *  VP_F_CONST:      scale
 *  VP_F_AFFINE:     scale * (a_0 + sum_d a_{d+1} x_d), a = centers[0..dim]
 *  VP_F_BALLS:      scale * sum_k amps[k] [ |x - c_k| < coefs[k] ], n_terms <= 4
 *  VP_F_BATCH:      scale * (the user's function): a batched ("vectorised")
 *                   integrand evaluated by `fn` on a whole iteration's
 *                   samples at once (Sec. 1: vegas evaluates the integrand
 *                   in batches).  Double precision only; not servable.
 * The host arrays are copied at create time. */
enum {
    VP_F_GAUSS_MIX = 1,
    VP_F_CORR_GAUSS = 2,
    VP_F_EXP_ABS = 3,
    VP_F_CONST = 4,
    VP_F_AFFINE = 5,
    VP_F_BALLS = 6,
    VP_F_BATCH = 100
};

/* A batched integrand.  Called from vp_iterate once per iteration, on the
 * host thread that called it, after the library has written the iteration's
 * n sample points to x_soa in device memory: x_soa[d * n + s] is coordinate d
 * of sample s (structure of arrays; the order of the samples is the
 * library's, chosen so that its kernels read and write them coalesced).
 * It must enqueue on hip_stream (a hipStream_t) work that writes f(x_s) to
 * f_out[s], s < n (device memory), and may return before that work is done;
 * a vector-valued integrand (n_out > 1 components) writes component a of
 * sample s to f_out[a * n + s];
 * the library's next kernels on the stream read f_out.  Both buffers belong
 * to the library and are valid only during the call.  A non-zero return
 * fails the iteration with VP_ERR_DEVICE. */
typedef int (*vp_batch_fn)(void* user, void* hip_stream, int64_t n, int32_t dim, const double* x_soa,
                           double* f_out);

typedef struct {
    int32_t kind;
    int32_t dim;
    int32_t n_terms;
    const double* centers; /* host */
    const double* coefs;   /* host, n_terms */
    const double* amps;    /* host, n_terms */
    const double* chol;    /* host, dim*dim (VP_F_CORR_GAUSS only, else NULL) */
    double scale;
    vp_batch_fn fn;        /* VP_F_BATCH only, else NULL */
    void* user;            /* passed to fn unchanged */
    int32_t n_out;         /* components: 0 or 1 scalar; 2..16 VP_F_BATCH only */
} vp_integrand;

/* Vector-valued integrands (Sec. 6: several integrals of one density, such
 * as its normalisation, means and covariances, estimated from the same
 * samples).  Component 0 drives the adaptation (sigma_h of the allocation,
 * the map's training data) and is the scalar result of vp_result_get.  Every
 * component a gets per hypercube the sums S1_a = sum J f_a and, for every
 * pair, S2_ab = sum (J f_a)(J f_b); the iteration's estimates and their
 * covariance are
 *   I_a = sum_h Omega S1_a / n_h,
 *   C_ab = sum_h (Omega^2 S2_ab / n_h - (Omega S1_a / n_h)(Omega S1_b / n_h)) / (n_h - 1)
 * (diagonal terms at least 0), the multivariable form of Eq. sigest. */

/* Arithmetic of the sampling path (the split is not in the paper):
 *  VP_FP64:          everything in double precision;
 *  VP_FP32_ACC64:    uniforms, map, x, J and f in single precision, all sums
 *                    (per hypercube and per increment) in double precision;
 *  VP_FP32_NEUMAIER: as VP_FP32_ACC64, with the sums kept as Neumaier-
 *                    compensated single-precision pairs, merged in double.
 * Estimates, reallocation and refinement are always double precision. */
enum { VP_FP64 = 0, VP_FP32_ACC64 = 1, VP_FP32_NEUMAIER = 2 };

/* Training data for the map (Sec. 2.3, 2.4):
 *  VP_HIST_WEIGHTED: d_i = sum(v^2 / n_h) / sum(1 / n_h) over the samples in
 *                    increment i (each sample weighted by its hypercube's
 *                    share of y-space; equals the printed average when all
 *                    n_h are equal);
 *  VP_HIST_LITERAL:  d_i = (1 / n_i) sum v^2, as printed. */
enum { VP_HIST_WEIGHTED = 0, VP_HIST_LITERAL = 1 };

/* The problem statement (Sec. 2 and 3): dimension, samples per iteration
 * N_ev, map increments N_g per axis, damping alpha (map, Sec. 2.3) and beta
 * (allocation, Sec. 3 Eq. dh), iteration count, integration box.
 *  dim 1..24 (split precisions: 1..16); n_ev 4 .. 2^31-1; n_g 1 .. 4096;
 *  alpha >= 0; beta >= 0; lower/upper: host arrays of dim or NULL for [0,1].
 *  n_st: stratifications per axis, 0 for the rule of Sec. 3 Eq. Nst_vegasp
 *        (largest n with 4 n^dim <= n_ev); a user value must keep
 *        2 n_st^dim <= n_ev.
 *  n_discard: iterations left out of the combined estimate (Sec. 2.5).
 *  realloc_plus2: use n_h = floor(q) + 2 instead of max(2, floor(q)).
 *  n_adapt: 0, or the number of adapting iterations: an iteration whose
 *        index (the one its Philox counters carry) is n_adapt or more
 *        neither reallocates nor refines, so the map and the allocation stay
 *        as the last adapting iteration left them (the frozen phase of
 *        Sec. 2.5, alpha = 0; with n_discard = n_adapt the combined estimate
 *        uses frozen iterations only).  >= 0.
 *  average: VP_AVG_WEIGHTED or VP_AVG_UNWEIGHTED (vp_result).
 *  strat: stratifications per axis N_st^mu (Sec. 4, mixed stratification):
 *        VP_STRAT_UNIFORM: n_st (or its rule) on every axis;
 *        VP_STRAT_MIXED:   N_st + 1 on the first d axes and N_st on the
 *                          others, N_st from the rule above and d the
 *                          largest with 4 (N_st + 1)^d N_st^(dim - d) <= n_ev
 *                          (n_st must be 0).
 *  n_st_axes: NULL, or a host array of dim counts >= 1 that overrides both
 *        (e.g. 46, 46, 1, ..., 1); their product must keep 2 samples per
 *        hypercube and stay below 2^31.
 * Hypercube h has digits k_mu in the mixed radix of the counts, axis 0 most
 * significant; y^mu = (k_mu + u) / N_st^mu.
 *  flags: 0 or an OR of
 *    VP_FLAG_CHECKS: at the start of every iteration a device kernel checks
 *        the state the iteration consumes (see vp_check_get); a violation
 *        makes vp_result_get (and a served request) report VP_ERR_INVARIANT;
 *    VP_FLAG_DETERMINISTIC: bitwise reproducible iterations (the same inputs
 *        on the same device give the same bits; a served request and a
 *        plain problem split the work differently and agree to rounding
 *        only).  The training
 *        data of every axis go through per-sample records that one wave per
 *        workgroup bins in sample order, and the per-chunk partials are added
 *        in a fixed order, so no sum depends on the timing of atomics (the
 *        other sums already are fixed-order).  Costs the records' memory
 *        (8 + 4 + 2 dim bytes per sample) and a binning pass; not available
 *        with VP_FP32_NEUMAIER. */
typedef struct {
    int32_t dim;
    int64_t n_ev;
    int32_t n_g;
    int32_t n_iter;
    double alpha;
    double beta;
    const double* lower;
    const double* upper;
    uint64_t seed;
    int32_t precision;
    int32_t hist_mode;
    int32_t realloc_plus2;
    int32_t n_discard;
    int32_t n_st;
    int32_t n_adapt;
    int32_t average;
    int32_t strat;
    const int32_t* n_st_axes;
    int32_t flags;
} vp_params;

enum { VP_FLAG_CHECKS = 1, VP_FLAG_DETERMINISTIC = 2 };

enum { VP_AVG_WEIGHTED = 0, VP_AVG_UNWEIGHTED = 1 };
enum { VP_STRAT_UNIFORM = 0, VP_STRAT_MIXED = 1 };

/* Combined estimate over iterations n_discard .. n_iter_done - 1 (Sec. 2.5):
 *  VP_AVG_WEIGHTED:   inverse-variance weighted mean I, error
 *                     (sum 1/sigma_j^2)^(-1/2); when some sigma_j is zero,
 *                     the plain mean with error 0;
 *  VP_AVG_UNWEIGHTED: the plain mean of the I_j, error (mean of the
 *                     sigma_j) / sqrt(count) (unbiased once the map and
 *                     allocation no longer adapt: see n_adapt);
 * chi^2 = sum (I_j - I)^2 / sigma_j^2 (NaN when some sigma_j is zero) with
 * dof = count - 1.
 * n_evals counts actual integrand evaluations (sum of n_h over iterations).
 * n_near_ties counts allocations where N_ev d_h / sum d lay within 1e-9
 * (relative) of an integer that decides n_h. */
typedef struct {
    double mean;
    double sdev;
    double chi2;
    int32_t dof;
    int32_t n_iter_done;
    int64_t n_evals;
    int64_t n_near_ties;
    int64_t n_nonfinite;
} vp_result;

/* Creates the device state of one integration: uniform map, uniform
 * allocation max(2, floor(N_ev / N_st^D)), iteration counter 0.
 * Fails with VP_ERR_INVALID_ARG on parameters outside the ranges above and
 * with VP_ERR_OOM when the device state does not fit. */
vp_status vp_problem_create(vp_ctx* ctx, const vp_params* params, const vp_integrand* f,
                            vp_problem** out);
vp_status vp_problem_destroy(vp_problem* p);
/* Derived sizes: stratifications of axis 0 and number of hypercubes. */
vp_status vp_problem_info(vp_problem* p, int32_t* n_st, int64_t* n_hc);
/* Stratifications of every axis: n_st_axes host array of dim entries. */
vp_status vp_problem_strat(vp_problem* p, int32_t* n_st_axes);
/* Where the sampling kernel keeps its per-workgroup data (diagnostics; either
 * pointer may be NULL).  map_place: VP_MAP_GLOBAL, the map read from device
 * memory; VP_MAP_LDS, all of it staged in LDS; VP_MAP_INNER, its two innermost
 * axes staged in LDS and the others read from device memory.  hist_axes: the
 * number of leading axes whose increment training data are accumulated in
 * LDS (the others are written out as per-sample records and binned by a
 * second pass). */
enum { VP_MAP_GLOBAL = 0, VP_MAP_LDS = 1, VP_MAP_INNER = 2 };
vp_status vp_problem_layout(vp_problem* p, int32_t* map_place, int32_t* hist_axes);

/* Enqueues n_iter iterations (asynchronous).  Each iteration (Sec. 2.3 and 3):
 * scan of n_h into sample offsets; sampling, map, integrand, per-hypercube
 * sums and increment training data; the iteration estimate I_j, sigma_j^2;
 * reallocation n_h' = max(2, floor(N_ev sigma_h^beta / sum)); refinement of
 * every axis of the map.  Both adaptations use this iteration's samples and
 * apply to the next. */
vp_status vp_iterate(vp_problem* p, int32_t n_iter);
/* Waits for the problem's enqueued work (synchronising). */
vp_status vp_sync(vp_problem* p);

/* Synchronising.  Combined estimate; optionally the per-iteration estimates
 * I_j (Eq. Iest), their standard deviations sigma_j and variances
 * V_j = sigma_j^2 (Eq. sigest): host arrays of at least cap entries, any of
 * them NULL; the first min(cap, n_iter_done) entries are written. */
vp_status vp_result_get(vp_problem* p, vp_result* out, double* I_j, double* sig_j, double* V_j, int32_t cap);

/* Device-side invariant checks (VP_FLAG_CHECKS), run on the state each
 * iteration starts from:
 *  VP_CHECK_MAP_ORDER  a map point is not finite, or an axis's points are not
 *                      strictly increasing (every increment of the map of
 *                      Sec. 2.2 has positive width);
 *  VP_CHECK_MAP_ENDS   an axis's end points differ from the integration box;
 *  VP_CHECK_NH_MIN     some n_h < 2 (the allocation rules of Sec. 3 keep two
 *                      samples per hypercube, which Eq. sigest needs);
 *  VP_CHECK_NH_SUM     the scanned sample total differs from sum n_h, or
 *                      exceeds n_ev + 2 N_hc.
 * Synchronising.  flags: OR of the bits seen so far (0: none); first_it: the
 * iteration index at which the first violation was seen, -1 if none.  Either
 * pointer may be NULL.  VP_ERR_STATE if the problem was created without
 * VP_FLAG_CHECKS. */
enum { VP_CHECK_MAP_ORDER = 1, VP_CHECK_MAP_ENDS = 2, VP_CHECK_NH_MIN = 4, VP_CHECK_NH_SUM = 8 };
vp_status vp_check_get(vp_problem* p, uint32_t* flags, int32_t* first_it);

/* Synchronising.  Vector results (n_out components, 1 for a scalar problem)
 * over iterations n_discard .. n_iter_done - 1:
 *  VP_AVG_WEIGHTED:   mean = (sum_j C_j^-1)^-1 sum_j C_j^-1 I_j with
 *                     covariance (sum_j C_j^-1)^-1; when some C_j is not
 *                     positive definite, the unweighted result and chi^2 NaN;
 *  VP_AVG_UNWEIGHTED: mean of the I_j, covariance (sum_j C_j) / count^2;
 * chi^2 = sum_j (I_j - mean)^T C_j^-1 (I_j - mean), dof = (count - 1) n_out.
 * mean: host [n_out]; cov: host [n_out][n_out]; I_j: host [cap][n_out] and
 * C_j: host [cap][n_out][n_out], the first min(cap, n_iter_done) iterations.
 * Any pointer may be NULL.  Vector histories hold 4096 iterations. */
vp_status vp_result_vec_get(vp_problem* p, double* mean, double* cov, double* chi2, int32_t* dof, double* I_j,
                            double* C_j, int32_t cap);

/* Synchronising state access for inspection, checkpoints and parity tests.
 * map: host [dim][n_g + 1]; n_h: host [n_hc]. */
vp_status vp_map_get(vp_problem* p, double* map);
vp_status vp_map_set(vp_problem* p, const double* map);       /* must be non-decreasing */
vp_status vp_alloc_get(vp_problem* p, int32_t* n_h);
vp_status vp_alloc_set(vp_problem* p, const int32_t* n_h);    /* every n_h >= 2, sum <= n_ev + 2 n_hc */
/* Iteration index used by the next iteration's Philox counters. */
vp_status vp_iteration_get(vp_problem* p, int32_t* it);
vp_status vp_iteration_set(vp_problem* p, int32_t it);
/* Sums of the last iteration: S1, S2 host [n_hc] (sum of J f and (J f)^2 per
 * hypercube), H, W host [dim][n_g] (training-data numerator and weight per
 * increment).  Any pointer may be NULL. */
vp_status vp_accum_get(vp_problem* p, double* S1, double* S2, double* H, double* W);

/* Per-sample dump, for inspection and parity tests (the uniform y of Sec. 3
 * in each hypercube; the map of Sec. 2.2, Eqs. y and jac).  vp_debug_dump
 * arms it for the next iteration: its sampling kernel records samples
 * [first, first + count) of that iteration, numbered in hypercube order
 * (sample s = offset(h) + j, offset the exclusive sum of n_h), with their
 * hypercube h, index j within it, increment index i^mu and point x^mu on
 * every axis, Jacobian J and f(x) (v = J f is the value summed).  Split
 * precisions report their single-precision values widened to double.
 * count 0 disarms; count <= 2^24.  Not available for VP_F_BATCH
 * (VP_ERR_STATE).  The device buffer is the library's, kept until the next
 * call or the problem's destruction.  Synchronising.
 * vp_debug_dump_get: synchronising; *n_out receives the number of samples
 * recorded (fewer than count when the iteration had fewer samples after
 * `first`); h, j, jac, fx: host [n_out]; idx, x: host [dim][n_out]; any
 * array may be NULL.  VP_ERR_STATE when no dump is armed or its iteration
 * has not run yet. */
vp_status vp_debug_dump(vp_problem* p, int64_t first, int64_t count);
vp_status vp_debug_dump_get(vp_problem* p, int64_t* n_out, int64_t* h, int32_t* j, int32_t* idx, double* x,
                            double* jac, double* fx);

/* Synchronising.  Preconditioned map (Sec. 5.2): trains the map on given
 * samples {x, f(x)} (from MCMC, a peak finder, ...) before integrating.  Each
 * of n_iter passes finds every point's increment on every axis by inverting
 * the current map, takes its Jacobian J (the product over the axes of
 * N_g Delta x_i), sets
 *   d_i^mu = (1 / n_i^mu) sum over the points in increment i of (J f)^2
 * (H and W of vp_accum_get then hold these sums and counts), and refines the
 * map from them with damping alpha as after an iteration.  The same points
 * serve every pass.  The allocation and the estimates are not touched; run
 * the integration afterwards (alpha = 0 in the problem's parameters keeps the
 * trained map).
 *  x: host [n][dim], every point inside the integration box; f: host [n],
 *  finite.  The arrays are copied; VP_ERR_INVALID_ARG on points outside the
 *  box or non-finite values. */
vp_status vp_map_train(vp_problem* p, int64_t n, const double* x, const double* f, int32_t n_iter, double alpha);

/* For callers that cannot allocate device memory (code running under HIP
 * graph capture elsewhere on the device, tight serving loops, harnesses that
 * forbid allocation): vp_map_train with the same arguments, results and
 * errors, except that it allocates nothing.  The points, their values and
 * the launch records are staged in a static 32 MiB device workspace of the
 * library (one per device, held until the process ends) instead of a buffer
 * allocated per call; x (n * dim doubles) and f (n doubles) must fit in it
 * with about 1 KiB to spare, else VP_ERR_INVALID_ARG.  The workspace is
 * shared by every call on a device: calls that overlap on one device (from
 * several threads, or on several problems whose streams run at once) race
 * and give undefined results.  Synchronising. */
vp_status vp_map_train_noalloc(vp_problem* p, int64_t n, const double* x, const double* f, int32_t n_iter,
                               double alpha);

/* Checkpoint: map, n_h, iteration index and estimate history, as an opaque
 * byte blob.  With buf == NULL, *size receives the required size. */
vp_status vp_state_export(vp_problem* p, void* buf, size_t* size);
vp_status vp_state_import(vp_problem* p, const void* buf, size_t size);

/* Profiling: total device time (ms, from HIP events on the context stream)
 * and launch count of one kernel family since creation or the last reset.
 * which: 0 sampling kernel, 1 whole iteration.  Timing is off until
 * vp_profile_enable(p, 1). */
vp_status vp_profile_enable(vp_problem* p, int32_t on);
vp_status vp_kernel_time(vp_problem* p, int32_t which, double* total_ms, int64_t* launches);

/* Convenience: create, run params->n_iter iterations, read the result,
 * destroy (synchronising). */
vp_status vp_integrate(vp_ctx* ctx, const vp_params* params, const vp_integrand* f,
                       vp_result* out);

/* ---------------------------------------------------------------- serving
 * A server integrates many independent requests on one GPU with continuous
 * batching (not in the paper; the per-request computation is exactly the
 * iteration above).  A scheduler thread admits submitted requests while the
 * device-memory budget and the slot count allow, keeps every admitted
 * request's state (map, allocation, sums, history) resident, and runs one
 * batched step at a time: every kernel of one iteration is launched once for
 * all active requests (sampling once per kernel instantiation).  A request
 * that arrives while others run is admitted at the next step boundary;
 * finished requests are retired at once, freeing memory for the queue.
 * With an unchanged set of active requests a step is replayed from a
 * captured HIP graph.  Each request computes what vp_integrate computes for
 * it, up to the order of floating-point sums: its sampling grid is sized
 * from the request alone, so its samples, counts and increment indices do
 * not depend on the mix; the order of the LDS-atomic additions into the
 * increment histograms is not fixed by the hardware, in or out of a mix.
 *
 * mem_budget_bytes: device bytes all active requests may hold (0: 3/4 of
 * the device's free memory).  max_slots: most requests active at once.
 * flags: VP_SERVER_NO_GRAPH launches every step directly.
 * The server uses its own stream on the context's device. */
enum { VP_SERVER_NO_GRAPH = 1 };

typedef struct {
    int64_t steps;          /* batched steps run */
    int64_t completed;      /* requests finished */
    int64_t cancelled;
    int64_t failed;
    int64_t samples;        /* samples drawn by finished requests */
    int64_t graph_launches; /* steps replayed from a captured graph */
    int64_t graph_captures;
    int32_t active;
    int32_t pending;
    int32_t peak_active;
    int32_t pad;
    int64_t mem_in_use;
    int64_t mem_peak;
    /* seconds spent by the scheduler: admitting (creating device state),
     * building plans and capturing graphs, running steps on the GPU
     * (enqueue to completion), and retiring (results, freeing) */
    double t_admit, t_plan, t_step, t_retire;
} vp_server_stats;

vp_status vp_server_create(vp_ctx* ctx, size_t mem_budget_bytes, int32_t max_slots, int32_t flags,
                           vp_server** out);
/* Thread-safe.  Copies params and integrand; fails with VP_ERR_INVALID_ARG
 * as vp_problem_create would, or VP_ERR_OOM when the request alone exceeds
 * the budget.  *ticket identifies the request. */
vp_status vp_server_submit(vp_server* s, const vp_params* params, const vp_integrand* f, uint64_t* ticket);
/* Thread-safe.  n requests at once (params[i], f[i]; tickets[i] receives
 * request i's ticket): all are checked as vp_server_submit checks one, and
 * either all are queued together -- in array order, so that the scheduler
 * sees them in one admission turn -- or none is (the status of the first
 * request that fails, its index in the detail message). */
vp_status vp_server_submit_many(vp_server* s, int32_t n, const vp_params* params, const vp_integrand* f,
                                uint64_t* tickets);
/* Thread-safe.  Device bytes the request would hold while admitted (the
 * figure the memory budget is charged), without submitting it. */
vp_status vp_server_request_bytes(vp_server* s, const vp_params* params, const vp_integrand* f, size_t* bytes);
/* Thread-safe.  VP_OK with the result once finished, VP_ERR_NOT_READY
 * before, VP_ERR_CANCELLED after a cancellation; a request that failed on
 * the device returns its error. */
vp_status vp_server_poll(vp_server* s, uint64_t ticket, vp_result* out);
/* Thread-safe; blocks until the request has finished (or was cancelled). */
vp_status vp_server_wait(vp_server* s, uint64_t ticket, vp_result* out);
/* Thread-safe.  Seconds on the server's monotonic clock (0 at creation):
 * submission, admission (-1 if not yet) and completion (-1 if not yet). */
vp_status vp_server_times(vp_server* s, uint64_t ticket, double* t_submit, double* t_admit, double* t_finish);
vp_status vp_server_now(vp_server* s, double* t);
/* Thread-safe.  A pending request is dropped; an active one is retired at
 * the next step boundary. */
vp_status vp_server_cancel(vp_server* s, uint64_t ticket);
vp_status vp_server_stats_get(vp_server* s, vp_server_stats* out);
/* Cancels what is left, stops the scheduler and frees everything. */
vp_status vp_server_destroy(vp_server* s);

#ifdef __cplusplus
}
#endif

#endif /* VEGASP_H */
