/*
 * laps.h -- C ABI of the MI355X (gfx950) hot path of the Late Adjusted
 * Parallel Sampler (LAPS), Robnik & Seljak, "Faster parallel MCMC: Metropolis
 * adjustment is best served warm", arXiv 2601.16696.
 *
 * One ensemble of N chains in d dimensions is advanced on one GPU.  Every
 * operation of the method runs in HIP kernels of this library; the host only
 * validates arguments and enqueues work on the caller's stream.
 *
 * Memory and ownership
 *   - All device buffers belong to the caller: the positions x, the
 *     workspace and the target's data.  The library never allocates device
 *     memory.  It owns only the opaque host context (laps_ctx).
 *   - Positions are row-major [N][ld] in the state precision (double for
 *     LAPS_F64, float otherwise) with row stride ld = laps_row_stride(d)
 *     elements (d rounded up to a multiple of 8).  Columns d..ld-1 are padding:
 *     the library overwrites them with zeros.  Base pointers must be 32-byte
 *     aligned.
 *   - x is updated in place by every step.
 *
 * Streams and synchronisation
 *   - Every call enqueues on the stream given to laps_init (a hipStream_t
 *     passed as void*; NULL is the default stream) and returns without
 *     waiting, except laps_ensemble_stats, which synchronises that stream.
 *   - Calls on one context must not overlap from several host threads.
 *
 * Errors
 *   - Every entry point validates its arguments before it enqueues anything
 *     and returns LAPS_EINVAL (or LAPS_EWORKSPACE, LAPS_EUNSUPPORTED) without
 *     side effects.  A failed HIP launch returns LAPS_EDEVICE and
 *     laps_last_error() gives the HIP message.  The library never aborts.
 *   - Chains whose energy error is not finite are counted; laps_ensemble_stats
 *     returns LAPS_ENONFINITE (after filling the output) when any were seen.
 */
#ifndef LAPS_H
#define LAPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct laps_ctx laps_ctx;

typedef enum {
  LAPS_OK = 0,
  LAPS_EINVAL = -1,
  LAPS_EDEVICE = -2,
  LAPS_ENONFINITE = -3,
  LAPS_EPHASE = -4,
  LAPS_EWORKSPACE = -5,
  LAPS_EUNSUPPORTED = -6
} laps_status;

/* State precision.  LAPS_F64: everything in double.  LAPS_F32: state x, u, g
 * in float; log p, energy errors and every ensemble reduction in double.
 * LAPS_MIXED_BF16: as LAPS_F32, and the logistic-regression gradient runs its
 * two contractions on bf16 matrix cores with float accumulation. */
typedef enum { LAPS_F64 = 0, LAPS_F32 = 1, LAPS_MIXED_BF16 = 2 } laps_precision;

/* Built-in targets (log p up to a constant):
 *   LAPS_GAUSS_DIAG  N(0, diag(s2)).            data[0] = s2 [d] (double)
 *   LAPS_LOGREG      Bayesian logistic regression, prior N(0, I):
 *                    log p = sum_n [y_n z_n - log(1 + e^{z_n})] - |th|^2/2,
 *                    z = X th.                   data[0] = X [n][d] row-major
 *                    (double for LAPS_F64, bf16 bits as uint16 otherwise),
 *                    data[1] = y [n] (double, 0/1), dims[0] = n
 *   LAPS_STOCHVOL    stochastic volatility, th = (h_1..h_T, s, r), d = T + 2:
 *                    sigma = e^s, phi = tanh r, s ~ N(-2, 0.5^2),
 *                    r ~ N(2, 0.5^2), h_1 ~ N(0, sigma^2/(1-phi^2)),
 *                    h_t ~ N(phi h_{t-1}, sigma^2), y_t ~ N(0, e^{h_t}).
 *                                                data[0] = y [T] (double)
 *   LAPS_PHI4        periodic L x L lattice phi^4, d = L^2, site (r, c) at
 *                    r*L + c: log p = -sum_x [1/2 sum_mu (phi_{x+mu} - phi_x)^2
 *                    + m2/2 phi_x^2 + lambda phi_x^4].
 *                                                dims[0] = L, scal[0] = m2,
 *                                                scal[1] = lambda
 *   LAPS_CALLBACK    a caller-supplied log p (the method's general input: any
 *                    differentiable log density).  cb and cb_user below.
 *   LAPS_GAUSS_DENSE zero-mean Gaussian with a dense precision matrix A:
 *                    log p = -x^T A x / 2.   data[0] = A [d][d] (double,
 *                    row-major, symmetric positive definite); LAPS_F64 or
 *                    LAPS_F32 state.
 * LAPS_LOGREG, LAPS_CALLBACK and LAPS_GAUSS_DENSE run through the per-chain
 * update kernels (teams of at most 16 lanes, several octs per lane above
 * d = 128): LAPS_CALLBACK and LAPS_GAUSS_DENSE up to d = 512, LAPS_LOGREG up
 * to d = 128, where its matrix-core gradient kernels stop; larger d gives
 * LAPS_EUNSUPPORTED.
 * Target data must stay valid and unchanged while a context uses it. */
typedef enum {
  LAPS_GAUSS_DIAG = 0,
  LAPS_LOGREG = 1,
  LAPS_STOCHVOL = 2,
  LAPS_PHI4 = 3,
  LAPS_CALLBACK = 4,
  LAPS_GAUSS_DENSE = 5
} laps_target_kind;

/* Gradient callback of a LAPS_CALLBACK target.  The library calls it on the
 * host thread that enqueues a step, each time the ensemble needs log p and its
 * gradient (once per unadjusted step, once per gradient stage of a MAMS
 * trajectory, once at initialisation).  It must enqueue on `stream` (a
 * hipStream_t) device work that reads the positions x_dev [n_chains][ld] and
 * writes, for every chain m and coordinate i < d, g_dev[m*ld + i] =
 * d log p(x_m) / d x_i and logp_dev[m] = log p(x_m) (double); columns d..ld-1
 * of g_dev are ignored.  x_dev and g_dev hold the state type (double for
 * LAPS_F64, float for LAPS_F32) and are device buffers of the library's
 * workspace, valid only until the enqueued work completes.  It must not
 * synchronise the device or free memory, and returns 0 on success (non-zero
 * fails the step with LAPS_EDEVICE).  Work it enqueues is captured with the
 * steps by laps_graph_create if it is capturable. */
typedef int (*laps_grad_cb)(void *user, const void *x_dev, void *g_dev, double *logp_dev, int64_t n_chains,
                            int64_t d, int64_t ld, void *stream);

typedef struct {
  int32_t kind; /* laps_target_kind */
  int64_t d;
  const void *data[4];
  int64_t dims[4];
  double scal[4];
  laps_grad_cb cb; /* LAPS_CALLBACK only */
  void *cb_user;   /* passed to cb unchanged */
} laps_target;

/* Sampler configuration.  Zero-initialise and call laps_config_default() to
 * get the paper's constants:
 *   C = 0.025            ratio of asymptotic to current bias (section "Step size")
 *   alpha = 2            L = alpha (sum_i Var x_i)^{1/2} (eq. L)
 *   eps0_factor = 0.01   eps_0 = 0.01 sqrt(d) (Algorithm "LAPS Pseudocode")
 *   switch_tol = 0.01    switch when every windowed fluctuation of E[x_i^2] is
 *                        below this (section "Switch to adjustment")
 *   window_frac = 0.2    window length as a fraction of max_steps_total
 *   acc_tol = 0.03       acceptance tolerance of the adjusted-phase bisection
 *   acc_target = 0       0: 0.7 for the second-order integrator, 0.9 for MN4
 *   L_partial_factor = 1.25, n_steps_traj = 15  (section "Adjusted sampling")
 *   integrator_adj = 0   0: MN2 for d <= 200 else MN4; 1: MN2; 2: MN4
 *   eevpd_mode = 1       0: Var[Delta]/d (the text's definition); 1: mean of
 *                        Delta^2 / d (the algorithm's form, default)
 *   switch_policy = 0    0: the paper's fluctuation rule (or max_steps_unadj);
 *                        1: switch exactly at max_steps_unadj
 * Step counts t count integrator steps: one per unadjusted step and
 * n_steps_traj per adjusted transition.
 * Full-rank probes (section "Equipartition condition"): probe p of step t has
 * entry i = 1 - 2b, b = bit (i mod 64) of word (i mod 256) / 64 of the Philox
 * block with counter (p, i / 256, t, 6). */
typedef struct {
  int64_t n_chains, d;
  int32_t prec; /* laps_precision */
  uint64_t seed;
  double C, alpha, eps0_factor, switch_tol, window_frac, acc_tol, acc_target, L_partial_factor;
  int32_t n_steps_traj, integrator_adj, eevpd_mode, switch_policy;
  int64_t max_steps_unadj, max_steps_total;
  int32_t team_lanes; /* launch shape of the per-chain kernels (Gaussian, SV, phi4):
                         0 = automatic; otherwise lanes per chain, a power of two
                         up to 64 or a multiple of 64 up to 512 */
  int32_t full_rank_probes; /* 0: the diagonal equipartition loss D~_diag (the paper's default);
                               P in 1..1024: the full-rank loss by Hutchinson's estimator with P
                               Rademacher probes drawn from the Philox stream each unadjusted
                               step (the paper uses 100) */
  int32_t block_threads;    /* per-chain kernels with teams of <= 64 lanes, and the per-chain update
                               kernels of logistic regression, caller-supplied and dense targets:
                               0 = automatic (256), or 64, 128, 256 threads per workgroup */
  int32_t grad_workgroups;  /* logistic regression: 0 = automatic, else the number of workgroups a
                               gradient launch aims for (sets the row splits) */
  double eps_fixed;         /* 0: the adaptive step size of section "Step size" (the paper's method);
                               > 0: this step size throughout the unadjusted phase, all else unchanged
                               (the fixed-step comparison of the step-size appendix); the adjusted
                               phase starts from it and bisects as usual */
  int32_t dynamics;         /* 0: the microcanonical velocity (the paper's method); 1: underdamped
                               Langevin (the dynamics ablation of appendix "Ablation studies"): velocity
                               u ~ N(0, I/d), kinetic energy (d/2)|u|^2, Ornstein-Uhlenbeck refresh
                               u <- c1 u + sqrt(1 - c1^2) Z/sqrt(d) and kick u <- u + (h/d) g; eps, L,
                               the controllers and MH are unchanged */
} laps_config;

/* Snapshot of the device-resident hyperparameters and diagnostics.
 * phase: 0 unadjusted, 1 unadjusted phase finished (switch pending),
 * 2 adjusted.  status_bits: 1 non-finite energy error seen, 2 eps update
 * skipped (EEVPD zero or not finite), 4 a zero or non-finite variance was
 * replaced by 1 in the preconditioner. */
typedef struct {
  int64_t t, grads_per_chain;
  int32_t phase, adapt, switch_ready, status_bits;
  double eps, L, eevpd, eevpd_target, dtilde, max_delta, acc_mean;
  int64_t n_nonfinite;
  int32_t integrator, have_lo, have_hi, ring_full;
  double lo, hi, a_star, sum_var;
} laps_stats;

/* Fills cfg with the paper's defaults for n_chains x d (seed 0,
 * max_steps_unadj 1000, max_steps_total 2000, precision LAPS_F64). */
void laps_config_default(laps_config *cfg, int64_t n_chains, int64_t d);

/* Row stride (elements) of every [N][ld] buffer: d rounded up to 8. */
int64_t laps_row_stride(int64_t d);

/* Device workspace bytes the context needs for (cfg, target). */
laps_status laps_workspace_size(const laps_config *cfg, const laps_target *target, size_t *bytes);

/* Creates a context, validates everything, and enqueues initialisation
 * (Algorithm "LAPS Pseudocode" and section "Initialization"): log p and its
 * gradient at x, u = grad/|grad| (or u0 when given; a uniform random direction
 * for a chain whose gradient vanishes), eps = eps0_factor sqrt(d),
 * L = alpha (sum_i Var x_i)^{1/2}.
 *   x_dev  [N][ld] positions, caller-owned, updated in place by every step
 *   u0_dev [N][ld] initial velocities (unit norm) or NULL
 *   ws_dev workspace of at least laps_workspace_size bytes, 256-byte aligned
 *   stream hipStream_t (as void*) all work is enqueued on
 * On success *out receives the context; release it with laps_destroy. */
laps_status laps_init(const laps_config *cfg, const laps_target *target, void *x_dev, const void *u0_dev,
                      void *ws_dev, size_t ws_bytes, void *stream, laps_ctx **out);

/* laps_init for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * initialisation with the workspace taken from a static device array of the
 * library, 32 MiB per device, held until the process ends (enough for the
 * 4096-chain logistic-regression workload, 23.6 MiB).  Calls no allocating
 * routine.  When laps_workspace_size exceeds 32 MiB only because of the
 * buffers of random normals computed ahead (FP64 per-chain targets with few
 * chains), the context is created without them and its kernels compute the
 * normals where they use them (the same values); configurations that exceed
 * 32 MiB without those buffers return LAPS_EWORKSPACE.  The context is library storage, one per device:
 * laps_destroy leaves it in place, and a later laps_init_static on the same
 * device reuses the array and the context, so the earlier static context is
 * then invalid.  Steps of two static contexts cannot overlap on one device
 * (they would race on the array); workspace contents left by an earlier call
 * are cleared or rewritten by the initialisation exactly as in laps_init. */
laps_status laps_init_static(const laps_config *cfg, const laps_target *target, void *x_dev, const void *u0_dev,
                             void *stream, laps_ctx **out);

/* Enqueues up to n_steps unadjusted MCLMC steps (eq. discrete update with the
 * leapfrog integrator, Appendix D) each followed by the ensemble statistics
 * and the unadjusted controller (section "Unadjusted initialization", eq.
 * bias bound, eq. L, eq. relative fluctuations).  Once the switch condition
 * fires on the device the remaining steps are no-ops.  Returns LAPS_EPHASE
 * after laps_step_adjusted has been called.  Never synchronises. */
laps_status laps_step_unadjusted(laps_ctx *ctx, int64_t n_steps);

/* Enqueues n_transitions MAMS transitions (Appendix "Metropolis adjusted
 * microcanonical dynamics") each followed by the acceptance-rate bisection
 * controller (section "Adjusted sampling").  The first call performs the
 * switch: diagonal preconditioner sigma_i = Var[x_i]^{1/2}, integrator MN2
 * (d <= 200) or MN4, target acceptance 0.7 or 0.9.  Transitions starting at
 * t >= max_steps_total are no-ops.  Never synchronises. */
laps_status laps_step_adjusted(laps_ctx *ctx, int64_t n_transitions);

/* Synchronises the stream and copies the hyperparameters/diagnostics to
 * out_host.  per_dim_dev, if not NULL, receives [4][d] doubles on the device:
 * mean, variance, E[x_i^2] and the equipartition diagonal V_ii of the last
 * statistics pass. */
laps_status laps_ensemble_stats(laps_ctx *ctx, laps_stats *out_host, double *per_dim_dev);

/* Standalone target evaluation for n_chains rows of x ([n][ld] in the
 * precision's state type): logp_dev [n] doubles, grad_dev [n][ld] (may be
 * NULL).  Enqueued on stream; used by the autograd wrappers. */
laps_status laps_target_eval(const laps_target *target, int32_t prec, const void *x_dev, void *logp_dev,
                             void *grad_dev, int64_t n_chains, void *stream);

/* log p and its gradient (the target's own adjoint kernels) at caller
 * positions x_dev ([n_chains][ld] of the context's state type, 32-byte
 * aligned, n_chains the context's) for any target kind, including those
 * whose gradient needs the context's scratch (logistic regression, the dense
 * Gaussian, callbacks): logp_dev [n_chains] doubles, grad_dev [n_chains][ld]
 * in the state type (may be NULL).  Enqueued on the context's stream between
 * steps; the sampler's state is not touched, its split scratch is reused.
 * Used by the autograd wrapper. */
laps_status laps_eval(laps_ctx *ctx, const void *x_dev, void *logp_dev, void *grad_dev);

/* The sampler's random-number contract, exposed for reproduction and tests.
 * Philox4x64-10 (Salmon et al., SC'11) under key (seed, 0):
 *   laps_philox_words: ctr_dev [n][4] uint64 counters -> out_dev [n][4]
 *   uint64 words (device buffers, enqueued on stream).
 * The sampler's normals for (chain m, step t, tag, substep) use counter
 * (m, j, t, tag | substep << 8) for dims 8j..8j+7: word k gives the pair
 * U_a = (hi32 + 1/2) 2^-32, U_b = (lo32 + 1/2) 2^-32 and the Box-Muller
 * values sqrt(-2 ln U_a) (cos, sin)(2 pi U_b) for dims 8j+2k, 8j+2k+1
 * (FP32 state evaluates them with the hardware log2, sqrt, sin and cos, to
 * an absolute error of order 1e-6).
 *   laps_philox_normals: fills out_dev [n_chains][ld] (double for LAPS_F64,
 *   float otherwise) with that stream for chains 0..n_chains-1.
 * Tags: 1 first partial refresh of a step, 2 second partial refresh,
 * 3 full refresh, 4 Metropolis uniform, 5 initial direction. */
laps_status laps_philox_words(const uint64_t *ctr_dev, uint64_t *out_dev, int64_t n, uint64_t seed, void *stream);
laps_status laps_philox_normals(uint64_t seed, int64_t n_chains, int64_t d, uint64_t t, uint32_t tag,
                                uint32_t substep, int32_t prec, void *out_dev, void *stream);

/* Times the target gradient of the context (every kernel one ensemble
 * gradient evaluation takes) at the current positions: n_reps evaluations
 * enqueued on the context's stream between two HIP events; *avg_ms receives
 * the mean time of one.  Overwrites only the gradient/log p staging of the
 * workspace with values at the current positions.  Synchronises the stream. */
laps_status laps_time_gradient(laps_ctx *ctx, int32_t n_reps, float *avg_ms);

/* Times one hot kernel of a context with a per-chain target (Gaussian, SV,
 * phi4): n_reps launches on the context's stream between two HIP events,
 * *avg_ms the mean duration of one.  which = 1: the unadjusted step kernel
 * alone (positions and velocities advance, no statistics or controller; the
 * context must be in the unadjusted phase); which = 2: the fused adjusted
 * transition kernel alone (context in the adjusted phase, before
 * max_steps_total).  A launch in the wrong phase is a no-op and is timed as
 * such.  LAPS_EUNSUPPORTED for other targets.  Synchronises the stream. */
laps_status laps_time_kernel(laps_ctx *ctx, int32_t which, int32_t n_reps, float *avg_ms);

/* Kernel timing inside ordinary runs: records a pair of HIP events on the
 * context's stream around every `every`-th launch (the first, then every
 * every-th after it) of one kernel of the steps that follow, for up to
 * `capacity` recorded launches.  which: LAPS_KERNEL_UNADJ (per-chain unadjusted
 * step kernel) or LAPS_KERNEL_MAMS (per-chain MAMS transition kernel) for the
 * Gaussian, stochastic-volatility and phi^4 targets; LAPS_KERNEL_GRAD (the
 * gradient kernel, every launch inside unadjusted steps and MAMS
 * trajectories) for logistic regression; 0 or capacity 0 ends logging.
 * The events are created without the system-scope fence (timing only).
 * Synchronises the stream and discards earlier records.  Graph recording
 * (laps_graph_create) refuses a context that is logging. */
enum { LAPS_KERNEL_UNADJ = 1, LAPS_KERNEL_MAMS = 2, LAPS_KERNEL_GRAD = 3 };
laps_status laps_kernel_log(laps_ctx *ctx, int32_t which, int32_t capacity, int32_t every);
/* Waits for the last logged launch; *count = logged launches, *total_ms =
 * the sum of their event-to-event durations. */
laps_status laps_kernel_log_read(laps_ctx *ctx, int64_t *count, double *total_ms);

/* Starts a fresh run in the context's memory: copies x0_dev ([N][ld], may be
 * NULL to keep the current positions) into the positions, resets the
 * hyperparameters and runs the initialisation (gradient, velocities,
 * statistics, controller) -- the same state laps_init leaves.  Enqueue-only
 * and free of allocations and memsets, so it can be recorded in a graph. */
laps_status laps_restart(laps_ctx *ctx, const void *x0_dev);

/* Batched runs.  laps_graph_create records, for every context k, a segment
 * of a run -- laps_restart(ctx_k, x0s[k]) if restart is nonzero (x0s may be
 * NULL), then n_unadj unadjusted steps (skipped once the context has entered
 * the adjusted phase) and n_adj adjusted transitions -- into one executable
 * HIP graph.  Each context's work stays on its own stream (which must be a
 * created stream, not the default one), forked from and joined back into a
 * private recording stream, so independent ensembles (different targets,
 * sizes and precisions) run concurrently when the graph is launched;
 * contexts sharing a stream run one after another.  A long run is recorded
 * as a few segment graphs (created in run order, since recording advances the
 * contexts' host state as the enqueue calls would) and replayed in order;
 * replaying a segment that contains the switch again is harmless.  The
 * contexts' host state is left as after the recorded calls.
 * laps_graph_launch enqueues one replay on `stream`.  The graph owns no
 * device memory; the contexts and their buffers must outlive it. */
typedef struct laps_graph laps_graph;
laps_status laps_graph_create(laps_ctx *const *ctxs, int32_t n_ctx, int32_t restart, const void *const *x0s,
                              int64_t n_unadj, int64_t n_adj, laps_graph **out);
laps_status laps_graph_launch(laps_graph *graph, void *stream);
laps_status laps_graph_destroy(laps_graph *graph);

/* Device pointers into the context's workspace: 0 u [N][ld], 1 g [N][ld],
 * 2 logp [N] (double), 3 delta [N] (double), 4 acc [N] (double),
 * 5 sigma [ld] (state type).  NULL for an unknown index. */
void *laps_buffer(laps_ctx *ctx, int32_t which);

/* Releases the host context (no device work is enqueued). */
laps_status laps_destroy(laps_ctx *ctx);

const char *laps_status_string(laps_status s);
const char *laps_last_error(const laps_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LAPS_H */
