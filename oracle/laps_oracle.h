/*
 * Plain FP64 CPU oracle of the Late Adjusted Parallel Sampler (LAPS),
 * Robnik & Seljak, "Faster parallel MCMC: Metropolis adjustment is best
 * served warm" (arXiv 2601.16696).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code with the GPU library: no headers, no helpers, no constant tables.
 *
 * Every function is single-threaded plain loops in double precision.
 * Ensemble sums run in chain order with Neumaier compensation; all
 * ensemble averages divide by M (the number of chains).
 *
 * Parity pins: see the test files under tests/ (oracle pins) -- each
 * function below names the passage of the paper it follows.
 */
#ifndef LAPS_ORACLE_H
#define LAPS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- counter-based random numbers (Philox4x64-10, Salmon et al. SC'11) ---- */
enum { ORC_TAG_O_FIRST = 1, ORC_TAG_O_SECOND = 2, ORC_TAG_FULL_REFRESH = 3,
       ORC_TAG_MH = 4, ORC_TAG_INIT_DIR = 5, ORC_TAG_PROBE = 6 };

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double orc_u01(uint64_t w);
/* d standard normals for (chain, step t, tag, substep). */
void orc_normals(uint64_t seed, uint64_t chain, uint64_t t, uint32_t tag,
                 uint32_t substep, int64_t d, double *z);
double orc_mh_uniform(uint64_t seed, uint64_t chain, uint64_t t);
/* Rademacher probe p of step t (entries +-1): entry i is 1 - 2 b, where b is
 * bit i mod 64 of word (i mod 256) / 64 of Philox block (p, i / 256, t, 6). */
void orc_rademacher(uint64_t seed, uint64_t t, int64_t p, int64_t d, double *z);

/* ---- targets (log p up to an additive constant, and its gradient) ---- */
enum { ORC_GAUSS_DIAG = 0, ORC_LOGREG = 1, ORC_STOCHVOL = 2, ORC_PHI4 = 3, ORC_GAUSS_DENSE = 5 };
typedef struct {
  int32_t kind;
  int64_t d;
  const double *a;  /* gauss: sigma^2 [d]; logreg: X [n][d]; stochvol: y [T]; gauss_dense: precision [d][d] */
  const double *b;  /* logreg: labels [n] in {0,1} */
  int64_t n;        /* logreg: n data rows; stochvol: T; phi4: side L */
  double p0, p1;    /* phi4: m^2, lambda */
} orc_target;

double orc_logp_grad(const orc_target *tg, const double *x, double *g);

/* ---- single-chain maps of the integrator (Appendix D) ---- */
void orc_map_O(double *u, const double *z, int64_t d, double h, double L);
double orc_map_B(double *u, const double *gt, int64_t d, double h);
void orc_map_A(double *x, const double *u, const double *sigma, int64_t d, double h);
/* Underdamped Langevin variant: velocity u ~ N(0, I/d) (mass d, so |u| ~ 1 and
 * eps, L keep the units of the microcanonical dynamics), kinetic energy
 * K(u) = (d/2)|u|^2. */
void orc_map_O_lang(double *u, const double *xi, int64_t d, double h, double L);
double orc_map_B_lang(double *u, const double *gt, int64_t d, double h);

/* coefficient sets: 0 = LF, 1 = MN2, 2 = MN4 */
int orc_integrator_coeffs(int which, double *b, double *a, int *K);

/* ---- ensemble sampler ---- */
typedef struct {
  int64_t n_chains, d;
  uint64_t seed;
  double C, alpha, eps0_factor, switch_tol, window_frac, acc_tol, acc_target, L_partial_factor;
  int32_t n_steps_traj, integrator_adj, eevpd_mode, switch_policy;
  int64_t max_steps_unadj, max_steps_total;
  int32_t full_rank_probes; /* 0: diagonal equipartition loss; P > 0: full rank, P Rademacher probes */
  double eps_fixed;         /* 0: the adaptive step size of the unadjusted phase; > 0: this step size
                               throughout the unadjusted phase (the fixed-step comparison of the
                               step-size appendix); the adjusted phase starts from it as usual */
  int32_t dynamics;         /* 0: microcanonical velocity (the method); 1: underdamped Langevin with a
                               Gaussian velocity (the dynamics ablation of appendix "Ablation studies") */
} orc_config;

typedef struct orc_ctx orc_ctx;

/* Full-rank equipartition loss by Hutchinson's trace estimator (section
 * "Equipartition condition", full-rank paragraph): for positions x and
 * gradients g of N chains ([N][d]) and P probes z ([P][d]),
 *   (1/(P d)) sum_p |z_p + (1/N) sum_m (x_m - xbar)(g_m . z_p)|^2,
 * the mean over probes of |(I - V) z|^2 / d with V from ensemble averages. */
double orc_dtilde_full(const double *x, const double *g, int64_t N, int64_t d, const double *z, int64_t P);

orc_ctx *orc_create(const orc_config *cfg, const orc_target *tg);
void orc_destroy(orc_ctx *c);
/* x0: [N][d]; u0 may be NULL (then u = g/|g|). */
int orc_init(orc_ctx *c, const double *x0, const double *u0);
/* moves every chain one unadjusted step with the current eps, L (no controller) */
void orc_unadj_move(orc_ctx *c);
/* ensemble statistics + unadjusted controller (eps, L, window, switch) */
void orc_unadj_control(orc_ctx *c);
int orc_step_unadjusted(orc_ctx *c, int64_t n);
void orc_do_switch(orc_ctx *c);
void orc_mams_move(orc_ctx *c);
void orc_adj_control(orc_ctx *c);
int orc_step_adjusted(orc_ctx *c, int64_t n);
int orc_run(orc_ctx *c);

/* accessors (arrays are owned by the context) */
typedef struct {
  int64_t t, grads_per_chain;
  int32_t phase, adapt, switch_ready, status_bits;
  double eps, L, eevpd, eevpd_target, dtilde, max_delta, acc_mean;
  int64_t n_nonfinite;
  int32_t integrator, have_lo, have_hi, ring_full;
  double lo, hi, a_star, sum_var;
} orc_stats;
void orc_get_stats(const orc_ctx *c, orc_stats *s);
double *orc_ptr(orc_ctx *c, int which);
void orc_set_hyper(orc_ctx *c, double eps, double L);

/* closed forms used by the controller */
double orc_F(double D);

/* neumaier-compensated sum of n doubles */
double orc_sum(const double *v, int64_t n);

#ifdef __cplusplus
}
#endif
#endif
