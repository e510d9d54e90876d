/*
 * Plain FP64 CPU oracle of LAPS (arXiv 2601.16696).
 *
 * TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It shares no code with the GPU path.
 *
 * Readings of the paper that are not fixed by its text are listed in the
 * repository's design notes under "Readings"; each is named below as R<n>
 * where it is taken.
 *
 * Parity status: every function here is pinned by a CPU test against a
 * closed form, a library routine, an invariant or brute force.  The
 * unadjusted controller trajectory as a whole (the eps(t) schedule and the
 * switch time) has no closed form: it is pinned by its single update's
 * arithmetic and by its equivariance under a change of units, and is
 * otherwise parity unpinned.
 */
#include "laps_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ======================================================================
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11,
 * "Parallel random numbers: as easy as 1, 2, 3").  The round function,
 * multipliers and Weyl key increments are those of the published
 * definition.  The sampler's own draws are addressed by counter
 * (chain, block, step, tag | substep << 8) under key (seed, 0).
 * ==================================================================== */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, &hi0, &lo0);
    mulhilo64(M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53 high bits, offset by half a unit: the result lies in (0, 1]. */
double orc_u01(uint64_t w) { return ((double)(w >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/* a 32-bit word offset by half a unit: exactly representable, in (0, 1). */
static double u01_32(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* d standard normals by the Box-Muller transform (Box & Muller 1958).  Philox
 * block j fills z[8j .. 8j+7]: word k gives the pair (U_a, U_b) from its high
 * and low 32 bits, z[8j+2k] = r cos(2 pi U_b), z[8j+2k+1] = r sin(2 pi U_b),
 * r = sqrt(-2 ln U_a). */
void orc_normals(uint64_t seed, uint64_t chain, uint64_t t, uint32_t tag,
                 uint32_t substep, int64_t d, double *z) {
  const uint64_t key[2] = {seed, 0};
  for (int64_t j = 0; 8 * j < d; ++j) {
    uint64_t ctr[4] = {chain, (uint64_t)j, t, (uint64_t)tag | ((uint64_t)substep << 8)};
    uint64_t w[4];
    orc_philox4x64_10(ctr, key, w);
    for (int k = 0; k < 4; ++k) {
      double ua = u01_32((uint32_t)(w[k] >> 32)), ub = u01_32((uint32_t)w[k]);
      double r = sqrt(-2.0 * log(ua));
      double ang = 2.0 * M_PI * ub;
      int64_t i0 = 8 * j + 2 * k;
      if (i0 < d) z[i0] = r * cos(ang);
      if (i0 + 1 < d) z[i0 + 1] = r * sin(ang);
    }
  }
}

double orc_mh_uniform(uint64_t seed, uint64_t chain, uint64_t t) {
  const uint64_t key[2] = {seed, 0};
  uint64_t ctr[4] = {chain, 0, t, (uint64_t)ORC_TAG_MH}, w[4];
  orc_philox4x64_10(ctr, key, w);
  return orc_u01(w[0]);
}

void orc_rademacher(uint64_t seed, uint64_t t, int64_t p, int64_t d, double *z) {
  const uint64_t key[2] = {seed, 0};
  for (int64_t i = 0; i < d; ++i) {
    uint64_t ctr[4] = {(uint64_t)p, (uint64_t)(i / 256), t, (uint64_t)ORC_TAG_PROBE}, w[4];
    orc_philox4x64_10(ctr, key, w);
    const int64_t b = i % 256;
    const uint64_t bit = (w[b / 64] >> (b % 64)) & 1u;
    z[i] = bit ? -1.0 : 1.0;
  }
}

/* ======================================================================
 * Compensated summation (Neumaier 1974) in the given order.
 * ==================================================================== */
double orc_sum(const double *v, int64_t n) {
  double s = 0.0, comp = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t = s + v[i];
    if (fabs(s) >= fabs(v[i])) comp += (s - t) + v[i];
    else comp += (v[i] - t) + s;
    s = t;
  }
  return s + comp;
}

typedef struct { double s, c; } nsum;
static void nsum_add(nsum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static double nsum_get(const nsum *a) { return a->s + a->c; }

/* ======================================================================
 * Targets.  log p is returned up to an additive constant.
 * ==================================================================== */
static double softplus(double z) { return (z > 0 ? z : 0.0) + log1p(exp(-fabs(z))); }
static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Diagonal Gaussian N(0, diag(sigma^2)). */
static double t_gauss(const orc_target *tg, const double *x, double *g) {
  double l = 0.0;
  for (int64_t i = 0; i < tg->d; ++i) {
    double s2 = tg->a[i];
    l += -0.5 * x[i] * x[i] / s2;
    if (g) g[i] = -x[i] / s2;
  }
  return l;
}

/* Bayesian logistic regression with a N(0, I) prior: z = X theta,
 * log p = sum_n [y_n z_n - softplus(z_n)] - |theta|^2 / 2. */
static double t_logreg(const orc_target *tg, const double *th, double *g) {
  const int64_t d = tg->d, n = tg->n;
  const double *X = tg->a, *y = tg->b;
  double l = 0.0;
  if (g) for (int64_t i = 0; i < d; ++i) g[i] = -th[i];
  for (int64_t i = 0; i < d; ++i) l -= 0.5 * th[i] * th[i];
  for (int64_t r = 0; r < n; ++r) {
    double z = 0.0;
    for (int64_t i = 0; i < d; ++i) z += X[r * d + i] * th[i];
    l += y[r] * z - softplus(z);
    if (g) {
      double res = y[r] - sigmoid(z);
      for (int64_t i = 0; i < d; ++i) g[i] += res * X[r * d + i];
    }
  }
  return l;
}

/* Stochastic volatility, theta = (h_1..h_T, s, r), sigma = e^s, phi = tanh r:
 * s ~ N(-2, 0.5^2), r ~ N(2, 0.5^2), h_1 ~ N(0, sigma^2/(1-phi^2)),
 * h_t ~ N(phi h_{t-1}, sigma^2), y_t ~ N(0, e^{h_t}). */
static double t_stochvol(const orc_target *tg, const double *x, double *g) {
  const int64_t T = tg->n;
  const double *y = tg->a;
  const double *h = x;
  const double s = x[T], r = x[T + 1];
  const double sig2 = exp(2.0 * s), phi = tanh(r), omp = 1.0 - phi * phi;
  double E = omp * h[0] * h[0];
  double cross = phi * h[0] * h[0];  /* phi h_1^2 + sum a_t h_{t-1} */
  double lik = 0.0;
  for (int64_t t = 1; t < T; ++t) {
    double a = h[t] - phi * h[t - 1];
    E += a * a;
    cross += a * h[t - 1];
  }
  for (int64_t t = 0; t < T; ++t) lik += -0.5 * h[t] - 0.5 * y[t] * y[t] * exp(-h[t]);
  double l = -2.0 * (s + 2.0) * (s + 2.0) - 2.0 * (r - 2.0) * (r - 2.0)
             - (double)T * s + 0.5 * log(omp) - E / (2.0 * sig2) + lik;
  if (g) {
    for (int64_t t = 0; t < T; ++t) {
      /* q_t = dE/dh_t / 2, E = (1-phi^2) h_1^2 + sum_{t>=2} a_t^2, a_t = h_t - phi h_{t-1} */
      const double a_n = (t + 1 < T) ? (h[t + 1] - phi * h[t]) : 0.0;
      const double own = (t == 0) ? omp * h[0] : (h[t] - phi * h[t - 1]);
      const double q = own - phi * a_n;
      g[t] = -q / sig2 - 0.5 + 0.5 * y[t] * y[t] * exp(-h[t]);
    }
    g[T] = -4.0 * (s + 2.0) - (double)T + E / sig2;
    g[T + 1] = -4.0 * (r - 2.0) - phi + omp * cross / sig2;
  }
  return l;
}

/* 2-D lattice phi^4 on an L x L periodic lattice, site (row, col) -> row*L+col:
 * S = sum_x [ 1/2 sum_mu (phi_{x+mu} - phi_x)^2 + m2/2 phi_x^2 + lambda phi_x^4 ],
 * log p = -S. */
static double t_phi4(const orc_target *tg, const double *x, double *g) {
  const int64_t L = tg->n;
  const double m2 = tg->p0, lam = tg->p1;
  double S = 0.0;
  for (int64_t r = 0; r < L; ++r)
    for (int64_t c = 0; c < L; ++c) {
      double f = x[r * L + c];
      double fr = x[r * L + (c + 1) % L], fd = x[((r + 1) % L) * L + c];
      S += 0.5 * (fr - f) * (fr - f) + 0.5 * (fd - f) * (fd - f) + 0.5 * m2 * f * f + lam * f * f * f * f;
      if (g) {
        double fl = x[r * L + (c + L - 1) % L], fu = x[((r + L - 1) % L) * L + c];
        g[r * L + c] = (fr + fl + fd + fu) - (4.0 + m2) * f - 4.0 * lam * f * f * f;
      }
    }
  return -S;
}

/* Gaussian with a dense precision matrix A (the rotated ill-conditioned
 * Gaussian of section "Results"): log p = -x^T A x / 2, gradient -A x. */
static double t_gauss_dense(const orc_target *tg, const double *x, double *g) {
  const int64_t d = tg->d;
  double l = 0.0;
  for (int64_t i = 0; i < d; ++i) {
    double ax = 0.0;
    for (int64_t k = 0; k < d; ++k) ax += tg->a[i * d + k] * x[k];
    l += -0.5 * x[i] * ax;
    if (g) g[i] = -ax;
  }
  return l;
}

double orc_logp_grad(const orc_target *tg, const double *x, double *g) {
  switch (tg->kind) {
    case ORC_GAUSS_DIAG: return t_gauss(tg, x, g);
    case ORC_GAUSS_DENSE: return t_gauss_dense(tg, x, g);
    case ORC_LOGREG: return t_logreg(tg, x, g);
    case ORC_STOCHVOL: return t_stochvol(tg, x, g);
    case ORC_PHI4: return t_phi4(tg, x, g);
    default: return NAN;
  }
}

/* ======================================================================
 * Maps of the splitting integrator (Appendix D).
 * ==================================================================== */
static double dot(const double *a, const double *b, int64_t d) {
  double s = 0.0;
  for (int64_t i = 0; i < d; ++i) s += a[i] * b[i];
  return s;
}

/* Partial refresh, eq. (O update): u <- (c1 u + c2 Z)/|c1 u + c2 Z|,
 * c1 = e^{-h/L}, c2 = sqrt(1 - c1^2), Z = xi / sqrt(d) (R2). */
void orc_map_O(double *u, const double *xi, int64_t d, double h, double L) {
  const double c1 = exp(-h / L);
  const double c2 = sqrt(-expm1(-2.0 * h / L));
  const double sd = sqrt((double)d);
  double nn = 0.0;
  for (int64_t i = 0; i < d; ++i) {
    u[i] = c1 * u[i] + c2 * xi[i] / sd;
    nn += u[i] * u[i];
  }
  const double inv = 1.0 / sqrt(nn);
  for (int64_t i = 0; i < d; ++i) u[i] *= inv;
}

/* Velocity update, closed form of the Riccati flow (eq. B MCHMC) and its
 * energy change (d-1) log(cosh delta + (e.u) sinh delta).  cosh - 1 is taken
 * as 2 sinh^2(delta/2) and the log as log1p, which are identities. */
double orc_map_B(double *u, const double *gt, int64_t d, double h) {
  double n = sqrt(dot(gt, gt, d));
  if (n == 0.0) return 0.0;  /* R15 */
  const double delta = h * n / (double)(d - 1);
  double c = 0.0;
  for (int64_t i = 0; i < d; ++i) c += (gt[i] / n) * u[i];
  if (fabs(delta) >= 20.0) {
    /* the same quotient divided through by cosh(delta): sech u + (tanh + c(1 - sech)) e
     * over 1 + c tanh, and log cosh = |delta| + log(1 + e^{-2|delta|}) - ln 2; cosh and
     * sinh themselves overflow beyond |delta| ~ 710 */
    const double ad = fabs(delta), e2 = exp(-2.0 * ad);
    const double tau = copysign((1.0 - e2) / (1.0 + e2), delta);
    const double sech = 2.0 * exp(-ad) / (1.0 + e2);
    const double Dh = 1.0 + c * tau;
    for (int64_t i = 0; i < d; ++i) u[i] = (sech * u[i] + (tau + c * (1.0 - sech)) * (gt[i] / n)) / Dh;
    return (double)(d - 1) * (ad + log1p(e2) - M_LN2 + log(Dh));
  }
  const double sh = sinh(delta);
  const double shh = sinh(0.5 * delta);
  const double chm1 = 2.0 * shh * shh;
  const double Dm1 = chm1 + c * sh;
  const double D = 1.0 + Dm1;
  const double coef = sh + c * chm1;
  for (int64_t i = 0; i < d; ++i) u[i] = (u[i] + coef * (gt[i] / n)) / D;
  return (double)(d - 1) * log1p(Dm1);
}

/* Underdamped Langevin variant (appendix "Ablation studies", dynamics
 * paragraph: the microcanonical velocity replaced by the usual Gaussian one).
 * Reading: the velocity has covariance I/d, i.e. mass d and kinetic energy
 * K(u) = (d/2)|u|^2, so that |u| ~ 1 as on the sphere and eps, L and the
 * controllers keep their meaning.
 * O: the exact Ornstein-Uhlenbeck step u <- c1 u + c2 Z, Z = xi/sqrt(d) ~ N(0, I/d),
 *    with the same c1 = e^{-h/L}, c2 = sqrt(1 - c1^2); nothing is normalised.
 * B: Hamilton's equation du/dt = g/d, exact for fixed g: u <- u + (h/d) g, and the
 *    change K(u') - K(u) = h g.u + h^2 |g|^2 / (2d), written out so that it does
 *    not cancel. */
void orc_map_O_lang(double *u, const double *xi, int64_t d, double h, double L) {
  const double c1 = exp(-h / L);
  const double c2 = sqrt(-expm1(-2.0 * h / L));
  const double sd = sqrt((double)d);
  for (int64_t i = 0; i < d; ++i) u[i] = c1 * u[i] + c2 * xi[i] / sd;
}

double orc_map_B_lang(double *u, const double *gt, int64_t d, double h) {
  const double gu = dot(gt, u, d), gg = dot(gt, gt, d);
  for (int64_t i = 0; i < d; ++i) u[i] += h / (double)d * gt[i];
  return h * gu + 0.5 * h * h * gg / (double)d;
}

/* Position update x <- x + h u; with a diagonal preconditioner sigma the
 * position moves by h sigma*u (R9). */
void orc_map_A(double *x, const double *u, const double *sigma, int64_t d, double h) {
  for (int64_t i = 0; i < d; ++i) x[i] += h * (sigma ? sigma[i] * u[i] : u[i]);
}

/* Integrator table (Table "integrators"): symmetric B A B ... B with the
 * coefficients not printed derived from symmetry and normalisation. */
int orc_integrator_coeffs(int which, double *b, double *a, int *K) {
  if (which == 0) {
    b[0] = 0.5; b[1] = 0.5; a[0] = 1.0; *K = 2;
  } else if (which == 1) {
    const double b1 = 0.1931833275;
    b[0] = b1; b[1] = 1.0 - 2.0 * b1; b[2] = b1;
    a[0] = 0.5; a[1] = 0.5; *K = 3;
  } else if (which == 2) {
    const double b1 = 0.0839831526, b2 = 0.6822365335;
    const double a1 = 0.2539785108, a2 = -0.032302867;
    const double b3 = 0.5 - b1 - b2, a3 = 1.0 - 2.0 * (a1 + a2);
    b[0] = b1; b[1] = b2; b[2] = b3; b[3] = b3; b[4] = b2; b[5] = b1;
    a[0] = a1; a[1] = a2; a[2] = a3; a[3] = a2; a[4] = a1; *K = 6;
  } else {
    return -1;
  }
  return 0;
}

/* ======================================================================
 * Ensemble sampler: Algorithm "LAPS Pseudocode" with the maps above.
 * ==================================================================== */
enum { PH_UNADJ = 0, PH_SWITCH_PENDING = 1, PH_ADJ = 2 };
enum { ST_NONFINITE = 1, ST_EPS_KEPT = 2, ST_SIGMA_FIX = 4 };

struct orc_ctx {
  orc_config cfg;
  orc_target tg;
  int64_t N, d;
  double *x, *u, *g, *logp, *delta, *acc;
  double *mean, *var, *m2, *Vii, *sigma, *ring, *wdelta;
  double *x0, *g0, *tmp, *z;
  int64_t t, grads, Tw, ring_count, ring_pos, n_nonfinite;
  int32_t phase, adapt, switch_ready, status, integ, have_lo, have_hi;
  double eps, L, eevpd, eevpd_target, dtilde, max_delta, acc_mean, lo, hi, a_star, sum_var;
};

static double *alloc0(int64_t n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

orc_ctx *orc_create(const orc_config *cfg, const orc_target *tg) {
  if (cfg->d < 2 || cfg->n_chains < 2 || tg->d != cfg->d) return NULL;
  if (!(cfg->eps_fixed >= 0.0) || !isfinite(cfg->eps_fixed)) return NULL;
  if (cfg->dynamics != 0 && cfg->dynamics != 1) return NULL;
  orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
  c->cfg = *cfg;
  c->tg = *tg;
  c->N = cfg->n_chains;
  c->d = cfg->d;
  const int64_t N = c->N, d = c->d;
  c->x = alloc0(N * d); c->u = alloc0(N * d); c->g = alloc0(N * d);
  c->logp = alloc0(N); c->delta = alloc0(N); c->acc = alloc0(N);
  c->mean = alloc0(d); c->var = alloc0(d); c->m2 = alloc0(d); c->Vii = alloc0(d);
  c->sigma = alloc0(d); c->wdelta = alloc0(d);
  /* R4-R6: window length = 20% of the total number of steps */
  c->Tw = (int64_t)llround(cfg->window_frac * (double)cfg->max_steps_total);
  if (c->Tw < 2) c->Tw = 2;
  c->ring = alloc0(c->Tw * d);
  c->x0 = alloc0(d); c->g0 = alloc0(d); c->tmp = alloc0(d); c->z = alloc0(d + 8);
  return c;
}

void orc_destroy(orc_ctx *c) {
  if (!c) return;
  double *ps[] = {c->x, c->u, c->g, c->logp, c->delta, c->acc, c->mean, c->var, c->m2,
                  c->Vii, c->sigma, c->wdelta, c->ring, c->x0, c->g0, c->tmp, c->z};
  for (size_t i = 0; i < sizeof(ps) / sizeof(ps[0]); ++i) free(ps[i]);
  free(c);
}

double orc_F(double D) {
  /* eq. (bias bound): F(D) = 4 D^{3/2} / (1 + D^{1/2})^2 */
  const double r = sqrt(D);
  return 4.0 * D * r / ((1.0 + r) * (1.0 + r));
}

/* Full-rank equipartition loss (section "Equipartition condition", full-rank
 * paragraph; Hutchinson 1989): V_ij = -E[(x_i - E x_i) g_j] (eq. for the
 * equipartition matrix, ensemble averages of eq. ECA) gives
 * (I - V) z = z + (1/N) sum_m (x_m - xbar)(g_m . z), and the loss (1/d)
 * Tr((I - V)(I - V)^T) is estimated as the mean of |(I - V) z|^2 / d over the
 * probes.  Plain loops; ensemble sums compensated, in chain order. */
double orc_dtilde_full(const double *x, const double *g, int64_t N, int64_t d, const double *z, int64_t P) {
  double *xbar = (double *)calloc((size_t)d, sizeof(double));
  double *s = (double *)calloc((size_t)N, sizeof(double));
  for (int64_t i = 0; i < d; ++i) {
    nsum a = {0, 0};
    for (int64_t m = 0; m < N; ++m) nsum_add(&a, x[m * d + i]);
    xbar[i] = nsum_get(&a) / (double)N;
  }
  nsum tot = {0, 0};
  for (int64_t p = 0; p < P; ++p) {
    const double *zp = z + p * d;
    for (int64_t m = 0; m < N; ++m) {  /* s_m = g_m . z_p */
      nsum a = {0, 0};
      for (int64_t i = 0; i < d; ++i) nsum_add(&a, g[m * d + i] * zp[i]);
      s[m] = nsum_get(&a);
    }
    for (int64_t i = 0; i < d; ++i) {
      nsum a = {0, 0};
      for (int64_t m = 0; m < N; ++m) nsum_add(&a, (x[m * d + i] - xbar[i]) * s[m]);
      const double w = zp[i] + nsum_get(&a) / (double)N;
      nsum_add(&tot, w * w);
    }
  }
  free(xbar);
  free(s);
  return nsum_get(&tot) / ((double)P * (double)d);
}

/* Per-dim ensemble moments of the current x and g (eq. ECA, 1/M averages,
 * R8): mean, two-pass variance, second moment and the equipartition
 * diagonal V_ii = -E[(x_i - E x_i) d_i log p]. */
static void ensemble_moments(orc_ctx *c) {
  const int64_t N = c->N, d = c->d;
  double sv = 0.0;
  for (int64_t i = 0; i < d; ++i) {
    nsum s = {0, 0}, s2 = {0, 0}, sq = {0, 0}, sv_ = {0, 0};
    for (int64_t m = 0; m < N; ++m) nsum_add(&s, c->x[m * d + i]);
    const double mu = nsum_get(&s) / (double)N;
    for (int64_t m = 0; m < N; ++m) {
      const double xv = c->x[m * d + i];
      const double dx = xv - mu;
      nsum_add(&s2, dx * dx);
      nsum_add(&sq, xv * xv);
      nsum_add(&sv_, -dx * c->g[m * d + i]);
    }
    c->mean[i] = mu;
    c->var[i] = nsum_get(&s2) / (double)N;
    c->m2[i] = nsum_get(&sq) / (double)N;
    c->Vii[i] = nsum_get(&sv_) / (double)N;
    sv += c->var[i];
  }
  c->sum_var = sv;
}

int orc_init(orc_ctx *c, const double *x0, const double *u0) {
  const int64_t N = c->N, d = c->d;
  memcpy(c->x, x0, sizeof(double) * N * d);
  for (int64_t m = 0; m < N; ++m) {
    double *x = c->x + m * d, *g = c->g + m * d, *u = c->u + m * d;
    c->logp[m] = orc_logp_grad(&c->tg, x, g);
    if (u0) {
      memcpy(u, u0 + m * d, sizeof(double) * d);
    } else {
      /* initialization section: velocity aligned with the gradient, unit norm */
      double n = sqrt(dot(g, g, d));
      if (n > 0.0 && isfinite(n)) {
        for (int64_t i = 0; i < d; ++i) u[i] = g[i] / n;
      } else {  /* R19: no gradient direction -> a uniform direction */
        orc_normals(c->cfg.seed, (uint64_t)m, 0, ORC_TAG_INIT_DIR, 0, d, c->z);
        double zn = sqrt(dot(c->z, c->z, d));
        for (int64_t i = 0; i < d; ++i) u[i] = c->z[i] / zn;
      }
    }
    c->delta[m] = 0.0;
    c->acc[m] = 0.0;
  }
  ensemble_moments(c);
  /* Algorithm: eps <- 0.01 sqrt(d), L <- eq. (L) on the initial ensemble */
  c->eps = c->cfg.eps_fixed > 0.0 ? c->cfg.eps_fixed : c->cfg.eps0_factor * sqrt((double)d);
  c->L = c->cfg.alpha * sqrt(c->sum_var);
  c->t = 0;
  c->grads = 1;
  c->phase = PH_UNADJ;
  c->adapt = 1;
  c->switch_ready = 0;
  c->status = 0;
  c->ring_count = 0;
  c->ring_pos = 0;
  c->n_nonfinite = 0;
  c->integ = 0;
  c->have_lo = c->have_hi = 0;
  c->lo = c->hi = 0.0;
  c->eevpd = c->eevpd_target = c->dtilde = c->max_delta = c->acc_mean = 0.0;
  for (int64_t i = 0; i < d; ++i) c->sigma[i] = 1.0;
  return 0;
}

/* Deterministic part Phi_eps = B_{b1 eps} A_{a1 eps} ... B_{bK eps} on one
 * chain (eq. integrator); returns the energy change of its A and B maps. */
static double integrate(orc_ctx *c, double *x, double *u, double *g, double *lp,
                        int which, double eps, const double *sigma) {
  const int64_t d = c->d;
  double b[8], a[8];
  int K;
  orc_integrator_coeffs(which, b, a, &K);
  double dE = 0.0;
  for (int k = 0; k < K; ++k) {
    /* B with the gradient in the sampler's coordinates (sigma*g when preconditioned) */
    for (int64_t i = 0; i < d; ++i) c->tmp[i] = sigma ? sigma[i] * g[i] : g[i];
    dE += c->cfg.dynamics ? orc_map_B_lang(u, c->tmp, d, b[k] * eps) : orc_map_B(u, c->tmp, d, b[k] * eps);
    if (k == K - 1) break;
    orc_map_A(x, u, sigma, d, a[k] * eps);
    const double lnew = orc_logp_grad(&c->tg, x, g);
    dE += *lp - lnew;  /* eq. position update: -log p(x') + log p(x) */
    *lp = lnew;
  }
  return dE;
}

/* The partial refresh of the configured dynamics with the normals in c->z. */
static void refresh(orc_ctx *c, double *u, double h, double L) {
  if (c->cfg.dynamics) orc_map_O_lang(u, c->z, c->d, h, L);
  else orc_map_O(u, c->z, c->d, h, L);
}

/* One unadjusted MCLMC step (eq. discrete update): O_{eps/2} Phi_eps O_{eps/2}
 * with the leapfrog coefficients, for every chain. */
void orc_unadj_move(orc_ctx *c) {
  if (c->phase != PH_UNADJ) return;
  const int64_t N = c->N, d = c->d;
  const double h = 0.5 * c->eps;
  for (int64_t m = 0; m < N; ++m) {
    double *x = c->x + m * d, *u = c->u + m * d, *g = c->g + m * d;
    orc_normals(c->cfg.seed, (uint64_t)m, (uint64_t)c->t, ORC_TAG_O_FIRST, 0, d, c->z);
    refresh(c, u, h, c->L);
    const double dE = integrate(c, x, u, g, &c->logp[m], 0, c->eps, NULL);
    orc_normals(c->cfg.seed, (uint64_t)m, (uint64_t)c->t, ORC_TAG_O_SECOND, 0, d, c->z);
    refresh(c, u, h, c->L);
    c->delta[m] = dE;
  }
}

/* Ensemble statistics and the unadjusted controller (Algorithm, first loop):
 * EEVPD, D~_diag, eps update through F(C D~), L from the variances, and the
 * moving-window fluctuation of E[x_i^2] that triggers the switch. */
void orc_unadj_control(orc_ctx *c) {
  if (c->phase != PH_UNADJ) return;
  const int64_t N = c->N, d = c->d;
  ensemble_moments(c);
  /* equipartition loss, diagonal form, or full rank from fresh probes of this step */
  if (c->cfg.full_rank_probes > 0) {
    const int64_t P = c->cfg.full_rank_probes;
    double *z = (double *)calloc((size_t)(P * d), sizeof(double));
    for (int64_t p = 0; p < P; ++p) orc_rademacher(c->cfg.seed, (uint64_t)c->t, p, d, z + p * d);
    c->dtilde = orc_dtilde_full(c->x, c->g, N, d, z, P);
    free(z);
  } else {
    nsum s = {0, 0};
    for (int64_t i = 0; i < d; ++i) nsum_add(&s, (1.0 - c->Vii[i]) * (1.0 - c->Vii[i]));
    c->dtilde = nsum_get(&s) / (double)d;
  }
  /* EEVPD: variance (R1, mode 0) or mean square (mode 1) of Delta, over d */
  {
    int64_t bad = 0;
    nsum s = {0, 0}, s2 = {0, 0};
    for (int64_t m = 0; m < N; ++m) {
      if (!isfinite(c->delta[m])) ++bad;
      nsum_add(&s, c->delta[m]);
    }
    const double mu = nsum_get(&s) / (double)N;
    for (int64_t m = 0; m < N; ++m) {
      const double v = (c->cfg.eevpd_mode == 1) ? c->delta[m] : c->delta[m] - mu;
      nsum_add(&s2, v * v);
    }
    c->eevpd = nsum_get(&s2) / (double)N / (double)d;
    c->n_nonfinite = bad;
    if (bad) c->status |= ST_NONFINITE;
  }
  c->eevpd_target = orc_F(c->cfg.C * c->dtilde);
  if (!(c->cfg.eps_fixed > 0.0)) {
    const double ratio = c->eevpd_target / c->eevpd;
    if (isfinite(ratio) && ratio > 0.0) c->eps *= pow(ratio, 1.0 / 6.0);
    else c->status |= ST_EPS_KEPT;  /* R20 */
  }
  c->L = c->cfg.alpha * sqrt(c->sum_var);
  /* window of E[x_i^2] (R4, R5) */
  memcpy(c->ring + c->ring_pos * d, c->m2, sizeof(double) * d);
  c->ring_pos = (c->ring_pos + 1) % c->Tw;
  if (c->ring_count < c->Tw) c->ring_count++;
  c->max_delta = INFINITY;
  c->switch_ready = 0;
  if (c->ring_count == c->Tw) {
    double mx = 0.0;
    for (int64_t i = 0; i < d; ++i) {
      nsum s = {0, 0}, s2 = {0, 0};
      for (int64_t k = 0; k < c->Tw; ++k) nsum_add(&s, c->ring[k * d + i]);
      const double mu = nsum_get(&s) / (double)c->Tw;
      for (int64_t k = 0; k < c->Tw; ++k) {
        const double v = c->ring[k * d + i] - mu;
        nsum_add(&s2, v * v);
      }
      const double sd = sqrt(nsum_get(&s2) / (double)(c->Tw - 1));
      c->wdelta[i] = sd / mu;
      if (!(c->wdelta[i] <= mx)) mx = c->wdelta[i];  /* NaN propagates as "not settled" */
    }
    c->max_delta = mx;
    c->switch_ready = (mx < c->cfg.switch_tol) ? 1 : 0;  /* R3 */
  }
  c->t += 1;
  c->grads += 1;
  /* R22: the paper's rule, or a fixed switch at max_steps_unadj */
  if ((c->cfg.switch_policy == 0 && c->switch_ready) || c->t >= c->cfg.max_steps_unadj)
    c->phase = PH_SWITCH_PENDING;
}

int orc_step_unadjusted(orc_ctx *c, int64_t n) {
  if (c->phase == PH_ADJ) return -4;
  for (int64_t k = 0; k < n && c->phase == PH_UNADJ; ++k) {
    orc_unadj_move(c);
    orc_unadj_control(c);
  }
  return 0;
}

/* Switch to the adjusted phase: diagonal preconditioner from the ensemble
 * variances (R9), integrator MN2 for d <= 200 else MN4, acceptance target
 * 0.7 / 0.9, eps carried over (R10), ADAPT on. */
void orc_do_switch(orc_ctx *c) {
  const int64_t d = c->d;
  for (int64_t i = 0; i < d; ++i) {
    double s = sqrt(c->var[i]);
    if (!(s > 0.0) || !isfinite(s)) { s = 1.0; c->status |= ST_SIGMA_FIX; }
    c->sigma[i] = s;
  }
  int integ = c->cfg.integrator_adj;
  if (integ == 0) integ = (d <= 200) ? 1 : 2;
  c->integ = integ;
  c->a_star = (c->cfg.acc_target > 0.0) ? c->cfg.acc_target : (integ == 2 ? 0.9 : 0.7);
  c->adapt = 1;
  c->have_lo = c->have_hi = 0;
  c->phase = PH_ADJ;
}

static int grads_per_step(int integ) { return integ == 2 ? 5 : (integ == 1 ? 2 : 1); }

/* One MAMS transition for every chain (appendix "Metropolis adjusted
 * microcanonical dynamics"): full refresh, n_steps_traj integrator steps each
 * wrapped in partial refreshes with L = 1.25 * n_steps_traj * eps (R17),
 * accept with probability min(1, e^{-Delta}) (R12, R13), restore on reject
 * (R14). */
void orc_mams_move(orc_ctx *c) {
  if (c->phase != PH_ADJ || c->t >= c->cfg.max_steps_total) return;
  const int64_t N = c->N, d = c->d;
  const int ns = c->cfg.n_steps_traj;
  const double eps = c->eps, h = 0.5 * eps;
  const double Lp = c->cfg.L_partial_factor * (double)ns * eps;
  int64_t bad = 0;
  for (int64_t m = 0; m < N; ++m) {
    double *x = c->x + m * d, *u = c->u + m * d, *g = c->g + m * d;
    memcpy(c->x0, x, sizeof(double) * d);
    memcpy(c->g0, g, sizeof(double) * d);
    const double l0 = c->logp[m];
    orc_normals(c->cfg.seed, (uint64_t)m, (uint64_t)c->t, ORC_TAG_FULL_REFRESH, 0, d, c->z);
    /* full refresh: uniform on the sphere, or N(0, I/d) for the Langevin variant */
    const double zn = c->cfg.dynamics ? sqrt((double)d) : sqrt(dot(c->z, c->z, d));
    for (int64_t i = 0; i < d; ++i) u[i] = c->z[i] / zn;
    double D = 0.0;
    for (int j = 0; j < ns; ++j) {
      orc_normals(c->cfg.seed, (uint64_t)m, (uint64_t)c->t, ORC_TAG_O_FIRST, (uint32_t)j, d, c->z);
      refresh(c, u, h, Lp);
      D += integrate(c, x, u, g, &c->logp[m], c->integ, eps, c->sigma);
      orc_normals(c->cfg.seed, (uint64_t)m, (uint64_t)c->t, ORC_TAG_O_SECOND, (uint32_t)j, d, c->z);
      refresh(c, u, h, Lp);
    }
    c->delta[m] = D;
    const double w = exp(-D);
    double a;
    if (isnan(D)) a = 0.0;
    else a = (w < 1.0) ? w : 1.0;
    c->acc[m] = a;
    if (!isfinite(D)) ++bad;
    const double U = orc_mh_uniform(c->cfg.seed, (uint64_t)m, (uint64_t)c->t);
    const int accept = (!isnan(D)) && (U < w);
    if (!accept) {
      memcpy(x, c->x0, sizeof(double) * d);
      memcpy(g, c->g0, sizeof(double) * d);
      c->logp[m] = l0;
    }
  }
  c->n_nonfinite = bad;
  if (bad) c->status |= ST_NONFINITE;
}

/* Adjusted-phase controller (Algorithm, second loop; R11): mean acceptance,
 * sticky ADAPT with tolerance acc_tol, double/halve to a bracket and then
 * bisect. */
void orc_adj_control(orc_ctx *c) {
  if (c->phase != PH_ADJ || c->t >= c->cfg.max_steps_total) return;
  c->acc_mean = orc_sum(c->acc, c->N) / (double)c->N;
  c->adapt = c->adapt && (fabs(c->acc_mean - c->a_star) > c->cfg.acc_tol);
  if (c->adapt) {
    if (c->acc_mean > c->a_star) {  /* step too small */
      c->lo = c->eps; c->have_lo = 1;
      c->eps = c->have_hi ? 0.5 * (c->lo + c->hi) : 2.0 * c->eps;
    } else {
      c->hi = c->eps; c->have_hi = 1;
      c->eps = c->have_lo ? 0.5 * (c->lo + c->hi) : 0.5 * c->eps;
    }
  }
  c->t += c->cfg.n_steps_traj;  /* R7 */
  c->grads += (int64_t)c->cfg.n_steps_traj * grads_per_step(c->integ);
}

int orc_step_adjusted(orc_ctx *c, int64_t n) {
  if (c->phase != PH_ADJ) orc_do_switch(c);
  for (int64_t k = 0; k < n; ++k) {
    orc_mams_move(c);
    orc_adj_control(c);
  }
  return 0;
}

int orc_run(orc_ctx *c) {
  orc_step_unadjusted(c, c->cfg.max_steps_unadj);
  orc_do_switch(c);
  while (c->t < c->cfg.max_steps_total) {
    orc_mams_move(c);
    orc_adj_control(c);
  }
  return 0;
}

void orc_get_stats(const orc_ctx *c, orc_stats *s) {
  s->t = c->t;
  s->grads_per_chain = c->grads;
  s->phase = c->phase;
  s->adapt = c->adapt;
  s->switch_ready = c->switch_ready;
  s->status_bits = c->status;
  s->eps = c->eps;
  s->L = c->L;
  s->eevpd = c->eevpd;
  s->eevpd_target = c->eevpd_target;
  s->dtilde = c->dtilde;
  s->max_delta = c->max_delta;
  s->acc_mean = c->acc_mean;
  s->n_nonfinite = c->n_nonfinite;
  s->integrator = c->integ;
  s->have_lo = c->have_lo;
  s->have_hi = c->have_hi;
  s->ring_full = (c->ring_count == c->Tw);
  s->lo = c->lo;
  s->hi = c->hi;
  s->a_star = c->a_star;
  s->sum_var = c->sum_var;
}

double *orc_ptr(orc_ctx *c, int which) {
  switch (which) {
    case 0: return c->x;
    case 1: return c->u;
    case 2: return c->g;
    case 3: return c->logp;
    case 4: return c->delta;
    case 5: return c->acc;
    case 6: return c->mean;
    case 7: return c->var;
    case 8: return c->m2;
    case 9: return c->Vii;
    case 10: return c->sigma;
    case 11: return c->ring;
    case 12: return c->wdelta;
    default: return NULL;
  }
}

void orc_set_hyper(orc_ctx *c, double eps, double L) {
  c->eps = eps;
  c->L = L;
}
