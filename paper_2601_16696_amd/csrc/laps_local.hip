// Per-chain kernels of the LAPS hot path for targets whose gradient is local
// to one chain: the diagonal Gaussian, stochastic volatility (tridiagonal
// AR(1) prior) and the 2-D phi^4 lattice.
//
// Layout: chain-major [N][ld] rows.  A team of T lanes holds one chain in
// registers; lane r owns octs r + q T (eight consecutive coordinates each, the
// unit of one Philox block), so every load is a contiguous 32- or 64-byte
// vector per lane and the team's accesses are coalesced.  Per-chain dot
// products are team reductions; per-dimension ensemble sums are accumulated in
// registers across all chains a workgroup visits and written once per
// workgroup as FP64 partial rows.
#include "laps_team.hpp"

namespace laps {

// ---------------------------------------------------------------------------
// Targets.  eval() returns this lane's share of log p (the caller reduces it
// with its own dot products) and fills g; coordinates >= d get g = 0.
// ---------------------------------------------------------------------------
// Diagonal Gaussian: log p = -1/2 sum x_i^2 / s2_i, g = -x / s2.
template <class Real, int Q>
struct GaussTgt {
  static constexpr bool kStage = false;
  Real inv[Q][8];
  __device__ void setup(const LocalArgs &a, int r, int T) {
    if (a.aux) {
      load_row<Real, Q>(static_cast<const Real *>(a.aux), r, T, a.d, true, inv);
      return;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t e = 8 * (int64_t)(r + q * T) + i;
        inv[q][i] = e < a.d ? (Real)(1.0 / a.tdata[e]) : Real(0);
      }
  }
  __device__ double eval(const LocalArgs &, const Real (&x)[Q][8], Real (&g)[Q][8], Real *, double *, int &, int,
                         int) {
    double lp = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        g[q][i] = -x[q][i] * inv[q][i];
        lp -= 0.5 * (double)x[q][i] * (double)x[q][i] * (double)inv[q][i];
      }
    return lp;
  }
};

// 2-D periodic phi^4 (L x L): g = sum of the four neighbours - (4 + m2) f
// - 4 lambda f^3; log p = -sum [1/2 (f_right - f)^2 + 1/2 (f_down - f)^2
// + m2/2 f^2 + lambda f^4].  Neighbours come from the chain staged in LDS.
template <class Real, int Q>
struct Phi4Tgt {
  static constexpr bool kStage = true;
  __device__ void setup(const LocalArgs &, int, int) {}
  __device__ double eval(const LocalArgs &a, const Real (&x)[Q][8], Real (&g)[Q][8], Real *stage, double *, int &,
                         int r, int T) {
    const int L = (int)a.tn;
    const int d = (int)a.d;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
      if (e0 < d)
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (e0 + i < d) stage[e0 + i] = x[q][i];
    }
    __syncthreads();
    const Real m2 = (Real)a.tp0, lam = (Real)a.tp1;
    const Real diag = Real(4) + m2;
    double lp = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + i;
        if (e < d) {
          const int row = e / L, col = e - row * L;
          const int cr = (col + 1 == L) ? 0 : col + 1, cl = (col == 0) ? L - 1 : col - 1;
          const int rd = (row + 1 == L) ? 0 : row + 1, ru = (row == 0) ? L - 1 : row - 1;
          const Real f = x[q][i];
          const Real fr = stage[row * L + cr], fl = stage[row * L + cl];
          const Real fd = stage[rd * L + col], fu = stage[ru * L + col];
          g[q][i] = (fr + fl + fd + fu) - diag * f - Real(4) * lam * f * f * f;
          const double df = (double)f, dr = (double)fr - df, dd = (double)fd - df;
          lp -= 0.5 * dr * dr + 0.5 * dd * dd + 0.5 * a.tp0 * df * df + a.tp1 * df * df * df * df;
        } else {
          g[q][i] = Real(0);
        }
      }
    }
    __syncthreads();
    return lp;
  }
};

// Stochastic volatility, theta = (h_1..h_T, s, r): sigma = e^s, phi = tanh r,
// E = (1 - phi^2) h_1^2 + sum_{t>=2} (h_t - phi h_{t-1})^2,
// log p = -2 (s+2)^2 - 2 (r-2)^2 - T s + 1/2 log(1 - phi^2) - E/(2 sigma^2)
//         - 1/2 sum h_t - 1/2 sum y_t^2 e^{-h_t}.
// The (s, r) gradients need sums over t, so eval() reduces (E, cross, lik)
// over the team before the two owner lanes finish them.
template <class Real, int Q>
struct SVTgt {
  static constexpr bool kStage = true;
  Real y2[Q][8];
  __device__ void setup(const LocalArgs &a, int r, int T) {
    if (a.aux) {
      load_row<Real, Q>(static_cast<const Real *>(a.aux), r, T, a.d, true, y2);
      return;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t e = 8 * (int64_t)(r + q * T) + i;
        y2[q][i] = e < a.tn ? (Real)(a.tdata[e] * a.tdata[e]) : Real(0);
      }
  }
  __device__ double eval(const LocalArgs &a, const Real (&x)[Q][8], Real (&g)[Q][8], Real *stage, double *red,
                         int &slot, int r, int T) {
    const int Tn = (int)a.tn;
    const int d = (int)a.d;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
      if (e0 < d)
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (e0 + i < d) stage[e0 + i] = x[q][i];
    }
    __syncthreads();
    const double s = (double)stage[Tn], rr = (double)stage[Tn + 1];
    const double sig2 = exp(2.0 * s), phi = tanh(rr), omp = 1.0 - phi * phi;
    const Real phR = (Real)phi, ompR = (Real)omp, isR = (Real)(1.0 / sig2);
    double v[3] = {0.0, 0.0, 0.0};  // E, cross, lik
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + i;
        if (e < Tn) {
          const Real h = x[q][i];
          const Real hp = (e > 0) ? stage[e - 1] : Real(0);
          const Real an = (e + 1 < Tn) ? (stage[e + 1] - phR * h) : Real(0);
          const Real own = (e == 0) ? ompR * h : (h - phR * hp);
          const Real eh = exp(-h);
          g[q][i] = -(own - phR * an) * isR - Real(0.5) + Real(0.5) * y2[q][i] * eh;
          if (e == 0) {
            v[0] += omp * (double)h * (double)h;
            v[1] += phi * (double)h * (double)h;
          } else {
            const double at = (double)h - phi * (double)hp;
            v[0] += at * at;
            v[1] += at * (double)hp;
          }
          v[2] += -0.5 * (double)h - 0.5 * (double)y2[q][i] * (double)eh;
        } else {
          g[q][i] = Real(0);
        }
      }
    }
    __syncthreads();
    team_sum<3>(v, T, red, slot);
    const double E = v[0], cross = v[1], lik = v[2];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + i;
        if (e == Tn) g[q][i] = (Real)(-4.0 * (s + 2.0) - (double)Tn + E / sig2);
        if (e == Tn + 1) g[q][i] = (Real)(-4.0 * (rr - 2.0) - phi + omp * cross / sig2);
      }
    }
    const double lp = -2.0 * (s + 2.0) * (s + 2.0) - 2.0 * (rr - 2.0) * (rr - 2.0) - (double)Tn * s +
                      0.5 * log(omp) - E / (2.0 * sig2) + lik;
    return (r == 0) ? lp : 0.0;
  }
};

// Integrator coefficients by integrator id (0 LF, 1 MN2, 2 MN4), in constant
// memory so that a rolled loop over the composition reads them by index.
__constant__ double kCoefB[3][6] = {
    {0.5, 0.5, 0.0, 0.0, 0.0, 0.0},
    {0.1931833275, 1.0 - 2.0 * 0.1931833275, 0.1931833275, 0.0, 0.0, 0.0},
    {0.0839831526, 0.6822365335, 0.5 - 0.0839831526 - 0.6822365335, 0.5 - 0.0839831526 - 0.6822365335, 0.6822365335,
     0.0839831526}};
__constant__ double kCoefA[3][5] = {
    {1.0, 0.0, 0.0, 0.0, 0.0},
    {0.5, 0.5, 0.0, 0.0, 0.0},
    {0.2539785108, -0.032302867, 1.0 - 2.0 * (0.2539785108 - 0.032302867), -0.032302867, 0.2539785108}};

// ---------------------------------------------------------------------------
// shared kernel prologue
// ---------------------------------------------------------------------------
#define LAPS_TEAM_PROLOGUE                                                                  \
  extern __shared__ double smem[];                                                          \
  double *red = smem;                                                                       \
  const int T = a.T;                                                                        \
  const int team = threadIdx.x / T, r = threadIdx.x - team * T;                             \
  Real *stage = reinterpret_cast<Real *>(smem + 2 * kRedSlots) + (Tgt::kStage ? (size_t)team * a.ld : 0); \
  int slot = 0;                                                                             \
  const int64_t N = a.N, d = a.d, ld = a.ld;                                                \
  const double dm1 = (double)(d - 1);

// ---------------------------------------------------------------------------
// Initialisation: log p and gradient at x, u = g/|g| (u0 if given; a uniform
// random direction when the gradient vanishes), per-dim sums for the initial
// variances (shift K = 0).
// ---------------------------------------------------------------------------
template <class Real, int Q, class Tgt, bool STATS>
__global__ void __launch_bounds__(512) k_init(LocalArgs a) {
  LAPS_TEAM_PROLOGUE
  Tgt tgt;
  tgt.setup(a, r, T);
  double S[4][Q][8] = {};
  double K0[Q][8] = {};
  const Real *X = static_cast<const Real *>(a.x);
  for (int64_t base = (int64_t)blockIdx.x * a.tpw; base < N; base += (int64_t)gridDim.x * a.tpw) {
    const int64_t m = base + team;
    const bool act = m < N;
    Real x[Q][8], g[Q][8], u[Q][8], z[Q][8];
    load_row<Real, Q>(X + m * ld, r, T, d, act, x);
    const double lp = tgt.eval(a, x, g, stage, red, slot, r, T);
    lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, 0, TAG_INIT_DIR, 0, z);
    double v[3] = {lp, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        v[1] += (double)g[q][i] * (double)g[q][i];
        v[2] += (double)z[q][i] * (double)z[q][i];
      }
    team_sum<3>(v, T, red, slot);
    if (a.u0) {
      load_row<Real, Q>(static_cast<const Real *>(a.u0) + m * ld, r, T, d, act, u);
    } else {
      const double gn = sqrt(v[1]);
      const bool useg = gn > 0.0 && isfinite(gn);
      const Real sc = (Real)(1.0 / (useg ? gn : sqrt(v[2])));
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) u[q][i] = (useg ? g[q][i] : z[q][i]) * sc;
    }
    if (act) {
      store_row<Real, Q>(static_cast<Real *>(a.x) + m * ld, r, T, d, x);
      store_row<Real, Q>(static_cast<Real *>(a.u) + m * ld, r, T, d, u);
      if (a.cache) store_row<Real, Q>(static_cast<Real *>(a.g) + m * ld, r, T, d, g);
      if (r == 0) {
        a.logp[m] = v[0];
        a.delta[m] = 0.0;
        a.acc[m] = 0.0;
      }
      if (STATS) accumulate_stats<Real, Q>(S, K0, x, g);
    }
  }
  if (STATS) write_partials<Real, Q>(a.partials, a.d, a.ld, S, red, T, r);
}

// ---------------------------------------------------------------------------
// One unadjusted step (eq. discrete update, leapfrog):
//   O_{eps/2}  B_{eps/2}  A_eps  [grad]  B_{eps/2}  O_{eps/2}
// Energy error Delta = (log p before - log p after) + the two B energies.
// The first O's normalisation and the first B's dot products share one team
// reduction (g.u = g.w / |w|).  Ensemble sums of the new state go to the
// workgroup's partial row.
// ---------------------------------------------------------------------------
template <class Real, int Q, class Tgt, bool STATS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(STATS ? 1 : 3))) k_unadj(LocalArgs a) {
  const DevHyper *H = a.hyp;
  if (H->phase != PH_UNADJ) return;
  LAPS_TEAM_PROLOGUE
  const double eps = H->eps, Lm = H->L;
  const uint64_t t = (uint64_t)H->t;
  const double h = 0.5 * eps;
  const double c1d = exp(-h / Lm), c2d = sqrt(-expm1(-2.0 * h / Lm)) / sqrt((double)d);
  const Real c1 = (Real)c1d, c2 = (Real)c2d, epsR = (Real)eps;
  Tgt tgt;
  tgt.setup(a, r, T);
  double S[4][Q][8] = {};
  double K[Q][8];
  if (STATS) load_shift<Q>(a.shiftK, r, T, d, K);
  Real *X = static_cast<Real *>(a.x);
  Real *U = static_cast<Real *>(a.u);
  for (int64_t base = (int64_t)blockIdx.x * a.tpw; base < N; base += (int64_t)gridDim.x * a.tpw) {
    const int64_t m = base + team;
    const bool act = m < N;
    Real x[Q][8], u[Q][8], g[Q][8], z[Q][8];
    load_row<Real, Q>(X + m * ld, r, T, d, act, x);
    load_row<Real, Q>(U + m * ld, r, T, d, act, u);
    const double lp0 = tgt.eval(a, x, g, stage, red, slot, r, T);
    // O (first half) fused with the dot products of the first B
    lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_O_FIRST, 0, z);
    double v4[4] = {lp0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const Real w = c1 * u[q][i] + c2 * z[q][i];
        u[q][i] = w;
        v4[1] += (double)w * (double)w;
        v4[2] += (double)g[q][i] * (double)w;
        v4[3] += (double)g[q][i] * (double)g[q][i];
      }
    team_sum<4>(v4, T, red, slot);
    const double inw = 1.0 / sqrt(v4[1]);
    const BMap b1 = b_map_t<Real>(v4[3], v4[2] * inw, h, dm1);
    const Real A1 = (Real)(b1.A * inw), B1 = (Real)b1.Bg;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        u[q][i] = A1 * u[q][i] + B1 * g[q][i];
        x[q][i] += epsR * u[q][i];
      }
    const double lp1 = tgt.eval(a, x, g, stage, red, slot, r, T);
    double v3[3] = {lp1, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        v3[1] += (double)g[q][i] * (double)g[q][i];
        v3[2] += (double)g[q][i] * (double)u[q][i];
      }
    team_sum<3>(v3, T, red, slot);
    const BMap b2 = b_map_t<Real>(v3[1], v3[2], h, dm1);
    const Real A2 = (Real)b2.A, B2 = (Real)b2.Bg;
    lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_O_SECOND, 0, z);
    double v1[1] = {0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const Real w = c1 * (A2 * u[q][i] + B2 * g[q][i]) + c2 * z[q][i];
        u[q][i] = w;
        v1[0] += (double)w * (double)w;
      }
    team_sum<1>(v1, T, red, slot);
    const Real in2 = (Real)(1.0 / sqrt(v1[0]));
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) u[q][i] *= in2;
    if (act) {
      store_row<Real, Q>(X + m * ld, r, T, d, x);
      store_row<Real, Q>(U + m * ld, r, T, d, u);
      if (a.cache) store_row<Real, Q>(static_cast<Real *>(a.g) + m * ld, r, T, d, g);
      if (r == 0) {
        a.delta[m] = (v4[0] - v3[0]) + b1.dK + b2.dK;
        a.logp[m] = v3[0];
      }
      if (STATS) accumulate_stats<Real, Q>(S, K, x, g);
    }
  }
  if (STATS) write_partials<Real, Q>(a.partials, a.d, a.ld, S, red, T, r);
}

// ---------------------------------------------------------------------------
// One MAMS transition per chain, fused (appendix "Metropolis adjusted
// microcanonical dynamics"): full refresh u = Z/|Z|, n_traj integrator steps
// O_{eps/2} Phi_eps O_{eps/2} with L_p = Lp_factor n_traj eps, in the
// preconditioned coordinates (x moves by h sigma*u, B uses sigma*g), then
// accept with probability min(1, e^{-Delta}).  The trajectory lives in
// registers: on rejection nothing is written, so x (and the cached g, log p)
// keep their starting values.
// ---------------------------------------------------------------------------
template <class Real, int Q, class Tgt, int INTEG>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3))) k_mams(LocalArgs a) {
  const DevHyper *H = a.hyp;
  if (H->phase != PH_ADJ || H->t >= a.max_total) return;
  LAPS_TEAM_PROLOGUE
  const double eps = H->eps;
  const uint64_t t = (uint64_t)H->t;
  const double h = 0.5 * eps;
  const double Lp = a.Lp_factor * (double)a.n_traj * eps;
  const double c1d = exp(-h / Lp), c2d = sqrt(-expm1(-2.0 * h / Lp)) / sqrt((double)d);
  const Real c1 = (Real)c1d, c2 = (Real)c2d;
  const Coeffs C = integrator_coeffs(INTEG);
  Tgt tgt;
  tgt.setup(a, r, T);
  Real sg[Q][8];
  load_row<Real, Q>(static_cast<const Real *>(a.sigma), r, T, d, true, sg);
  Real *X = static_cast<Real *>(a.x);
  for (int64_t base = (int64_t)blockIdx.x * a.tpw; base < N; base += (int64_t)gridDim.x * a.tpw) {
    const int64_t m = base + team;
    const bool act = m < N;
    Real x[Q][8], u[Q][8], g[Q][8], z[Q][8];
    load_row<Real, Q>(X + m * ld, r, T, d, act, x);
    double lp = tgt.eval(a, x, g, stage, red, slot, r, T);
    lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_FULL_REFRESH, 0, z);
    double v2[2] = {lp, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) v2[1] += (double)z[q][i] * (double)z[q][i];
    team_sum<2>(v2, T, red, slot);
    lp = v2[0];
    {
      const Real iz = (Real)(1.0 / sqrt(v2[1]));
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) u[q][i] = z[q][i] * iz;
    }
    double D = 0.0;
    for (int j = 0; j < a.n_traj; ++j) {
      lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_O_FIRST, (uint32_t)j, z);
      double v3[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const Real w = c1 * u[q][i] + c2 * z[q][i];
          const Real gt = sg[q][i] * g[q][i];
          u[q][i] = w;
          v3[0] += (double)w * (double)w;
          v3[1] += (double)gt * (double)w;
          v3[2] += (double)gt * (double)gt;
        }
      team_sum<3>(v3, T, red, slot);
      const double inw = 1.0 / sqrt(v3[0]);
      BMap b = b_map_t<Real>(v3[2], v3[1] * inw, C.b[0] * eps, dm1);
      D += b.dK;
      {
        const Real Ab = (Real)(b.A * inw), Bb = (Real)b.Bg;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) u[q][i] = Ab * u[q][i] + Bb * sg[q][i] * g[q][i];
      }
      constexpr int KB = INTEG == 2 ? 6 : (INTEG == 1 ? 3 : 2);
#pragma unroll 1
      for (int k = 0; k < KB - 1; ++k) {
        const Real ha = (Real)(kCoefA[INTEG][k] * eps);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) x[q][i] += ha * sg[q][i] * u[q][i];
        const double lpn = tgt.eval(a, x, g, stage, red, slot, r, T);
        double w3[3] = {lpn, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const Real gt = sg[q][i] * g[q][i];
            w3[1] += (double)gt * (double)gt;
            w3[2] += (double)gt * (double)u[q][i];
          }
        team_sum<3>(w3, T, red, slot);
        D += lp - w3[0];
        lp = w3[0];
        b = b_map_t<Real>(w3[1], w3[2], kCoefB[INTEG][k + 1] * eps, dm1);
        D += b.dK;
        const Real Ab = (Real)b.A, Bb = (Real)b.Bg;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) u[q][i] = Ab * u[q][i] + Bb * sg[q][i] * g[q][i];
      }
      lane_normals<Real, Q>(a.seed, (uint64_t)m, r, T, d, t, TAG_O_SECOND, (uint32_t)j, z);
      double v1[1] = {0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const Real w = c1 * u[q][i] + c2 * z[q][i];
          u[q][i] = w;
          v1[0] += (double)w * (double)w;
        }
      team_sum<1>(v1, T, red, slot);
      const Real in2 = (Real)(1.0 / sqrt(v1[0]));
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) u[q][i] *= in2;
    }
    const double wacc = exp(-D);
    const bool nanD = (D != D);
    const double am = nanD ? 0.0 : (wacc < 1.0 ? wacc : 1.0);
    const double U01 = mh_uniform(a.seed, (uint64_t)m, t);
    const bool accept = !nanD && (U01 < wacc);
    if (act) {
      if (accept) {
        store_row<Real, Q>(X + m * ld, r, T, d, x);
        if (a.cache) store_row<Real, Q>(static_cast<Real *>(a.g) + m * ld, r, T, d, g);
        if (r == 0) a.logp[m] = lp;
      }
      if (r == 0) {
        a.acc[m] = am;
        a.delta[m] = D;
      }
    }
  }
}

// Standalone evaluation: log p and (optionally) its gradient for each row.
template <class Real, int Q, class Tgt>
__global__ void __launch_bounds__(512) k_eval(LocalArgs a) {
  LAPS_TEAM_PROLOGUE
  Tgt tgt;
  tgt.setup(a, r, T);
  const Real *X = static_cast<const Real *>(a.x);
  for (int64_t base = (int64_t)blockIdx.x * a.tpw; base < N; base += (int64_t)gridDim.x * a.tpw) {
    const int64_t m = base + team;
    const bool act = m < N;
    Real x[Q][8], g[Q][8];
    load_row<Real, Q>(X + m * ld, r, T, d, act, x);
    double v[1] = {tgt.eval(a, x, g, stage, red, slot, r, T)};
    team_sum<1>(v, T, red, slot);
    if (act) {
      if (a.g_out) store_row<Real, Q>(static_cast<Real *>(a.g_out) + m * ld, r, T, d, g);
      if (r == 0) a.logp_out[m] = v[0];
    }
  }
}

// Column sums over a block of chains: thread i of grid column cb owns
// dimension i and walks chains cb, cb + CB, ... in order (coalesced across the
// threads of a row).
template <class Real>
__global__ void __launch_bounds__(256) k_stats(const Real *x, const Real *g, const double *shiftK, double *partials,
                                               int64_t N, int64_t d, int64_t ld, int CB, const DevHyper *hyp) {
  if (hyp && hyp->phase != PH_UNADJ) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int cb = blockIdx.y;
  if (i >= d) return;
  const double K = shiftK[i];
  double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  int64_t m = cb;
  for (; m + 3 * CB < N; m += 4 * CB) {
    double xv[4], gv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      xv[k] = (double)x[(m + k * CB) * ld + i] - K;
      gv[k] = (double)g[(m + k * CB) * ld + i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s1 += xv[k];
      s2 += xv[k] * xv[k];
      s3 += xv[k] * gv[k];
      s4 += gv[k];
    }
  }
  for (; m < N; m += CB) {
    const double xv = (double)x[m * ld + i] - K, gv = (double)g[m * ld + i];
    s1 += xv;
    s2 += xv * xv;
    s3 += xv * gv;
    s4 += gv;
  }
  double *P = partials + (size_t)cb * 4 * ld;
  P[i] = s1;
  P[ld + i] = s2;
  P[2 * ld + i] = s3;
  P[3 * ld + i] = s4;
}

hipError_t launch_stats(bool dbl, const void *x, const void *g, const double *shiftK, double *partials, int64_t N,
                        int64_t d, int64_t ld, int CB, const DevHyper *hyp, hipStream_t s) {
  const dim3 grid((unsigned)((d + 255) / 256), (unsigned)CB);
  if (dbl)
    hipLaunchKernelGGL(k_stats<double>, grid, dim3(256), 0, s, (const double *)x, (const double *)g, shiftK,
                       partials, N, d, ld, CB, hyp);
  else
    hipLaunchKernelGGL(k_stats<float>, grid, dim3(256), 0, s, (const float *)x, (const float *)g, shiftK, partials,
                       N, d, ld, CB, hyp);
  return hipGetLastError();
}

// per-dim constants of the targets in the state type: 1/s2 (Gaussian), y^2 (SV)
template <class Real>
__global__ void k_prep_aux(int kind, const double *src, Real *aux, int64_t d, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ld) return;
  Real v = Real(0);
  if (kind == 0 && i < d) v = (Real)(1.0 / src[i]);
  if (kind == 2 && i < d - 2) v = (Real)(src[i] * src[i]);
  aux[i] = v;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <class Real, int Q, class Tgt>
static hipError_t launch_kind(KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem, hipStream_t s) {
  switch (kk) {
    case KK_INIT:
      if (a.stats)
        hipLaunchKernelGGL((k_init<Real, Q, Tgt, true>), dim3(grid), dim3(block), shmem, s, a);
      else
        hipLaunchKernelGGL((k_init<Real, Q, Tgt, false>), dim3(grid), dim3(block), shmem, s, a);
      break;
    case KK_UNADJ:
      if (a.stats)
        hipLaunchKernelGGL((k_unadj<Real, Q, Tgt, true>), dim3(grid), dim3(block), shmem, s, a);
      else
        hipLaunchKernelGGL((k_unadj<Real, Q, Tgt, false>), dim3(grid), dim3(block), shmem, s, a);
      break;
    case KK_MAMS_MN2: hipLaunchKernelGGL((k_mams<Real, Q, Tgt, 1>), dim3(grid), dim3(block), shmem, s, a); break;
    case KK_MAMS_MN4: hipLaunchKernelGGL((k_mams<Real, Q, Tgt, 2>), dim3(grid), dim3(block), shmem, s, a); break;
    case KK_EVAL: hipLaunchKernelGGL((k_eval<Real, Q, Tgt>), dim3(grid), dim3(block), shmem, s, a); break;
  }
  return hipGetLastError();
}

template <class Real, int Q>
static hipError_t launch_q(int kind, KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem,
                           hipStream_t s) {
  if (kind == 0) return launch_kind<Real, Q, GaussTgt<Real, Q>>(kk, a, grid, block, shmem, s);
  if (kind == 2) return launch_kind<Real, Q, SVTgt<Real, Q>>(kk, a, grid, block, shmem, s);
  if (kind == 3) return launch_kind<Real, Q, Phi4Tgt<Real, Q>>(kk, a, grid, block, shmem, s);
  return hipErrorInvalidValue;
}

hipError_t launch_local(int kind, bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block,
                        size_t shmem, hipStream_t s) {
  if (dbl) {
    if (Q == 1) return launch_q<double, 1>(kind, kk, a, grid, block, shmem, s);
    if (Q == 2) return launch_q<double, 2>(kind, kk, a, grid, block, shmem, s);
  } else {
    if (Q == 1) return launch_q<float, 1>(kind, kk, a, grid, block, shmem, s);
    if (Q == 2) return launch_q<float, 2>(kind, kk, a, grid, block, shmem, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_prep_aux(int kind, bool dbl, const void *src, void *aux, int64_t d, int64_t ld, hipStream_t s) {
  const int grid = (int)((ld + 255) / 256);
  if (dbl)
    hipLaunchKernelGGL(k_prep_aux<double>, dim3(grid), dim3(256), 0, s, kind, (const double *)src, (double *)aux, d,
                       ld);
  else
    hipLaunchKernelGGL(k_prep_aux<float>, dim3(grid), dim3(256), 0, s, kind, (const double *)src, (float *)aux, d,
                       ld);
  return hipGetLastError();
}

}  // namespace laps
