// Per-chain kernels of the LAPS hot path for targets whose gradient is local
// to one chain: the diagonal Gaussian, stochastic volatility (tridiagonal
// AR(1) prior) and the 2-D phi^4 lattice.
//
// Layout: chain-major [N][ld] rows.  A team of T lanes holds one chain in
// registers; lane r owns octs r + q T (q < Q, eight consecutive coordinates
// each, the unit of one Philox block), so every load is a contiguous 32- or
// 64-byte vector per lane and the team's accesses are coalesced.  Teams of up
// to 64 lanes live inside one wavefront: their dot products are xor
// butterflies and their neighbour exchanges cross-lane moves, with no
// workgroup barrier; only chains too long for 64 lanes x Q octs use
// multi-wavefront teams.  Q grows with d so that the per-chain scalar work
// (velocity-map coefficients, reductions, target hyperparameters) is shared by
// many coordinates per lane.
//
// Per-dimension constants (1/s2, y^2, the preconditioner sigma) are staged
// once per workgroup in LDS.  Per-dimension ensemble sums are either
// accumulated in registers across the chains a workgroup visits (one oct per
// lane) or left to the column-sum kernel.
#pragma once
#include "laps_team.hpp"

namespace laps {

// LDS exchange inside a team.  A team inside one wavefront only needs its own
// LDS operations to stay in program order (the wavefront's LDS accesses
// execute in issue order), which a wavefront-scope fence enforces on the
// compiler; a multi-wavefront team needs the workgroup barrier.
__device__ __forceinline__ void team_sync(int T) {
  if (T <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Per-oct partial sums: FP32 state sums the eight terms of an oct in float and
// adds the oct's sum in double; FP64 state stays in double throughout.
template <class Real>
__device__ __forceinline__ double widen(Real v) {
  return (double)v;
}

// Keeps the scheduler from hoisting the next oct's loads and transcendentals
// above this oct's arithmetic: with Q octs per lane unrolled, unrestricted
// hoisting multiplies the live registers and forces spills.
__device__ __forceinline__ void oct_fence() { __builtin_amdgcn_sched_barrier(0); }

struct Team {
  int r, T;
  double *red;
  int slot;
};

// Team-wide broadcast of the coordinates e0 and e1 of the chain (every lane
// gets both): the owners contribute their values, the rest zeros.
template <class Real, int Q>
__device__ __forceinline__ void team_coords(const Real (&x)[Q][8], int e0, int e1, Team &tm, double (&out)[2]) {
  out[0] = 0.0;
  out[1] = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = 8 * (tm.r + q * tm.T);
    if (b + 8 > e0 && b <= e1) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (b + i == e0) out[0] = (double)x[q][i];
        if (b + i == e1) out[1] = (double)x[q][i];
      }
    }
  }
  team_sum<2>(out, tm.T, tm.red, tm.slot);
}

// ---------------------------------------------------------------------------
// Targets.  eval() returns this lane's share of log p (the caller reduces it
// with its own dot products) and fills g; coordinates >= d get g = 0.
//   kAux:   uses one per-dimension constant row (staged in LDS)
//   kCache: the gradient is costly, so the unadjusted step keeps g and log p
//           from the previous step instead of re-evaluating at its start
//   kStage: needs a team-private copy of the chain in LDS (neighbours)
// ---------------------------------------------------------------------------

// Diagonal Gaussian: log p = -1/2 sum x_i^2 / s2_i, g = -x / s2.
template <class Real, int Q>
struct GaussTgt {
  static constexpr bool kAux = true, kCache = false;
  static __host__ __device__ constexpr bool stage(int) { return false; }
  static __device__ Real aux_at(const LocalArgs &a, int64_t i) { return i < a.d ? (Real)(1.0 / a.tdata[i]) : Real(0); }
  __device__ double eval(const LocalArgs &a, const Real (&x)[Q][8], Real (&g)[Q][8], Team &tm, const Real *aux,
                         Real *) {
    double lp = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (tm.r + q * tm.T);
      Real inv[8];
      if (e0 < a.d) {
        ld8<Real>(aux + e0, inv);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) inv[i] = Real(0);
      }
      Real p = Real(0);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        g[q][i] = -x[q][i] * inv[i];
        p += x[q][i] * g[q][i];
      }
      lp += 0.5 * widen(p);
    }
    return lp;
  }
};

// 2-D periodic phi^4 (L x L): g = sum of the four neighbours - (4 + m2) f
// - 4 lambda f^3; log p = -sum [1/2 (f_right - f)^2 + 1/2 (f_down - f)^2
// + m2/2 f^2 + lambda f^4].  The chain is staged in the team's LDS row.  When
// L is a multiple of 8 (Phi4Tgt) an oct never straddles a lattice row, so the
// vertical neighbours are whole octs and the horizontal ones mostly in
// registers; other L (Phi4AnyTgt, one oct per lane) read every neighbour from
// LDS.
template <class Real>
struct Phi4Terms {
  Real diag, lam4, hm2, lam;
  __device__ Phi4Terms(const LocalArgs &a) {
    const Real m2 = (Real)a.tp0;
    lam = (Real)a.tp1;
    diag = Real(4) + m2;
    lam4 = Real(4) * lam;
    hm2 = Real(0.5) * m2;
  }
  // gradient of one site, and its share of -log p
  __device__ __forceinline__ Real site(Real f, Real fl, Real fr, Real fu, Real fd, Real &g) const {
    const Real f2 = f * f;
    g = (fr + fl + fd + fu) - diag * f - lam4 * f2 * f;
    const Real dr = fr - f, dd = fd - f;
    return Real(0.5) * (dr * dr + dd * dd) + hm2 * f2 + lam * f2 * f2;
  }
};

template <class Real, int Q>
struct Phi4Tgt {
  static constexpr bool kAux = false, kCache = true;
  static __host__ __device__ constexpr bool stage(int) { return true; }
  static __device__ Real aux_at(const LocalArgs &, int64_t) { return Real(0); }
  __device__ double eval(const LocalArgs &a, const Real (&x)[Q][8], Real (&g)[Q][8], Team &tm, const Real *,
                         Real *stage) {
    const int L = (int)a.tn;
    const int d = (int)a.d;
    const int r = tm.r, T = tm.T;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
      if (e0 < d) st8<Real>(stage + e0, x[q]);
    }
    team_sync(T);
    const Phi4Terms<Real> P(a);
    const int wpr = L >> 3;  // octs per lattice row
    double lp = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int oct = r + q * T;
      const int e0 = 8 * oct;
      if (e0 < d) {
        const int row = oct / wpr, c0 = e0 - row * L;
        const int up = (row == 0 ? L - 1 : row - 1) * L + c0;
        const int dn = (row + 1 == L ? 0 : row + 1) * L + c0;
        Real fu[8], fd[8];
        ld8<Real>(stage + up, fu);
        ld8<Real>(stage + dn, fd);
        const Real le = stage[row * L + (c0 == 0 ? L - 1 : c0 - 1)];
        const Real re = stage[row * L + (c0 + 8 == L ? 0 : c0 + 8)];
        Real p = Real(0);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          p += P.site(x[q][i], i ? x[q][i - 1] : le, i < 7 ? x[q][i + 1] : re, fu[i], fd[i], g[q][i]);
        lp -= widen(p);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) g[q][i] = Real(0);
      }
    }
    team_sync(T);
    return lp;
  }
};

template <class Real, int Q>
struct Phi4AnyTgt {
  static constexpr bool kAux = false, kCache = true;
  static __host__ __device__ constexpr bool stage(int) { return true; }
  static __device__ Real aux_at(const LocalArgs &, int64_t) { return Real(0); }
  __device__ double eval(const LocalArgs &a, const Real (&x)[Q][8], Real (&g)[Q][8], Team &tm, const Real *,
                         Real *stage) {
    const int L = (int)a.tn;
    const int d = (int)a.d;
    const int r = tm.r, T = tm.T;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
      if (e0 < d) st8<Real>(stage + e0, x[q]);
    }
    team_sync(T);
    const Phi4Terms<Real> P(a);
    double lp = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
      Real p = Real(0);
      int row = e0 / L, col = e0 - row * L;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = e0 + i;
        if (e < d) {
          const int rb = row * L;
          const int cl = col == 0 ? L - 1 : col - 1, cr = col + 1 == L ? 0 : col + 1;
          const int up = e >= L ? e - L : e - L + d, dn = e + L < d ? e + L : e + L - d;
          p += P.site(x[q][i], stage[rb + cl], stage[rb + cr], stage[up], stage[dn], g[q][i]);
        } else {
          g[q][i] = Real(0);
        }
        if (++col == L) {
          col = 0;
          ++row;
        }
      }
      lp -= widen(p);
    }
    team_sync(T);
    return lp;
  }
};

// Stochastic volatility, theta = (h_1..h_T, s, r): sigma = e^s, phi = tanh r,
// E = (1 - phi^2) h_1^2 + sum_{t>=2} (h_t - phi h_{t-1})^2,
// log p = -2 (s+2)^2 - 2 (r-2)^2 - T s + 1/2 log(1 - phi^2) - E/(2 sigma^2)
//         - 1/2 sum h_t - 1/2 sum y_t^2 e^{-h_t}.
// Neighbours h_{t-1}, h_{t+1} of an oct's end coordinates come from the
// adjacent lanes by cross-lane moves (multi-wavefront teams go through LDS);
// (s, r) are broadcast by a team sum.  The (s, r) gradients need sums over t,
// so (E, cross, lik) are reduced over the team before the two owner lanes
// finish them.
template <class Real, int Q>
struct SVTgt {
  static constexpr bool kAux = true, kCache = true;
  static __host__ __device__ constexpr bool stage(int T) { return T > 64; }
  static __device__ Real aux_at(const LocalArgs &a, int64_t i) {
    return i < a.tn ? (Real)(a.tdata[i] * a.tdata[i]) : Real(0);
  }
  __device__ double eval(const LocalArgs &a, const Real (&x)[Q][8], Real (&g)[Q][8], Team &tm, const Real *aux,
                         Real *stage) {
    const int Tn = (int)a.tn;
    const int d = (int)a.d;
    const int r = tm.r, T = tm.T;
    Real prv[Q], nxt[Q];
    double sr[2];
    if (T <= 64) {
      Real rp[Q], rn[Q];
      const int lp_ = (r + T - 1) & (T - 1), ln_ = (r + 1) & (T - 1);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        rp[q] = __shfl(x[q][7], lp_, T);
        rn[q] = __shfl(x[q][0], ln_, T);
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        prv[q] = (r == 0) ? (q > 0 ? rp[q > 0 ? q - 1 : 0] : Real(0)) : rp[q];
        nxt[q] = (r == T - 1) ? (q + 1 < Q ? rn[q + 1 < Q ? q + 1 : 0] : Real(0)) : rn[q];
      }
      team_coords<Real, Q>(x, Tn, Tn + 1, tm, sr);
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int e0 = 8 * (r + q * T);
        if (e0 < d) st8<Real>(stage + e0, x[q]);
      }
      team_sync(T);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int e0 = 8 * (r + q * T);
        prv[q] = (e0 > 0 && e0 < d) ? stage[e0 - 1] : Real(0);
        nxt[q] = (e0 + 8 < d) ? stage[e0 + 8] : Real(0);
      }
      sr[0] = (double)stage[Tn];
      sr[1] = (double)stage[Tn + 1];
      team_sync(T);
    }
    const double s = sr[0], rr = sr[1];
    const double sig2 = exp(2.0 * s), phi = tanh(rr), omp = 1.0 - phi * phi;
    const Real phR = (Real)phi, ompR = (Real)omp, isR = (Real)(1.0 / sig2);
    double v[3] = {0.0, 0.0, 0.0};  // E, cross, lik
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
      Real y2[8];
      if (e0 < d) {
        ld8<Real>(aux + e0, y2);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) y2[i] = Real(0);
      }
      Real pE = Real(0), pC = Real(0), pL = Real(0);
      if (e0 > 0 && e0 + 8 < Tn) {
        // interior oct: every coordinate is a latent h_t with both neighbours
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const Real h = x[q][i];
          const Real hp = i ? x[q][i - 1] : prv[q];
          const Real hn = i < 7 ? x[q][i + 1] : nxt[q];
          const Real an = hn - phR * h;
          const Real at = h - phR * hp;
          const Real eh = sizeof(Real) == 4 ? (Real)__expf(-(float)h) : (Real)exp(-(double)h);
          g[q][i] = -(at - phR * an) * isR - Real(0.5) + Real(0.5) * y2[i] * eh;
          pE += at * at;
          pC += at * hp;
          pL += Real(-0.5) * h - Real(0.5) * y2[i] * eh;
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int e = e0 + i;
          const Real h = x[q][i];
          const Real hp = i ? x[q][i - 1] : prv[q];
          const Real hn = i < 7 ? x[q][i + 1] : nxt[q];
          if (e < Tn) {
            const Real an = (e + 1 < Tn) ? (hn - phR * h) : Real(0);
            const Real at = (e == 0) ? h : (h - phR * hp);
            const Real own = (e == 0) ? ompR * h : at;
            const Real eh = sizeof(Real) == 4 ? (Real)__expf(-(float)h) : (Real)exp(-(double)h);
            g[q][i] = -(own - phR * an) * isR - Real(0.5) + Real(0.5) * y2[i] * eh;
            pE += (e == 0) ? ompR * h * h : at * at;
            pC += (e == 0) ? phR * h * h : at * hp;
            pL += Real(-0.5) * h - Real(0.5) * y2[i] * eh;
          } else {
            g[q][i] = Real(0);
          }
        }
      }
      v[0] += widen(pE);
      v[1] += widen(pC);
      v[2] += widen(pL);
      oct_fence();
    }
    team_sum<3>(v, T, tm.red, tm.slot);
    const double E = v[0], cross = v[1], lik = v[2];
    const Real gs = (Real)(-4.0 * (s + 2.0) - (double)Tn + E / sig2);
    const Real gr = (Real)(-4.0 * (rr - 2.0) - phi + omp * cross / sig2);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e0 = 8 * (r + q * T);
      if (e0 + 8 > Tn && e0 <= Tn + 1) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int e = e0 + i;
          if (e == Tn) g[q][i] = gs;
          if (e == Tn + 1) g[q][i] = gr;
        }
      }
    }
    const double lp = -2.0 * (s + 2.0) * (s + 2.0) - 2.0 * (rr - 2.0) * (rr - 2.0) - (double)Tn * s +
                      0.5 * log(omp) - E / (2.0 * sig2) + lik;
    return (r == 0) ? lp : 0.0;
  }
};

// Integrator coefficients by integrator id (0 LF, 1 MN2, 2 MN4), in constant
// memory so that a rolled loop over the composition reads them by index.
static __constant__ double kCoefB[3][6] = {
    {0.5, 0.5, 0.0, 0.0, 0.0, 0.0},
    {0.1931833275, 1.0 - 2.0 * 0.1931833275, 0.1931833275, 0.0, 0.0, 0.0},
    {0.0839831526, 0.6822365335, 0.5 - 0.0839831526 - 0.6822365335, 0.5 - 0.0839831526 - 0.6822365335, 0.6822365335,
     0.0839831526}};
static __constant__ double kCoefA[3][5] = {
    {1.0, 0.0, 0.0, 0.0, 0.0},
    {0.5, 0.5, 0.0, 0.0, 0.0},
    {0.2539785108, -0.032302867, 1.0 - 2.0 * (0.2539785108 - 0.032302867), -0.032302867, 0.2539785108}};

// ---------------------------------------------------------------------------
// LDS layout of the per-chain kernels:
//   [reduction slots | aux row (kAux) | sigma row (adjusted phase) | body]
// body = the teams' chain copies (kStage) or, at the end of a statistics
// pass, the staging buffer of the per-dim partial row.  The host sizes it.
// ---------------------------------------------------------------------------
template <class Real>
__device__ __forceinline__ void stage_row(Real *dst, const void *src, int64_t ld) {
  const float4 *s = static_cast<const float4 *>(src);
  float4 *t = reinterpret_cast<float4 *>(dst);
  const int64_t n = ld * (int64_t)sizeof(Real) / 16;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) t[i] = s[i];
}

#define LAPS_TEAM_DECLS(WITH_SIGMA)                                                                 \
  extern __shared__ double smem[];                                                                  \
  const int T = a.T;                                                                                \
  const int team = threadIdx.x / T, r = threadIdx.x - team * T;                                     \
  const int64_t N = a.N, d = a.d, ld = a.ld;                                                        \
  const double dm1 = (double)(d - 1);                                                               \
  Team tm{r, T, smem, 0};                                                                           \
  Real *caux = reinterpret_cast<Real *>(smem + 2 * kRedSlots);                                      \
  Real *csig = caux + (Tgt::kAux ? ld : 0);                                                         \
  Real *body = csig + ((WITH_SIGMA) ? ld : 0);                                                      \
  Real *stage = Tgt::stage(T) ? body + (size_t)team * ld : nullptr;

#define LAPS_TEAM_STAGE(WITH_SIGMA)                                                                 \
  if (Tgt::kAux) {                                                                                  \
    if (a.aux)                                                                                      \
      stage_row<Real>(caux, a.aux, ld);                                                             \
    else                                                                                            \
      for (int64_t i_ = threadIdx.x; i_ < ld; i_ += blockDim.x) caux[i_] = Tgt::aux_at(a, i_);      \
  }                                                                                                 \
  if (WITH_SIGMA) stage_row<Real>(csig, a.sigma, ld);                                               \
  if (Tgt::kAux || (WITH_SIGMA)) __syncthreads();

#define LAPS_TEAM_PROLOGUE(WITH_SIGMA) \
  LAPS_TEAM_DECLS(WITH_SIGMA)          \
  LAPS_TEAM_STAGE(WITH_SIGMA)

// ---------------------------------------------------------------------------
// Initialisation: log p and gradient at x, u = g/|g| (u0 if given; a uniform
// random direction when the gradient vanishes), per-dim sums for the initial
// variances (shift K = 0).
// ---------------------------------------------------------------------------
template <class Real, int Q, class Tgt, bool STATS>
__global__ void __launch_bounds__(512) k_init(LocalArgs a) {
  LAPS_TEAM_PROLOGUE(false)
  Tgt tgt;
  double S[4][STATS ? Q : 1][8] = {};
  double K0[STATS ? Q : 1][8] = {};
  const Real *X = static_cast<const Real *>(a.x);
  const bool keep_g = Tgt::kCache || a.cache;
  for (int64_t base = (int64_t)blockIdx.x * a.tpw; base < N; base += (int64_t)gridDim.x * a.tpw) {
    const int64_t m = base + team;
    const bool act = m < N;
    Real x[Q][8], g[Q][8], u[Q][8];
    load_row<Real, Q>(X + m * ld, r, T, d, act, x);
    const double lp = tgt.eval(a, x, g, tm, caux, stage);
    // fallback direction when the gradient vanishes: a normalised normal vector
#pragma unroll
    for (int q = 0; q < Q; ++q) oct_normals<Real>(a.seed, (uint64_t)m, r + q * T, d, 0, TAG_INIT_DIR, 0, u[q]);
    double v[3] = {lp, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Real p1 = Real(0), p2 = Real(0);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        p1 += g[q][i] * g[q][i];
        p2 += u[q][i] * u[q][i];
      }
      v[1] += widen(p1);
      v[2] += widen(p2);
    }
    team_sum<3>(v, T, tm.red, tm.slot);
    if (a.u0) {
      load_row<Real, Q>(static_cast<const Real *>(a.u0) + m * ld, r, T, d, act, u);
    } else {
      const double gn = sqrt(v[1]);
      const bool useg = gn > 0.0 && isfinite(gn);
      const Real sc = (Real)(1.0 / (useg ? gn : sqrt(v[2])));
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) u[q][i] = (useg ? g[q][i] : u[q][i]) * sc;
    }
    if (act) {
      store_row<Real, Q>(static_cast<Real *>(a.x) + m * ld, r, T, d, x);
      store_row<Real, Q>(static_cast<Real *>(a.u) + m * ld, r, T, d, u);
      if (keep_g) store_row<Real, Q>(static_cast<Real *>(a.g) + m * ld, r, T, d, g);
      if (r == 0) {
        a.logp[m] = v[0];
        a.delta[m] = 0.0;
        a.acc[m] = 0.0;
      }
      if constexpr (STATS) accumulate_stats<Real, Q>(S, K0, x, g);
    }
  }
  if constexpr (STATS) write_partials<Real, Q>(a.partials, a.d, a.ld, S, reinterpret_cast<double *>(body), T, r);
}

// ---------------------------------------------------------------------------
// One unadjusted step (eq. discrete update, leapfrog):
//   O_{eps/2}  B_{eps/2}  A_eps  [grad]  B_{eps/2}  O_{eps/2}
// Energy error Delta = (log p before - log p after) + the two B energies.
// The first O's normalisation and the first B's dot products share one team
// reduction (g.u = g.w / |w|).  Costly targets start from the gradient and
// log p the previous step stored (identical to re-evaluating at the same x).
// Ensemble sums of the new state go to the workgroup's partial row (STATS) or
// are left to the column-sum kernel, which reads the stored x and g.
// ---------------------------------------------------------------------------
//
// When the chain workgroups leave compute units idle (few chains, FP64
// normals), zn_blocks more workgroups are appended to the launch.  They
// compute the normals of the two partial refreshes of step t + 1 (one Philox
// block and four Box-Muller pairs per thread and oct, the values oct_normals
// returns) into the slot of step t + 1 and tag it; the next step's chain
// workgroups then load their normals instead of computing them, and compute
// them as before when the slot is not tagged with their step.  The normals
// depend only on (seed, chain, oct, step), so a tagged slot is valid across
// restarts, and a step's results do not depend on where its normals came from.
template <class Real>
__device__ void fill_step_noise(const LocalArgs &a, uint64_t t1, int64_t idx) {
  const int64_t octs = (a.d + 7) / 8, per = a.N * octs;
  if (idx == 0) a.zn_tag[t1 & 1] = t1 + 1;
  if (idx >= 2 * per) return;
  const int k = (int)(idx / per);
  const int64_t rem = idx - k * per, m = rem / octs, oct = rem - m * octs;
  Real z[8];
  oct_normals<Real>(a.seed, (uint64_t)m, oct, a.d, t1, k == 0 ? TAG_O_FIRST : TAG_O_SECOND, 0, z);
  st8<Real>(static_cast<Real *>(a.zn) + (((int64_t)(t1 & 1) * 2 + k) * a.N + m) * a.ld + 8 * oct, z);
}

// The normals of refresh k (0 first, 1 second) of step t for oct `oct` of
// chain m: from the tagged slot zs when there is one, else computed.
template <class Real>
__device__ __forceinline__ void step_normals(const LocalArgs &a, const Real *zs, bool act, int k, int64_t m,
                                             int64_t oct, uint64_t t, Real (&z)[8]) {
  if (zs) {
    if (act && 8 * oct < a.d) {
      ld8<Real>(zs + ((int64_t)k * a.N + m) * a.ld + 8 * oct, z);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) z[i] = Real(0);
    }
  } else {
    oct_normals<Real>(a.seed, (uint64_t)m, oct, a.d, t, k == 0 ? TAG_O_FIRST : TAG_O_SECOND, 0, z);
  }
}

template <class Real, int Q, class Tgt, bool STATS>
__global__ void __launch_bounds__(512) k_unadj(LocalArgs a) {
  // The phase word, the step's scalars, both normal slots' tags and the
  // launch's first independent loads (the shift row, the staged aux row) are
  // issued together; the phase is tested after the staging barrier (uniformly)
  // and before the first global store, so no load waits for another.
  const DevHyper *H = a.hyp;
  const int phase = H->phase;
  const double eps = H->eps, Lm = H->L;
  const uint64_t t = (uint64_t)H->t;
  const uint64_t tag0 = a.zn_blocks > 0 ? a.zn_tag[0] : 0, tag1 = a.zn_blocks > 0 ? a.zn_tag[1] : 0;
  LAPS_TEAM_DECLS(false)
  double K[STATS ? Q : 1][8];
  if constexpr (STATS) load_shift<Q>(a.shiftK, r, T, d, K);
  LAPS_TEAM_STAGE(false)
  if (phase != PH_UNADJ) {
    __builtin_amdgcn_s_waitcnt(0);
    return;
  }
  const int cgrid = (int)gridDim.x - a.zn_blocks;  // chain workgroups
  if ((int)blockIdx.x >= cgrid) {
    fill_step_noise<Real>(a, t + 1, (int64_t)(blockIdx.x - cgrid) * blockDim.x + threadIdx.x);
    return;
  }
  const Real *zs = (a.zn_blocks > 0 && ((t & 1) ? tag1 : tag0) == t + 1)
                       ? static_cast<const Real *>(a.zn) + (size_t)(t & 1) * 2 * N * ld
                       : nullptr;
  const double h = 0.5 * eps;
  const double c1d = exp(-h / Lm), c2d = sqrt(-expm1(-2.0 * h / Lm)) / sqrt((double)d);
  const Real c1 = (Real)c1d, c2 = (Real)c2d, epsR = (Real)eps;
  Tgt tgt;
  double S[4][STATS ? Q : 1][8] = {};
  const bool keep_g = Tgt::kCache || a.cache;
  Real *X = static_cast<Real *>(a.x);
  Real *U = static_cast<Real *>(a.u);
  Real *Gb = static_cast<Real *>(a.g);
  for (int64_t base = (int64_t)blockIdx.x * a.tpw; base < N; base += (int64_t)cgrid * a.tpw) {
    const int64_t m = base + team;
    const bool act = m < N;
    Real x[Q][8], u[Q][8], g[Q][8];
    load_row<Real, Q>(X + m * ld, r, T, d, act, x);
    load_row<Real, Q>(U + m * ld, r, T, d, act, u);
    double lp0;
    if constexpr (Tgt::kCache) {
      load_row<Real, Q>(Gb + m * ld, r, T, d, act, g);
      lp0 = (act && r == 0) ? a.logp[m] : 0.0;
    } else {
      lp0 = tgt.eval(a, x, g, tm, caux, stage);
    }
    // O (first half) fused with the dot products of the first B
    double v4[4] = {lp0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Real z[8];
      step_normals<Real>(a, zs, act, 0, m, r + q * T, t, z);
      Real p1 = Real(0), p2 = Real(0), p3 = Real(0);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const Real w = c1 * u[q][i] + c2 * z[i];
        u[q][i] = w;
        p1 += w * w;
        p2 += g[q][i] * w;
        p3 += g[q][i] * g[q][i];
      }
      v4[1] += widen(p1);
      v4[2] += widen(p2);
      v4[3] += widen(p3);
      oct_fence();
    }
    team_sum<4>(v4, T, tm.red, tm.slot);
    const double inw = refresh_scale(a.dyn, v4[1]);
    const BMap b1 = b_map_dyn<Real>(a.dyn, v4[3], v4[2] * inw, h, dm1);
    const Real A1 = (Real)(b1.A * inw), B1 = (Real)b1.Bg;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        u[q][i] = A1 * u[q][i] + B1 * g[q][i];
        x[q][i] += epsR * u[q][i];
      }
    const double lp1 = tgt.eval(a, x, g, tm, caux, stage);
    double v3[3] = {lp1, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Real p1 = Real(0), p2 = Real(0);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        p1 += g[q][i] * g[q][i];
        p2 += g[q][i] * u[q][i];
      }
      v3[1] += widen(p1);
      v3[2] += widen(p2);
    }
    team_sum<3>(v3, T, tm.red, tm.slot);
    const BMap b2 = b_map_dyn<Real>(a.dyn, v3[1], v3[2], h, dm1);
    const Real A2 = (Real)b2.A, B2 = (Real)b2.Bg;
    double v1[1] = {0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Real z[8];
      step_normals<Real>(a, zs, act, 1, m, r + q * T, t, z);
      Real p1 = Real(0);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const Real w = c1 * (A2 * u[q][i] + B2 * g[q][i]) + c2 * z[i];
        u[q][i] = w;
        p1 += w * w;
      }
      v1[0] += widen(p1);
      oct_fence();
    }
    team_sum<1>(v1, T, tm.red, tm.slot);
    const Real in2 = (Real)refresh_scale(a.dyn, v1[0]);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 8; ++i) u[q][i] *= in2;
    if (act) {
      store_row<Real, Q>(X + m * ld, r, T, d, x);
      store_row<Real, Q>(U + m * ld, r, T, d, u);
      if (keep_g) store_row<Real, Q>(Gb + m * ld, r, T, d, g);
      if (r == 0) {
        a.delta[m] = (v4[0] - v3[0]) + b1.dK + b2.dK;
        a.logp[m] = v3[0];
      }
      if constexpr (STATS) accumulate_stats<Real, Q>(S, K, x, g);
    }
  }
  if constexpr (STATS) write_partials<Real, Q>(a.partials, a.d, a.ld, S, reinterpret_cast<double *>(body), T, r);
}

// ---------------------------------------------------------------------------
// One MAMS transition per chain, fused (appendix "Metropolis adjusted
// microcanonical dynamics"): full refresh u = Z/|Z|, n_traj integrator steps
// O_{eps/2} Phi_eps O_{eps/2} with L_p = Lp_factor n_traj eps, in the
// preconditioned coordinates (x moves by h sigma*u, B uses sigma*g), then
// accept with probability min(1, e^{-Delta}).  The trajectory lives in
// registers and only the preconditioned gradient sigma*g is kept; on
// rejection nothing is written, so x and log p keep their starting values.
// ---------------------------------------------------------------------------
//
// As for the unadjusted step, workgroups appended to the launch (zm_blocks,
// FP64 one-oct-per-lane chains on an otherwise idle chip) compute the normals
// of the next transition (it starts n_traj steps later): row 0 the full
// refresh, rows 1 + 2j and 2 + 2j the two partial refreshes of integrator
// step j.  The chain workgroups of that transition load them one step ahead
// of their use when the slot is tagged with their start step, and compute
// them as before otherwise; both give the same values.
template <class Real>
__device__ void fill_transition_noise(const LocalArgs &a, uint64_t tn, int64_t wb) {
  const int KR = 2 * a.n_traj + 1;
  const int64_t octs = (a.d + 7) / 8, per = a.N * octs, total = (int64_t)KR * per;
  const uint64_t slot = (tn / (uint64_t)a.n_traj) & 1;
  const int64_t stride = (int64_t)a.zm_blocks * blockDim.x;
  int64_t idx = wb * blockDim.x + threadIdx.x;
  if (idx == 0) a.zm_tag[slot] = tn + 1;
  Real *base = static_cast<Real *>(a.zm) + (size_t)slot * KR * a.N * a.ld;
  for (; idx < total; idx += stride) {
    const int rr = (int)(idx / per);
    const int64_t rem = idx - rr * per, m = rem / octs, oct = rem - m * octs;
    const uint32_t tag = rr == 0 ? TAG_FULL_REFRESH : ((rr & 1) ? TAG_O_FIRST : TAG_O_SECOND);
    const uint32_t sub = rr == 0 ? 0u : (uint32_t)((rr - 1) / 2);
    Real z[8];
    oct_normals<Real>(a.seed, (uint64_t)m, oct, a.d, tn, tag, sub, z);
    st8<Real>(base + ((int64_t)rr * a.N + m) * a.ld + 8 * oct, z);
  }
}

// Row rr of a transition's normals for oct `oct` of chain m from slot zs.
template <class Real>
__device__ __forceinline__ void load_transition_normals(const LocalArgs &a, const Real *zs, bool act, int rr,
                                                        int64_t m, int64_t oct, Real (&z)[8]) {
  if (act && 8 * oct < a.d) {
    ld8<Real>(zs + ((int64_t)rr * a.N + m) * a.ld + 8 * oct, z);
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = Real(0);
  }
}

template <class Real, int Q, class Tgt, int INTEG>
__global__ void __launch_bounds__(512) k_mams(LocalArgs a) {
  const DevHyper *H = a.hyp;
  if (H->phase != PH_ADJ || H->t >= a.max_total) return;
  // chain workgroups (the host appends normals workgroups only for one oct per lane)
  const int cgrid = Q == 1 ? (int)gridDim.x - a.zm_blocks : (int)gridDim.x;
  if (Q == 1 && (int)blockIdx.x >= cgrid) {
    const uint64_t tn = (uint64_t)H->t + (uint64_t)a.n_traj;
    if (tn < (uint64_t)a.max_total) fill_transition_noise<Real>(a, tn, (int64_t)blockIdx.x - cgrid);
    return;
  }
  LAPS_TEAM_PROLOGUE(true)
  const double eps = H->eps;
  const uint64_t t = (uint64_t)H->t;
  const double h = 0.5 * eps;
  const double Lp = a.Lp_factor * (double)a.n_traj * eps;
  const double c1d = exp(-h / Lp), c2d = sqrt(-expm1(-2.0 * h / Lp)) / sqrt((double)d);
  const Real c1 = (Real)c1d, c2 = (Real)c2d;
  const Coeffs C = integrator_coeffs(INTEG);
  Tgt tgt;
  Real *X = static_cast<Real *>(a.x);
  // this transition's normals, when the previous launch wrote them (one oct per lane only: holding the
  // next step's normals across the gradient stages needs 2 x 8 Q more registers)
  const int KR = 2 * a.n_traj + 1;
  const uint64_t zslot = a.n_traj > 0 ? (t / (uint64_t)a.n_traj) & 1 : 0;
  const Real *zs = (Q == 1 && a.zm_blocks > 0 && a.zm_tag[zslot] == t + 1)
                       ? static_cast<const Real *>(a.zm) + (size_t)zslot * KR * N * ld
                       : nullptr;
  // sigma * v for the lane's octs, sigma read from LDS
  auto precond = [&](Real (&v)[Q][8]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t e0 = 8 * (int64_t)(r + q * T);
      if (e0 < d) {
        Real sg[8];
        ld8<Real>(csig + e0, sg);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[q][i] *= sg[i];
      }
    }
  };
  for (int64_t base = (int64_t)blockIdx.x * a.tpw; base < N; base += (int64_t)cgrid * a.tpw) {
    const int64_t m = base + team;
    const bool act = m < N;
    Real x[Q][8], u[Q][8], g[Q][8];
    Real zf[Q][8];  // loaded normals of the next first partial refresh
    load_row<Real, Q>(X + m * ld, r, T, d, act, x);
    if (zs) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        load_transition_normals<Real>(a, zs, act, 0, m, r + q * T, u[q]);
        load_transition_normals<Real>(a, zs, act, 1, m, r + q * T, zf[q]);
      }
    }
    double lp = tgt.eval(a, x, g, tm, caux, stage);
    precond(g);
    double v2[2] = {lp, 0.0};
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (!zs) oct_normals<Real>(a.seed, (uint64_t)m, r + q * T, d, t, TAG_FULL_REFRESH, 0, u[q]);
      Real p = Real(0);
#pragma unroll
      for (int i = 0; i < 8; ++i) p += u[q][i] * u[q][i];
      v2[1] += widen(p);
    }
    team_sum<2>(v2, T, tm.red, tm.slot);
    lp = v2[0];
    {
      const Real iz = (Real)full_refresh_scale(a.dyn, v2[1], d);
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int i = 0; i < 8; ++i) u[q][i] *= iz;
    }
    double D = 0.0;
    for (int j = 0; j < a.n_traj; ++j) {
      // loaded path: this step's second-refresh normals are requested now and used after the
      // gradient stages; the next step's first-refresh normals once this step's are used
      Real zsec[Q][8];
      if (zs) {
#pragma unroll
        for (int q = 0; q < Q; ++q) load_transition_normals<Real>(a, zs, act, 2 + 2 * j, m, r + q * T, zsec[q]);
      }
      double v3[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        Real z[8];
        if (zs) {
#pragma unroll
          for (int i = 0; i < 8; ++i) z[i] = zf[q][i];
        } else {
          oct_normals<Real>(a.seed, (uint64_t)m, r + q * T, d, t, TAG_O_FIRST, (uint32_t)j, z);
        }
        Real p1 = Real(0), p2 = Real(0), p3 = Real(0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const Real w = c1 * u[q][i] + c2 * z[i];
          u[q][i] = w;
          p1 += w * w;
          p2 += g[q][i] * w;
          p3 += g[q][i] * g[q][i];
        }
        v3[0] += widen(p1);
        v3[1] += widen(p2);
        v3[2] += widen(p3);
        oct_fence();
      }
      if (zs && j + 1 < a.n_traj) {
#pragma unroll
        for (int q = 0; q < Q; ++q) load_transition_normals<Real>(a, zs, act, 3 + 2 * j, m, r + q * T, zf[q]);
      }
      team_sum<3>(v3, T, tm.red, tm.slot);
      const double inw = refresh_scale(a.dyn, v3[0]);
      BMap b = b_map_dyn<Real>(a.dyn, v3[2], v3[1] * inw, C.b[0] * eps, dm1);
      D += b.dK;
      {
        const Real Ab = (Real)(b.A * inw), Bb = (Real)b.Bg;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) u[q][i] = Ab * u[q][i] + Bb * g[q][i];
      }
      constexpr int KB = INTEG == 2 ? 6 : (INTEG == 1 ? 3 : 2);
#pragma unroll 1
      for (int k = 0; k < KB - 1; ++k) {
        const Real ha = (Real)(kCoefA[INTEG][k] * eps);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int64_t e0 = 8 * (int64_t)(r + q * T);
          if (e0 < d) {
            Real sg[8];
            ld8<Real>(csig + e0, sg);
#pragma unroll
            for (int i = 0; i < 8; ++i) x[q][i] += ha * (sg[i] * u[q][i]);
          }
        }
        const double lpn = tgt.eval(a, x, g, tm, caux, stage);
        precond(g);
        double w3[3] = {lpn, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          Real p1 = Real(0), p2 = Real(0);
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            p1 += g[q][i] * g[q][i];
            p2 += g[q][i] * u[q][i];
          }
          w3[1] += widen(p1);
          w3[2] += widen(p2);
        }
        team_sum<3>(w3, T, tm.red, tm.slot);
        D += lp - w3[0];
        lp = w3[0];
        b = b_map_dyn<Real>(a.dyn, w3[1], w3[2], kCoefB[INTEG][k + 1] * eps, dm1);
        D += b.dK;
        const Real Ab = (Real)b.A, Bb = (Real)b.Bg;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int i = 0; i < 8; ++i) u[q][i] = Ab * u[q][i] + Bb * g[q][i];
      }
      double v1[1] = {0.0};
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        Real z[8];
        if (zs) {
#pragma unroll
          for (int i = 0; i < 8; ++i) z[i] = zsec[q][i];
        } else {
          oct_normals<Real>(a.seed, (uint64_t)m, r + q * T, d, t, TAG_O_SECOND, (uint32_t)j, z);
        }
        Real p = Real(0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const Real w = c1 * u[q][i] + c2 * z[i];
          u[q][i] = w;
          p += w * w;
        }
        v1[0] += widen(p);
        oct_fence();
      }
      team_sum<1>(v1, T, tm.red, tm.slot);
      const Real in2 = (Real)refresh_scale(a.dyn, v1[0]);
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
  LAPS_TEAM_PROLOGUE(false)
  Tgt tgt;
  const Real *X = static_cast<const Real *>(a.x);
  for (int64_t base = (int64_t)blockIdx.x * a.tpw; base < N; base += (int64_t)gridDim.x * a.tpw) {
    const int64_t m = base + team;
    const bool act = m < N;
    Real x[Q][8], g[Q][8];
    load_row<Real, Q>(X + m * ld, r, T, d, act, x);
    double v[1] = {tgt.eval(a, x, g, tm, caux, stage)};
    team_sum<1>(v, T, tm.red, tm.slot);
    if (act) {
      if (a.g_out) store_row<Real, Q>(static_cast<Real *>(a.g_out) + m * ld, r, T, d, g);
      if (r == 0) a.logp_out[m] = v[0];
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch for one target type
// ---------------------------------------------------------------------------
template <class Real, int Q, class Tgt>
hipError_t launch_kind(KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem, hipStream_t s) {
  void (*fn)(LocalArgs) = nullptr;
  switch (kk) {
    case KK_INIT:
      fn = k_init<Real, Q, Tgt, false>;
      if constexpr (Q == 1)
        if (a.stats) fn = k_init<Real, Q, Tgt, true>;
      break;
    case KK_UNADJ:
      fn = k_unadj<Real, Q, Tgt, false>;
      if constexpr (Q == 1)
        if (a.stats) fn = k_unadj<Real, Q, Tgt, true>;
      break;
    case KK_MAMS_MN2: fn = k_mams<Real, Q, Tgt, 1>; break;
    case KK_MAMS_MN4: fn = k_mams<Real, Q, Tgt, 2>; break;
    case KK_EVAL: fn = k_eval<Real, Q, Tgt>; break;
  }
  if (!fn) return hipErrorInvalidValue;
  const hipError_t e = grant_lds(reinterpret_cast<const void *>(fn), shmem);
  if (e != hipSuccess) return e;
  LocalArgs arg = a;
  void *args[] = {&arg};
  return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(grid), dim3(block), args, shmem, s);
}

// Octs per lane that have kernel instances: 1..6 for FP32 state, 1..2 for
// FP64 (whose registers hold half as many coordinates).
template <template <class, int> class TgtT>
hipError_t launch_target(bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem,
                         hipStream_t s) {
  if (dbl) {
    switch (Q) {
      case 1: return launch_kind<double, 1, TgtT<double, 1>>(kk, a, grid, block, shmem, s);
      case 2: return launch_kind<double, 2, TgtT<double, 2>>(kk, a, grid, block, shmem, s);
    }
  } else {
    switch (Q) {
      case 1: return launch_kind<float, 1, TgtT<float, 1>>(kk, a, grid, block, shmem, s);
      case 2: return launch_kind<float, 2, TgtT<float, 2>>(kk, a, grid, block, shmem, s);
      case 3: return launch_kind<float, 3, TgtT<float, 3>>(kk, a, grid, block, shmem, s);
      case 4: return launch_kind<float, 4, TgtT<float, 4>>(kk, a, grid, block, shmem, s);
      case 5: return launch_kind<float, 5, TgtT<float, 5>>(kk, a, grid, block, shmem, s);
      case 6: return launch_kind<float, 6, TgtT<float, 6>>(kk, a, grid, block, shmem, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace laps
