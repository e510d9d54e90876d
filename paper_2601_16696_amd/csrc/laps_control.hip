// Ensemble statistics and controllers of LAPS, all on the device:
//  - k_finalize: per-dimension moments from the workgroups' FP64 partial rows
//    (mean, variance, E[x_i^2], equipartition diagonal V_ii), the moving
//    window of E[x_i^2] and its relative fluctuation, block scalars;
//  - k_ctl_unadj: EEVPD, D~_diag, eps from F(C D~), L from the variances,
//    window bookkeeping and the switch flag (one workgroup);
//  - k_switch: the diagonal preconditioner and the adjusted-phase settings;
//  - k_ctl_adj: mean acceptance and the double/halve-then-bisect rule.
// Every sum runs in a fixed order so that a run is bitwise reproducible.
#include "laps_internal.hpp"

namespace laps {

// Fixed-order block reduction of NV doubles over a block; the result is
// valid in thread 0.  op: 0 sum, 1 NaN-propagating max.  Inside a wavefront
// an xor butterfly from 32 lanes down to 1, each lane combining (own,
// partner): the partners of 32 and 16 through the lane swaps, those of 8, 4,
// 2, 1 by rotations inside 16-lane rows (a rotation by 16 - K hands lane l the
// value of lane l + K mod 16, which is l ^ K for every lane whose value
// reaches lane 0, as bit K of such a lane is clear at level K).
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&op)[NV], double *sh) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double o = xor_partner<32>(v[k]);
    v[k] = op[k] == 0 ? v[k] + o : nanmax(v[k], o);
    o = xor_partner<16>(v[k]);
    v[k] = op[k] == 0 ? v[k] + o : nanmax(v[k], o);
    o = dpp_f64<0x128>(v[k]);  // row_ror:8
    v[k] = op[k] == 0 ? v[k] + o : nanmax(v[k], o);
    o = dpp_f64<0x12C>(v[k]);  // row_ror:12
    v[k] = op[k] == 0 ? v[k] + o : nanmax(v[k], o);
    o = dpp_f64<0x12E>(v[k]);  // row_ror:14
    v[k] = op[k] == 0 ? v[k] + o : nanmax(v[k], o);
    o = dpp_f64<0x12F>(v[k]);  // row_ror:15
    v[k] = op[k] == 0 ? v[k] + o : nanmax(v[k], o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wave * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = sh[k];
      for (int w = 1; w < nw; ++w) s = op[k] == 0 ? s + sh[w * NV + k] : nanmax(s, sh[w * NV + k]);
      v[k] = s;
    }
  }
  __syncthreads();
}

__global__ void k_hyper_init(CtlArgs c) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  DevHyper *H = c.hyp;
  H->eps = c.eps_fixed > 0.0 ? c.eps_fixed : c.eps0_factor * sqrt((double)c.d);
  H->L = 0.0;
  H->eevpd = H->eevpd_target = H->dtilde = H->max_delta = H->acc_mean = H->sum_var = 0.0;
  H->lo = H->hi = 0.0;
  H->a_star = 0.0;
  H->t = 0;
  H->grads = 1;
  H->n_nonfinite = 0;
  H->ring_count = 0;
  H->ring_pos = 0;
  H->phase = PH_UNADJ;
  H->adapt = 1;
  H->switch_ready = 0;
  H->status = 0;
  H->integ = 0;
  H->have_lo = H->have_hi = 0;
  H->switched = 0;
}

__device__ __forceinline__ double F_bias(double D) {
  const double r = sqrt(D);
  return 4.0 * D * r / ((1.0 + r) * (1.0 + r));
}

// Sum (and NaN count) of a per-chain array over one 256-thread block.
__device__ __forceinline__ void chain_sums(const double *a, int64_t N, double shiftv, int sq, double &sum,
                                           double &bad, double *sh) {
  double s = 0.0, nb = 0.0;
  int64_t m = threadIdx.x;
  const int64_t B = blockDim.x;
  for (; m + 3 * B < N; m += 4 * B) {
    const double a0 = a[m], a1 = a[m + B], a2 = a[m + 2 * B], a3 = a[m + 3 * B];
    const double v0 = a0 - shiftv, v1 = a1 - shiftv, v2 = a2 - shiftv, v3 = a3 - shiftv;
    s += sq ? ((v0 * v0 + v1 * v1) + (v2 * v2 + v3 * v3)) : ((v0 + v1) + (v2 + v3));
    nb += (double)(!isfinite(a0)) + (double)(!isfinite(a1)) + (double)(!isfinite(a2)) + (double)(!isfinite(a3));
  }
  for (; m < N; m += B) {
    const double v = a[m] - shiftv;
    s += sq ? v * v : v;
    if (!isfinite(a[m])) nb += 1.0;
  }
  double v2[2] = {s, nb};
  const int op[2] = {0, 0};
  block_reduce<2>(v2, op, sh);
  sum = v2[0];
  bad = v2[1];
}

// The unadjusted-phase controller (one workgroup of 128 or 256 threads, after the
// statistics pass of the step has written its block scalars).
__device__ void ctl_unadj_body(const CtlArgs &c, double *sh, double &mean_sh) {
  DevHyper *H = c.hyp;
  // The phase, the energy errors and the statistics pass's block scalars are
  // loaded together, and their sums share one block reduction; the phase is
  // tested after it (uniformly, so every thread takes the same path).
  const int phase = H->phase;
  double s = 0.0, q = 0.0, nb = 0.0;
  const int64_t B = blockDim.x, N = c.N;
  int64_t m = threadIdx.x;
  // The thread's first kPre energy errors (m, m + B, ...) and its first block
  // scalars are loaded at once (clamped indices, values past the end unused);
  // the sums below take them in the order of the plain strided loops: groups
  // of four while a whole group remains, then single values.
  constexpr int kPre = 16;
  double pv[kPre];
#pragma unroll
  for (int j = 0; j < kPre; ++j) {
    const int64_t idx = m + j * B;
    pv[j] = c.delta[idx < N ? idx : N - 1];
  }
  const int bf = (int)threadIdx.x < c.nb ? (int)threadIdx.x : c.nb - 1;
  const double pf0 = c.part2[bf * 4 + 0], pf1 = c.part2[bf * 4 + 1], pf2 = c.part2[bf * 4 + 2];
  int j = 0;  // index of m's value among the thread's
#pragma unroll
  for (int g = 0; g < kPre / 4; ++g) {
    if (m + 3 * B < N) {
      const double a0 = pv[4 * g], a1 = pv[4 * g + 1], a2 = pv[4 * g + 2], a3 = pv[4 * g + 3];
      s += (a0 + a1) + (a2 + a3);
      q += (a0 * a0 + a1 * a1) + (a2 * a2 + a3 * a3);
      nb += (double)(!isfinite(a0)) + (double)(!isfinite(a1)) + (double)(!isfinite(a2)) + (double)(!isfinite(a3));
      m += 4 * B;
      j += 4;
    }
  }
  for (; m + 3 * B < N; m += 4 * B) {
    const double a0 = c.delta[m], a1 = c.delta[m + B], a2 = c.delta[m + 2 * B], a3 = c.delta[m + 3 * B];
    s += (a0 + a1) + (a2 + a3);
    q += (a0 * a0 + a1 * a1) + (a2 * a2 + a3 * a3);
    nb += (double)(!isfinite(a0)) + (double)(!isfinite(a1)) + (double)(!isfinite(a2)) + (double)(!isfinite(a3));
    j += 4;
  }
  // at most three values remain (m + 3 B >= N)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (m < N) {
      double v = 0.0;
      if (j < kPre) {
#pragma unroll
        for (int i = 0; i < kPre; ++i) v = (i == j) ? pv[i] : v;
      } else {
        v = c.delta[m];
      }
      s += v;
      q += v * v;
      if (!isfinite(v)) nb += 1.0;
      m += B;
      ++j;
    }
  }
  double p3[3] = {0.0, 0.0, -INFINITY};
  if ((int)threadIdx.x < c.nb) {
    p3[0] += pf0;
    p3[1] += pf1;
    p3[2] = nanmax(p3[2], pf2);
  }
  for (int b = threadIdx.x + blockDim.x; b < c.nb; b += blockDim.x) {
    p3[0] += c.part2[b * 4 + 0];
    p3[1] += c.part2[b * 4 + 1];
    p3[2] = nanmax(p3[2], c.part2[b * 4 + 2]);
  }
  double pr = 0.0;  // full-rank loss: the probe blocks' squared norms
  if (c.probes > 0)
    for (int b = threadIdx.x; b < c.nbh; b += blockDim.x) pr += c.pPart[b];
  double v6[7] = {s, q, nb, p3[0], p3[1], p3[2], pr};
  const int op6[7] = {0, 0, 0, 0, 0, 1, 0};
  block_reduce<7>(v6, op6, sh);
  if (phase != PH_UNADJ) return;
  const double sum = v6[0], bad = v6[2];
  double sq = v6[1];
  p3[0] = v6[3];
  p3[1] = v6[4];
  p3[2] = v6[5];
  if (c.eevpd_mode != 1) {
    // variance: a second pass about the mean
    if (threadIdx.x == 0) mean_sh = sum / (double)c.N;
    __syncthreads();
    double sum2, bad2;
    chain_sums(c.delta, c.N, mean_sh, 1, sum2, bad2, sh);
    sq = sum2;
  }
  if (threadIdx.x != 0) return;
  const double sD = p3[0], sV = p3[1], mx = p3[2];
  H->dtilde = c.probes > 0 ? v6[6] / ((double)c.probes * (double)c.d) : sD / (double)c.d;
  H->eevpd = sq / (double)c.N / (double)c.d;
  H->n_nonfinite = (int64_t)bad;
  if (bad > 0.0) H->status |= ST_NONFINITE;
  H->eevpd_target = F_bias(c.C * H->dtilde);
  const double ratio = H->eevpd_target / H->eevpd;
  if (c.eps_fixed > 0.0) {
    // fixed step size: the update is skipped, the diagnostics still computed
  } else if (isfinite(ratio) && ratio > 0.0) {
    H->eps *= pow(ratio, 1.0 / 6.0);
  } else {
    H->status |= ST_EPS_KEPT;
  }
  H->sum_var = sV;
  H->L = c.alpha * sqrt(sV);
  H->ring_pos = (H->ring_pos + 1) % c.Tw;
  if (H->ring_count < c.Tw) H->ring_count += 1;
  if (H->ring_count == c.Tw) {
    H->max_delta = mx;
    H->switch_ready = (mx < c.switch_tol) ? 1 : 0;
  } else {
    H->max_delta = INFINITY;
    H->switch_ready = 0;
  }
  H->t += 1;
  H->grads += 1;
  if ((c.switch_policy == 0 && H->switch_ready) || H->t >= c.max_unadj) H->phase = PH_SWITCH_PENDING;
}

// DIMS dimensions per THREADS-thread block (8 up to d = 1024, else 32): row
// group rg (0 .. THREADS/DIMS - 1) of dimension column dl sums partial rows rg,
// rg + groups, ...; the group sums are combined first inside each wavefront
// by xor butterflies over the group bits, then over the wavefronts in order
// through LDS, so the result does not depend on timing.  The moving window is
// reduced the same way over its slots.
template <int DIMS>
__device__ __forceinline__ void fin_combine(double (&v)[4], double *sh, int dl, int rg) {
  // xor levels DIMS .. 32 (own + partner): 8 by a rotation by 8 inside 16-lane
  // rows (exactly lane l ^ 8), 16 and 32 through the lane swaps
  if (DIMS <= 8) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += dpp_f64<0x128>(v[k]);
  }
  if (DIMS <= 16) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = xor_pair_sum<16>(v[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = xor_pair_sum<32>(v[k]);
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) < DIMS)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[(wave * 4 + k) * DIMS + dl] = v[k];
  __syncthreads();
  if (rg == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[(w * 4 + k) * DIMS + dl];
      v[k] = s;
    }
  }
  __syncthreads();
}

template <int DIMS, int THREADS>
__global__ void __launch_bounds__(THREADS) k_finalize(CtlArgs c, int mode) {
  constexpr int kFinDims = DIMS, kFinGroups = THREADS / DIMS;
  const DevHyper *H = c.hyp;
  if (mode == FIN_UNADJ && H->phase != PH_UNADJ) return;
  __shared__ double sh[16 * 4 * kFinDims];
  __shared__ double bsh[16 * 4];
  __shared__ double mu_sh[kFinDims];
  const int dl = threadIdx.x % kFinDims, rg = threadIdx.x / kFinDims;
  const int64_t i = (int64_t)blockIdx.x * kFinDims + dl;
  const int64_t d = c.d, ld = c.ld;
  const bool act = i < d;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (act) {
    int gI = rg;
    for (; gI + 3 * kFinGroups < c.G; gI += 4 * kFinGroups) {
      const double *P0 = c.partials + (size_t)gI * 4 * ld + i;
      const double *P1 = P0 + (size_t)kFinGroups * 4 * ld;
      const double *P2 = P1 + (size_t)kFinGroups * 4 * ld;
      const double *P3 = P2 + (size_t)kFinGroups * 4 * ld;
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += ((P0[k * ld] + P1[k * ld]) + (P2[k * ld] + P3[k * ld]));
    }
    for (; gI < c.G; gI += kFinGroups) {
      const double *P = c.partials + (size_t)gI * 4 * ld + i;
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += P[k * ld];
    }
  }
  fin_combine<DIMS>(v, sh, dl, rg);
  double Dp = 0.0, vp = 0.0, wd = -INFINITY;
  const bool full = mode == FIN_UNADJ && (H->ring_count + 1 >= c.Tw);
  if (rg == 0 && act) {
    const double invN = 1.0 / (double)c.N;
    const double K = c.shiftK[i];
    const double m1 = v[0] * invN;
    const double mean = K + m1;
    const double var = v[1] * invN - m1 * m1;
    const double m2 = var + mean * mean;
    const double V = -(v[2] * invN - m1 * (v[3] * invN));
    c.mean[i] = mean;
    c.var[i] = var;
    c.m2[i] = m2;
    c.Vii[i] = V;
    c.shiftK[i] = mean;
    Dp = (1.0 - V) * (1.0 - V);
    vp = var;
    if (mode == FIN_UNADJ) c.ring[H->ring_pos * ld + i] = m2;
    mu_sh[dl] = m2;
  }
  if (full) {
    __syncthreads();  // the new window entry (and the shift) is visible to the whole block
    // mean and sample variance over the window slots in one pass, about the
    // newest entry K: mu = K + s1 / Tw, var = (s2 - s1^2 / Tw) / (Tw - 1)
    const double K = mu_sh[dl];
    double w1[4] = {0.0, 0.0, 0.0, 0.0};
    if (act) {
      int64_t k = rg;
      for (; k + 7 * kFinGroups < c.Tw; k += 8 * kFinGroups) {
        double r[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) r[j] = c.ring[(k + j * kFinGroups) * ld + i];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const double e = r[j] - K;
          w1[0] += e;
          w1[1] += e * e;
        }
      }
      for (; k < c.Tw; k += kFinGroups) {
        const double e = c.ring[k * ld + i] - K;
        w1[0] += e;
        w1[1] += e * e;
      }
    }
    fin_combine<DIMS>(w1, sh, dl, rg);
    if (rg == 0 && act) {
      const double Tw = (double)c.Tw;
      const double mu = K + w1[0] / Tw;
      const double vw = (w1[1] - w1[0] * (w1[0] / Tw)) / (Tw - 1.0);
      wd = sqrt(vw > 0.0 ? vw : 0.0) / mu;
      c.wdelta[i] = wd;
    }
  }
  double r3[3] = {Dp, vp, wd};
  const int op[3] = {0, 0, 1};
  block_reduce<3>(r3, op, bsh);
  if (threadIdx.x == 0) {
    c.part2[blockIdx.x * 4 + 0] = r3[0];
    c.part2[blockIdx.x * 4 + 1] = r3[1];
    c.part2[blockIdx.x * 4 + 2] = r3[2];
  }
}

__global__ void __launch_bounds__(256) k_ctl_init(CtlArgs c) {
  __shared__ double sh[4 * 4];
  (void)sh;
  if (threadIdx.x != 0) return;
  double sv = 0.0;
  for (int b = 0; b < c.nb; ++b) sv += c.part2[b * 4 + 1];
  DevHyper *H = c.hyp;
  H->sum_var = sv;
  H->L = c.alpha * sqrt(sv);
}

__global__ void __launch_bounds__(256) k_ctl_unadj(CtlArgs c) {
  __shared__ double sh[16 * 8];
  __shared__ double mean_sh;
  ctl_unadj_body(c, sh, mean_sh);
}

// One thread per dimension; block 0 thread 0 also sets the phase block.
__global__ void __launch_bounds__(256) k_switch(CtlArgs c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  DevHyper *H = c.hyp;
  if (i < c.ld) {
    double s = 1.0;
    if (i < c.d) {
      s = sqrt(c.var[i]);
      if (!(s > 0.0) || !isfinite(s)) {
        s = 1.0;
        atomicOr(&H->status, ST_SIGMA_FIX);
      }
    } else {
      s = 0.0;
    }
    if (c.sigma_double)
      static_cast<double *>(c.sigma)[i] = s;
    else
      static_cast<float *>(c.sigma)[i] = (float)s;
  }
  // once per run: a repeated switch (a replayed graph chunk) only rewrites
  // the same preconditioner and leaves the bisection state alone
  if (i == 0 && !H->switched) {
    H->phase = PH_ADJ;
    H->integ = c.integ;
    H->a_star = c.acc_target > 0.0 ? c.acc_target : (c.integ == 2 ? 0.9 : 0.7);
    H->adapt = 1;
    H->have_lo = 0;
    H->have_hi = 0;
    H->switched = 1;
  }
}

__global__ void __launch_bounds__(256) k_ctl_adj(CtlArgs c) {
  DevHyper *H = c.hyp;
  if (H->phase != PH_ADJ || H->t >= c.max_total) return;
  __shared__ double sh[16 * 4];
  double sa, bad0;
  chain_sums(c.acc, c.N, 0.0, 0, sa, bad0, sh);
  double sd, bad;
  chain_sums(c.delta, c.N, 0.0, 0, sd, bad, sh);
  if (threadIdx.x != 0) return;
  const double abar = sa / (double)c.N;
  H->acc_mean = abar;
  H->n_nonfinite = (int64_t)bad;
  if (bad > 0.0) H->status |= ST_NONFINITE;
  H->adapt = H->adapt && (fabs(abar - H->a_star) > c.acc_tol);
  if (H->adapt) {
    if (abar > H->a_star) {
      H->lo = H->eps;
      H->have_lo = 1;
      H->eps = H->have_hi ? 0.5 * (H->lo + H->hi) : 2.0 * H->eps;
    } else {
      H->hi = H->eps;
      H->have_hi = 1;
      H->eps = H->have_lo ? 0.5 * (H->lo + H->hi) : 0.5 * H->eps;
    }
  }
  const int gps = c.integ == 2 ? 5 : (c.integ == 1 ? 2 : 1);
  H->t += c.n_traj;
  H->grads += (int64_t)c.n_traj * gps;
}

hipError_t launch_hyper_init(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_hyper_init, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}
// Plain fill, used instead of a memset node so that the restart sequence can
// be recorded in a graph.
__global__ void k_fill(double *p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
// ---------------------------------------------------------------------------
// Full-rank equipartition loss by Hutchinson's estimator (section
// "Equipartition condition", full-rank paragraph): with Rademacher probes z_p
// of this step and V_ij = -E[(x_i - xbar_i) g_j] from ensemble averages,
//   D~ = (1/(P d)) sum_p |z_p + (1/N) sum_m (x_m - xbar)(g_m . z_p)|^2.
// Probe entry i of z_p is 1 - 2b, b = bit i mod 64 of word (i mod 256) / 64 of
// Philox block (p, i / 256, t, TAG_PROBE); probes are regenerated where they
// are used (a lane computes the block of its own probe), never stored.
// Three passes, every sum in a fixed order:
//   k_probe_dots:    S = G Z, s[m][p] = g_m . z_p, on the FP64 matrix cores
//                    (one wavefront per 16 chains x 16 probes, 4 dims per step)
//   k_probe_project: W_c = S_c^T (X_c - xbar), w_c[p][i] = sum over chunk c of
//                    (x_mi - xbar_i) s[m][p], on the FP64 matrix cores (one
//                    wavefront per 16 probes x 16 dims of a kProbeChunk-chain
//                    chunk)
//   k_probe_norms:   per block, sum of (z_pi + (1/N) sum_c w_c[p][i])^2
// and the controller adds the block sums in order.  Lane layout of
// v_mfma_f64_16x16x4_f64 (A 16 x 4, B 4 x 16, D 16 x 16): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[l / 16 + 4 i][l % 16].
// ---------------------------------------------------------------------------
typedef double pf64x4 __attribute__((ext_vector_type(4)));

// The four Philox words of block blk (dims 256 blk .. 256 blk + 255) of probe p
// at step t (all zero for a probe past the end), and entry i of that block.
__device__ __forceinline__ void probe_words(const CtlArgs &c, int64_t p, int64_t blk, uint64_t t, uint64_t (&w)[4]) {
  w[0] = (uint64_t)p;
  w[1] = (uint64_t)blk;
  w[2] = t;
  w[3] = (uint64_t)TAG_PROBE;
  philox4x64_10(w, c.seed, 0);
}
__device__ __forceinline__ double probe_entry(const uint64_t (&w)[4], int64_t i) {
  return ((w[(i & 255) >> 6] >> (i & 63)) & 1u) ? -1.0 : 1.0;
}

template <class Real>
__global__ void __launch_bounds__(256) k_probe_dots(CtlArgs c) {
  const DevHyper *H = c.hyp;
  if (H->phase != PH_UNADJ) return;
  const int lane = threadIdx.x & 63;
  const int64_t PT = (c.probes + 15) / 16;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ((c.N + 15) / 16) * PT) return;
  const int64_t m0 = (tile / PT) * 16, p0 = (tile % PT) * 16;
  const int lo = lane & 15, hi = lane >> 4;
  const Real *g = static_cast<const Real *>(c.g);
  const int64_t ma = m0 + lo, mc = ma < c.N ? ma : c.N - 1;  // A: g[ma][k0 + hi]
  pf64x4 acc = pf64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t pb = p0 + lo;  // B: z[e][pb], from the words of the lane's own probe
  uint64_t w[4] = {0, 0, 0, 0};
  // 16 K-steps (64 dims) at a time: their operands are loaded before the first product
  for (int64_t kb = 0; kb < c.d; kb += 64) {
    if ((kb & 255) == 0) probe_words(c, pb, kb >> 8, (uint64_t)H->t, w);
    // Indices are clamped to entries that exist and the bounds are applied as
    // 0 / 1 factors, so that every load is used unconditionally: the compiler
    // then issues all of them before the first wait instead of sinking each
    // into a branch of its own that waits for it.
    double av[16], bv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t e = kb + 4 * j + hi;
      const double gv = (double)g[mc * c.ld + (e < c.d ? e : c.d - 1)];
      av[j] = gv * ((ma < c.N && e < c.d) ? 1.0 : 0.0);
      bv[j] = (pb < c.probes && e < c.d) ? probe_entry(w, e) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[j], acc, 0, 0, 0);
  }
  const int64_t p = p0 + lo;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + hi + 4 * i;
    if (m < c.N && p < c.probes) c.pS[m * c.probes + p] = acc[i];
  }
}

template <class Real>
__global__ void __launch_bounds__(256) k_probe_project(CtlArgs c) {
  const DevHyper *H = c.hyp;
  if (H->phase != PH_UNADJ) return;
  const int lane = threadIdx.x & 63;
  const int64_t P = c.probes, d = c.d;
  const int64_t PT = (P + 15) / 16, DTl = (d + 15) / 16;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= PT * DTl) return;
  const int64_t p0 = (tile / DTl) * 16, i0 = (tile % DTl) * 16;
  const int lo = lane & 15, hi = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.y * kProbeChunk;
  const int64_t m1 = (m0 + kProbeChunk < c.N) ? m0 + kProbeChunk : c.N;
  const Real *x = static_cast<const Real *>(c.x);
  const int64_t pa = p0 + lo, ib = i0 + lo;     // A: s[m][pa] (row pa, column m), B: x[m][ib] - xbar[ib]
  const double xb = ib < d ? c.mean[ib] : 0.0;
  pf64x4 acc = pf64x4{0.0, 0.0, 0.0, 0.0};
  // the chunk's kProbeChunk / 4 K-steps: every operand is loaded before the first product
  // (indices clamped and bounds applied as factors, as in k_probe_dots, so that
  // all the loads are in flight together)
  constexpr int KS = kProbeChunk / 4;
  const int64_t pc = pa < P ? pa : P - 1, ic = ib < d ? ib : d - 1;
  double av[KS], bv[KS];
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    const int64_t m = m0 + 4 * j + hi;
    const bool ok = m < m1;
    const int64_t mcl = ok ? m : m1 - 1;
    const double sv = c.pS[mcl * P + pc];
    const double xv = (double)x[mcl * c.ld + ic];
    av[j] = sv * ((ok && pa < P) ? 1.0 : 0.0);
    bv[j] = (xv - xb) * ((ok && ib < d) ? 1.0 : 0.0);
  }
#pragma unroll
  for (int j = 0; j < KS; ++j) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[j], acc, 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t pp = p0 + hi + 4 * i;
    if (pp < P && ib < d) c.pW[((int64_t)blockIdx.y * P + pp) * d + ib] = acc[i];
  }
}

__global__ void __launch_bounds__(256) k_probe_norms(CtlArgs c) {
  const DevHyper *H = c.hyp;
  if (H->phase != PH_UNADJ) return;
  __shared__ double sh[4 * 1];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t P = c.probes, d = c.d;
  double v = 0.0;
  if (idx < d * P) {
    const int64_t p = idx / d, i = idx - p * d;
    double w = 0.0;
#pragma unroll 8
    for (int ch = 0; ch < c.NC; ++ch) w += c.pW[((int64_t)ch * P + p) * d + i];
    uint64_t wz[4];
    probe_words(c, p, i >> 8, (uint64_t)H->t, wz);
    const double z = probe_entry(wz, i);
    const double r = z + w / (double)c.N;
    v = r * r;
  }
  double v1[1] = {v};
  const int op[1] = {0};
  block_reduce<1>(v1, op, sh);
  if (threadIdx.x == 0) c.pPart[blockIdx.x] = v1[0];
}

hipError_t launch_probes(const CtlArgs &c, hipStream_t s) {
  if (c.probes <= 0) return hipSuccess;
  const int64_t PT = (c.probes + 15) / 16;
  const int64_t t1 = ((c.N + 15) / 16) * PT, t2 = PT * ((c.d + 15) / 16);  // 16 x 16 tiles, one per wavefront
  const dim3 g1((unsigned)((t1 + 3) / 4)), g2((unsigned)((t2 + 3) / 4), (unsigned)c.NC);
  if (c.sigma_double) {
    hipLaunchKernelGGL(k_probe_dots<double>, g1, dim3(256), 0, s, c);
    hipLaunchKernelGGL(k_probe_project<double>, g2, dim3(256), 0, s, c);
  } else {
    hipLaunchKernelGGL(k_probe_dots<float>, g1, dim3(256), 0, s, c);
    hipLaunchKernelGGL(k_probe_project<float>, g2, dim3(256), 0, s, c);
  }
  hipLaunchKernelGGL(k_probe_norms, dim3((unsigned)c.nbh), dim3(256), 0, s, c);
  return hipGetLastError();
}

// Launch shapes of the scalar controllers and the statistics finalisation,
// from a sweep on the MI355X: one workgroup of 128 threads (N <= 2048) or 256
// for the controllers (against 1024: 9.3 -> 4.8 us at N = 1024, 9.6 -> 6.5 us
// at N = 4096), 512 threads per finalisation workgroup (9.5 -> 7.6 us at
// d = 100 and G = 64 partial rows, 10.8 -> 10.0 us at G = 256).
static unsigned ctl_threads(int64_t N) { return N <= 2048 ? 128u : 256u; }

hipError_t launch_ctl_unadj(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_unadj, dim3(1), dim3(ctl_threads(c.N)), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_finalize(const CtlArgs &c, int mode, hipStream_t s) {
  if (fin_dims(c.d) == 8)
    hipLaunchKernelGGL((k_finalize<8, 512>), dim3(c.nb), dim3(512), 0, s, c, mode);
  else
    hipLaunchKernelGGL((k_finalize<32, 512>), dim3(c.nb), dim3(512), 0, s, c, mode);
  return hipGetLastError();
}
hipError_t launch_ctl_init(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(256), 0, s, c);
  return hipGetLastError();
}
hipError_t launch_switch(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_switch, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, s, c);
  return hipGetLastError();
}
hipError_t launch_ctl_adj(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_adj, dim3(1), dim3(ctl_threads(c.N)), 0, s, c);
  return hipGetLastError();
}

}  // namespace laps
