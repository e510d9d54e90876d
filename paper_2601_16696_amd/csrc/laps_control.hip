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

// Fixed-order block reduction of NV doubles over a 256-thread block; the
// result is valid in thread 0.  op: 0 sum, 1 NaN-propagating max.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&op)[NV], double *sh) {
#pragma unroll
  for (int msk = 32; msk >= 1; msk >>= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double o = __shfl_xor(v[k], msk);
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
  H->eps = c.eps0_factor * sqrt((double)c.d);
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

// One thread per dimension.
__global__ void __launch_bounds__(256) k_finalize(CtlArgs c, int mode) {
  const DevHyper *H = c.hyp;
  if (mode == FIN_UNADJ && H->phase != PH_UNADJ) return;
  __shared__ double sh[4 * 4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t d = c.d, ld = c.ld;
  double Dp = 0.0, vp = 0.0, wd = -INFINITY;
  if (i < d) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    for (int gI = 0; gI < c.G; ++gI) {
      const double *P = c.partials + (size_t)gI * 4 * ld;
      s1 += P[i];
      s2 += P[ld + i];
      s3 += P[2 * ld + i];
      s4 += P[3 * ld + i];
    }
    const double invN = 1.0 / (double)c.N;
    const double K = c.shiftK[i];
    const double m1 = s1 * invN;
    const double mean = K + m1;
    const double var = s2 * invN - m1 * m1;
    const double m2 = var + mean * mean;
    const double V = -(s3 * invN - m1 * (s4 * invN));
    c.mean[i] = mean;
    c.var[i] = var;
    c.m2[i] = m2;
    c.Vii[i] = V;
    c.shiftK[i] = mean;
    Dp = (1.0 - V) * (1.0 - V);
    vp = var;
    if (mode == FIN_UNADJ) {
      const int64_t pos = H->ring_pos;
      c.ring[pos * ld + i] = m2;
      const int64_t cnt = H->ring_count + 1 < c.Tw ? H->ring_count + 1 : c.Tw;
      if (cnt == c.Tw) {
        // two-pass mean and sample variance over the window (slot order)
        double mu = 0.0;
        for (int64_t k = 0; k < c.Tw; ++k) mu += c.ring[k * ld + i];
        mu /= (double)c.Tw;
        double ss = 0.0;
        for (int64_t k = 0; k < c.Tw; ++k) {
          const double e = c.ring[k * ld + i] - mu;
          ss += e * e;
        }
        wd = sqrt(ss / (double)(c.Tw - 1)) / mu;
        c.wdelta[i] = wd;
      }
    }
  }
  double v[3] = {Dp, vp, wd};
  const int op[3] = {0, 0, 1};
  block_reduce<3>(v, op, sh);
  if (threadIdx.x == 0) {
    c.part2[blockIdx.x * 4 + 0] = v[0];
    c.part2[blockIdx.x * 4 + 1] = v[1];
    c.part2[blockIdx.x * 4 + 2] = v[2];
  }
}

__device__ __forceinline__ double F_bias(double D) {
  const double r = sqrt(D);
  return 4.0 * D * r / ((1.0 + r) * (1.0 + r));
}

// Sum (and NaN count) of a per-chain array over one 256-thread block.
__device__ __forceinline__ void chain_sums(const double *a, int64_t N, double shiftv, int sq, double &sum,
                                           double &bad, double *sh) {
  double s = 0.0, nb = 0.0;
  for (int64_t m = threadIdx.x; m < N; m += blockDim.x) {
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
  DevHyper *H = c.hyp;
  if (H->phase != PH_UNADJ) return;
  __shared__ double sh[4 * 4];
  __shared__ double mean_sh;
  double sum, bad;
  chain_sums(c.delta, c.N, 0.0, 0, sum, bad, sh);
  if (threadIdx.x == 0) mean_sh = sum / (double)c.N;
  __syncthreads();
  const double mu = mean_sh;
  double sq, bad2;
  chain_sums(c.delta, c.N, c.eevpd_mode == 1 ? 0.0 : mu, 1, sq, bad2, sh);
  if (threadIdx.x != 0) return;
  double sD = 0.0, sV = 0.0, mx = -INFINITY;
  for (int b = 0; b < c.nb; ++b) {
    sD += c.part2[b * 4 + 0];
    sV += c.part2[b * 4 + 1];
    mx = nanmax(mx, c.part2[b * 4 + 2]);
  }
  H->dtilde = sD / (double)c.d;
  H->eevpd = sq / (double)c.N / (double)c.d;
  H->n_nonfinite = (int64_t)bad;
  if (bad > 0.0) H->status |= ST_NONFINITE;
  H->eevpd_target = F_bias(c.C * H->dtilde);
  const double ratio = H->eevpd_target / H->eevpd;
  if (isfinite(ratio) && ratio > 0.0)
    H->eps *= pow(ratio, 1.0 / 6.0);
  else
    H->status |= ST_EPS_KEPT;
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
  if (i == 0) {
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
  __shared__ double sh[4 * 4];
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
hipError_t launch_finalize(const CtlArgs &c, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(c.nb), dim3(256), 0, s, c, mode);
  return hipGetLastError();
}
hipError_t launch_ctl_init(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(256), 0, s, c);
  return hipGetLastError();
}
hipError_t launch_ctl_unadj(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_unadj, dim3(1), dim3(256), 0, s, c);
  return hipGetLastError();
}
hipError_t launch_switch(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_switch, dim3((unsigned)((c.ld + 255) / 256)), dim3(256), 0, s, c);
  return hipGetLastError();
}
hipError_t launch_ctl_adj(const CtlArgs &c, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_adj, dim3(1), dim3(256), 0, s, c);
  return hipGetLastError();
}

}  // namespace laps
