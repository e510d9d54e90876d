// Device-side building blocks of the LAPS hot path for gfx950: the
// device-resident hyperparameter block, the counter-based random numbers,
// team reductions and the scalar parts of the integrator maps.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace laps {

// Hyperparameters and diagnostics, resident in device memory.  Only the
// single-workgroup controller kernels write it; every step kernel reads it at
// launch, so a captured sequence of steps needs no host round trip.
struct DevHyper {
  double eps, L, eevpd, eevpd_target, dtilde, max_delta, acc_mean, sum_var, lo, hi, a_star;
  int64_t t, grads, n_nonfinite, ring_count, ring_pos;
  int32_t phase, adapt, switch_ready, status, integ, have_lo, have_hi, switched;
};

enum { PH_UNADJ = 0, PH_SWITCH_PENDING = 1, PH_ADJ = 2 };
enum { TAG_O_FIRST = 1, TAG_O_SECOND = 2, TAG_FULL_REFRESH = 3, TAG_MH = 4, TAG_INIT_DIR = 5, TAG_PROBE = 6 };
enum { ST_NONFINITE = 1, ST_EPS_KEPT = 2, ST_SIGMA_FIX = 4 };

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 64x64
// multiplies with Weyl-sequence key bumps between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

// Eight standard normals for dims 8*oct .. 8*oct+7 of chain m: word k of the
// block gives (U_a, U_b) = ((hi32 + 1/2) 2^-32, (lo32 + 1/2) 2^-32) and the
// Box-Muller pair r cos(2 pi U_b), r sin(2 pi U_b), r = sqrt(-2 ln U_a).
template <class Real>
__device__ __forceinline__ void normals8(uint64_t seed, uint64_t m, uint64_t oct, uint64_t t, uint32_t tag,
                                         uint32_t substep, Real (&z)[8]);

template <>
__device__ __forceinline__ void normals8<double>(uint64_t seed, uint64_t m, uint64_t oct, uint64_t t, uint32_t tag,
                                                 uint32_t substep, double (&z)[8]) {
  uint64_t c[4] = {m, oct, t, (uint64_t)tag | ((uint64_t)substep << 8)};
  philox4x64_10(c, seed, 0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double ua = ((double)(uint32_t)(c[k] >> 32) + 0.5) * 2.3283064365386963e-10;
    const double ub = ((double)(uint32_t)c[k] + 0.5) * 2.3283064365386963e-10;
    const double r = sqrt(-2.0 * log(ua));
    double s, co;
    sincospi(2.0 * ub, &s, &co);
    z[2 * k] = r * co;
    z[2 * k + 1] = r * s;
  }
}

// FP32 state: the same uniforms, with the hardware base-2 logarithm, square
// root and the sine/cosine of an angle given in revolutions (U_b is already a
// fraction of a turn, so no range reduction is needed).  Each of these has a
// relative (log2, sqrt) or absolute (sin, cos) error near 1e-7 on (0, 1], so
// the normals carry an absolute error of order 1e-6 against FP64.
template <>
__device__ __forceinline__ void normals8<float>(uint64_t seed, uint64_t m, uint64_t oct, uint64_t t, uint32_t tag,
                                                uint32_t substep, float (&z)[8]) {
  uint64_t c[4] = {m, oct, t, (uint64_t)tag | ((uint64_t)substep << 8)};
  philox4x64_10(c, seed, 0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float ua = fmaf((float)(uint32_t)(c[k] >> 32), 2.3283064365386963e-10f, 1.1641532182693481e-10f);
    const float ub = fmaf((float)(uint32_t)c[k], 2.3283064365386963e-10f, 1.1641532182693481e-10f);
    // -2 ln U = -2 ln(2) log2(U)
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
    z[2 * k] = r * __builtin_amdgcn_cosf(ub);
    z[2 * k + 1] = r * __builtin_amdgcn_sinf(ub);
  }
}

// Metropolis uniform of chain m for the transition starting at step t: the
// 53 high bits of word 0 of block (m, 0, t, TAG_MH), offset by half a unit.
__device__ __forceinline__ double mh_uniform(uint64_t seed, uint64_t m, uint64_t t) {
  uint64_t c[4] = {m, 0, t, (uint64_t)TAG_MH};
  philox4x64_10(c, seed, 0);
  return ((double)(c[0] >> 11) + 0.5) * 1.1102230246251565e-16;
}

// ---------------------------------------------------------------------------
// Team reductions.  A team of T lanes owns one chain: T <= 64 is an aligned
// lane group inside a wavefront (butterflies, no barrier); T > 64 is the
// whole workgroup (butterfly per wavefront, then a fixed-order sum over
// wavefronts through LDS, double-buffered so one barrier suffices).  Every
// lane ends with the identical value, and the order of additions is fixed.
// ---------------------------------------------------------------------------
constexpr int kRedSlots = 16 * 8;  // doubles per buffer: 16 wavefronts x 8 values

// A double moved between lanes by a DPP row permutation (CTRL: 0x00-0xFF quad
// permutation, 0x140 mirror of the 16-lane row, 0x141 mirror of each 8-lane half).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// own + partner for the lane partner l ^ MSK (MSK = 16 or 32) with the gfx950
// lane swaps instead of an LDS permute: v_permlane16_swap(v, v) gives every
// lane the value of the even 16-lane row of its pair in the first result and
// of the odd row in the second (v_permlane32_swap the same for the two 32-lane
// halves), so first + second is the pair's sum in every lane, equal to
// own + partner (addition is commutative).
template <int MSK>
__device__ __forceinline__ void xor_pair(double v, double &e, double &o) {
  static_assert(MSK == 16 || MSK == 32, "row or half swap");
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const auto l = MSK == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, true, false)
                           : __builtin_amdgcn_permlane32_swap(lo, lo, true, false);
  const auto h = MSK == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, true, false)
                           : __builtin_amdgcn_permlane32_swap(hi, hi, true, false);
  e = __longlong_as_double((long long)(((uint64_t)h[0] << 32) | l[0]));
  o = __longlong_as_double((long long)(((uint64_t)h[1] << 32) | l[1]));
}
template <int MSK>
__device__ __forceinline__ double xor_pair_sum(double v) {
  double e, o;
  xor_pair<MSK>(v, e, o);
  return e + o;
}
// The value of lane l ^ MSK itself (lane swaps and a select by the lane's bit).
template <int MSK>
__device__ __forceinline__ double xor_partner(double v) {
  double e, o;
  xor_pair<MSK>(v, e, o);
  return (threadIdx.x & MSK) ? e : o;
}

// Sum over each aligned group of T lanes (T a power of two up to 64), the same
// value in every lane of a group.  Masks of 16 and 32 are xor shuffles; below
// 16 the partners are the DPP row mirror (i <-> 15 - i), the half-row mirror
// (i <-> 7 - i) and the quad swaps, which pair lanes as the xor butterfly does
// at the granularity reached so far, without a trip through LDS.  Every pair
// is added as (own + partner), so both partners hold identical sums.
template <int NV>
__device__ __forceinline__ void group_sum(double (&v)[NV], int T) {
  // (xor_pair_sum's lane swaps give these two levels the same sums, but in the
  // FP64 stochastic-volatility step kernel the compiler then contracted one
  // multiply-add elsewhere differently, so those runs changed at the bit
  // level; kept as shuffles)
  for (int msk = T >> 1; msk >= 16; msk >>= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], msk);
  }
  if (T >= 16) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += dpp_f64<0x140>(v[k]);
  }
  if (T >= 8) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += dpp_f64<0x141>(v[k]);
  }
  if (T >= 4) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += dpp_f64<0x4E>(v[k]);  // quad lanes (2, 3, 0, 1)
  }
  if (T >= 2) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += dpp_f64<0xB1>(v[k]);  // quad lanes (1, 0, 3, 2)
  }
}

template <int NV>
__device__ __forceinline__ void team_sum(double (&v)[NV], int T, double *red, int &slot) {
  if (T <= 64) {
    group_sum<NV>(v, T);
    return;
  }
  group_sum<NV>(v, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = T >> 6;
  const int w0 = (wave / nw) * nw;  // first wavefront of this lane's team
  double *buf = red + slot * kRedSlots;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) buf[wave * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += buf[(w0 + w) * NV + k];
    v[k] = s;
  }
  slot ^= 1;
}

// NaN-propagating maximum (a NaN fluctuation means "not settled").
__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

// ---------------------------------------------------------------------------
// Velocity update B_h (closed-form solution of the Riccati flow at fixed x):
// with n = |g~|, delta = h n / (d-1), c = e.u,
//   u' = (u + (sinh delta + c (cosh delta - 1)) e) / (cosh delta + c sinh delta)
//   dK = (d-1) log(cosh delta + c sinh delta).
// Returned as u' = A u + Bg g~ so the per-element update is one fma.
// Below |delta| = 20 both hyperbolic terms come from one expm1 (no
// cancellation for small delta); beyond it the quotient is divided through by
// cosh delta (tanh/sech form) to avoid overflow.
// ---------------------------------------------------------------------------
struct BMap {
  double A, Bg, dK;
};

__device__ __forceinline__ BMap b_map(double gg, double gu, double h, double dm1) {
  BMap r;
  if (gg == 0.0) {
    r.A = 1.0;
    r.Bg = 0.0;
    r.dK = 0.0;
    return r;
  }
  const double n = sqrt(gg);
  const double in = 1.0 / n;
  const double delta = h * n / dm1;
  const double c = gu * in;
  const double ad = fabs(delta);
  if (ad < 20.0) {
    // one expm1 of |delta| gives both hyperbolic terms:
    // cosh - 1 = E^2 / (2 (E + 1)), sinh = E - (cosh - 1), E = e^|delta| - 1
    const double E = expm1(ad);
    const double chm1 = 0.5 * E * E / (E + 1.0);
    const double sh = copysign(E - chm1, delta);
    const double Dm1 = chm1 + c * sh;
    const double invD = 1.0 / (1.0 + Dm1);
    r.A = invD;
    r.Bg = (sh + c * chm1) * in * invD;
    r.dK = dm1 * log1p(Dm1);
  } else {
    const double e2 = exp(-2.0 * ad);
    const double tau = copysign((1.0 - e2) / (1.0 + e2), delta);
    const double sech = 2.0 * exp(-ad) / (1.0 + e2);
    const double Dh = 1.0 + c * tau;
    r.A = sech / Dh;
    r.Bg = (tau + c * (1.0 - sech)) * in / Dh;
    r.dK = dm1 * (ad + log1p(e2) - 0.69314718055994531 + log(Dh));
  }
  return r;
}

// The same map with the per-chain scalars in float, for the FP32 state: the
// coefficients only multiply float vectors (reciprocals from the hardware
// 1-ulp instruction), and the energy term is returned as a double for the FP64
// energy accumulation.
__device__ __forceinline__ BMap b_map_f(double gg, double gu, double h, double dm1) {
  BMap r;
  if (gg == 0.0) {
    r.A = 1.0;
    r.Bg = 0.0;
    r.dK = 0.0;
    return r;
  }
  const float n = __builtin_amdgcn_sqrtf((float)gg);
  const float in = __builtin_amdgcn_rcpf(n);
  const float delta = (float)(h / dm1) * n;
  const float c = (float)gu * in;
  const float ad = fabsf(delta);
  if (ad < 20.0f) {
    const float E = expm1f(ad);
    const float chm1 = 0.5f * E * E * __builtin_amdgcn_rcpf(E + 1.0f);
    const float sh = copysignf(E - chm1, delta);
    const float Dm1 = chm1 + c * sh;
    const float invD = __builtin_amdgcn_rcpf(1.0f + Dm1);
    r.A = invD;
    r.Bg = (sh + c * chm1) * in * invD;
    r.dK = dm1 * (double)log1pf(Dm1);
  } else {
    const float e2 = __expf(-2.0f * ad);
    const float tau = copysignf((1.0f - e2) * __builtin_amdgcn_rcpf(1.0f + e2), delta);
    const float sech = 2.0f * __expf(-ad) * __builtin_amdgcn_rcpf(1.0f + e2);
    const float iDh = __builtin_amdgcn_rcpf(1.0f + c * tau);
    r.A = sech * iDh;
    r.Bg = (tau + c * (1.0f - sech)) * in * iDh;
    r.dK = dm1 * ((double)ad + (double)log1pf(e2) - 0.69314718055994531 - (double)__logf(iDh));
  }
  return r;
}

template <class Real>
__device__ __forceinline__ BMap b_map_t(double gg, double gu, double h, double dm1) {
  return sizeof(Real) == 8 ? b_map(gg, gu, h, dm1) : b_map_f(gg, gu, h, dm1);
}

// Underdamped Langevin variant (the dynamics ablation of appendix "Ablation
// studies"): Gaussian velocity with covariance I/d (mass d, so |u| ~ 1 and eps,
// L keep their units).  The kick is exact for fixed g, u' = u + (h/d) g~, with
// kinetic change (d/2)(|u'|^2 - |u|^2) = h g~.u + h^2 |g~|^2 / (2d); the refresh
// is the microcanonical one without the renormalisation.  dyn selects the
// dynamics for the whole launch (a uniform branch).
template <class Real>
__device__ __forceinline__ BMap b_map_dyn(int dyn, double gg, double gu, double h, double dm1) {
  if (dyn) {
    const double dd = dm1 + 1.0;
    BMap r;
    r.A = 1.0;
    r.Bg = h / dd;
    r.dK = h * gu + 0.5 * h * h * gg / dd;
    return r;
  }
  return b_map_t<Real>(gg, gu, h, dm1);
}

// Scale applied after a partial refresh with squared norm ww: back onto the
// unit sphere (microcanonical), none (Langevin).
__device__ __forceinline__ double refresh_scale(int dyn, double ww) { return dyn ? 1.0 : 1.0 / sqrt(ww); }

// Scale of a full refresh of d standard normals with squared norm zz: uniform
// on the sphere (microcanonical) or N(0, I/d) (Langevin).
__device__ __forceinline__ double full_refresh_scale(int dyn, double zz, int64_t d) {
  return dyn ? 1.0 / sqrt((double)d) : 1.0 / sqrt(zz);
}

// Integrator coefficient sets (Table "Integrators"): symmetric B A B ... B,
// the coefficients not printed follow from symmetry and normalisation.
struct Coeffs {
  int K;
  double b[6], a[5];
};

__host__ __device__ inline Coeffs integrator_coeffs(int which) {
  Coeffs c{};
  if (which == 0) {
    c.K = 2;
    c.b[0] = 0.5;
    c.b[1] = 0.5;
    c.a[0] = 1.0;
  } else if (which == 1) {
    const double b1 = 0.1931833275;
    c.K = 3;
    c.b[0] = b1;
    c.b[1] = 1.0 - 2.0 * b1;
    c.b[2] = b1;
    c.a[0] = 0.5;
    c.a[1] = 0.5;
  } else {
    const double b1 = 0.0839831526, b2 = 0.6822365335, a1 = 0.2539785108, a2 = -0.032302867;
    const double b3 = 0.5 - b1 - b2, a3 = 1.0 - 2.0 * (a1 + a2);
    c.K = 6;
    c.b[0] = b1;
    c.b[1] = b2;
    c.b[2] = b3;
    c.b[3] = b3;
    c.b[4] = b2;
    c.b[5] = b1;
    c.a[0] = a1;
    c.a[1] = a2;
    c.a[2] = a3;
    c.a[3] = a2;
    c.a[4] = a1;
  }
  return c;
}

}  // namespace laps
