// Gaussian with a dense precision matrix A (the randomly rotated,
// ill-conditioned Gaussian of section "Results"): log p = -x^T A x / 2 and
// g = -A x for every chain, as one matrix product X A on the matrix cores.
//
// A workgroup holds 16 chains; each of its wavefronts (up to 16) computes
// 16-wide output tiles t = w, w + nw, ... of those chains, four input dims per
// instruction:
//   FP64 state: v_mfma_f64_16x16x4_f64; FP32 state: v_mfma_f32_16x16x4_f32.
// Lane l supplies X[m0 + l%16][k0 + l/16] and A[k0 + l/16][j0 + l%16]; its
// results are (chain, dim) = (m0 + l/16 + 4i, j0 + l%16) for FP64 and
// (m0 + 4(l/16) + i, j0 + l%16) for FP32 (lane layouts measured on the MI355X).
// log p = x.g / 2 is summed per chain in FP64 over a wavefront's tiles in
// order, across the 16 lanes of a chain by xor butterflies, then over the
// wavefronts in order through LDS (a fixed order throughout).
// Outputs go to the single partial-sum split that the per-chain update
// kernels read (g and log p without a prior term).
#include "laps_internal.hpp"

namespace laps {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

template <class Real>
struct DenseMfma;
template <>
struct DenseMfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return (lane >> 4) + 4 * i; }
};
template <>
struct DenseMfma<float> {
  typedef f32x4v acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

template <class Real>
__global__ void __launch_bounds__(1024) k_dense_grad(LogregArgs a) {
  if (a.gate != 0) {
    const DevHyper *H = a.hyp;
    if (a.gate == 1 && H->phase != PH_UNADJ) return;
    if (a.gate == 2 && !(H->phase == PH_ADJ && H->t < a.max_total)) return;
  }
  typedef DenseMfma<Real> M;
  typedef typename M::acc_t acc_t;
  __shared__ double lsh[16 * 16];  // [wavefront][chain]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t N = a.N, d = a.d, ld = a.ld;
  const int64_t m0 = (int64_t)blockIdx.x * 16;
  const LrOffsets off = logreg_layout(sizeof(Real) == 8 ? 0 : 1, 0, d, N, ld, 1);
  const Real *X = static_cast<const Real *>(a.x);
  const Real *A = reinterpret_cast<const Real *>(a.scratch + off.total);  // [d][d] in the state type
  Real *G = reinterpret_cast<Real *>(a.scratch + off.Gp);
  double *LP = reinterpret_cast<double *>(a.scratch + off.lp);
  const int64_t ma = m0 + (lane & 15);  // chain of this lane's input operand
  const int kl = lane >> 4;             // input dim within a group of four
  const int jl = lane & 15;             // output dim within a tile
  const int64_t JT = (d + 15) / 16;
  double lp[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t t = wave; t < JT; t += nw) {
    const int64_t j = t * 16 + jl;
    acc_t acc = acc_t{0, 0, 0, 0};
    int64_t k0 = 0;
    for (; k0 + 16 <= d; k0 += 16) {
      // four groups of four input dims: their eight loads are issued together
      Real av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t k = k0 + 4 * u + kl;
        av[u] = ma < N ? X[ma * ld + k] : Real(0);
        bv[u] = j < d ? A[k * d + j] : Real(0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = M::mma(av[u], bv[u], acc);
    }
    for (; k0 < d; k0 += 4) {
      const int64_t k = k0 + kl;
      const Real av = (ma < N && k < d) ? X[ma * ld + k] : Real(0);
      const Real bv = (k < d && j < d) ? A[k * d + j] : Real(0);
      acc = M::mma(av, bv, acc);
    }
    if (j < d) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + M::row(lane, i);
        if (m < N) {
          const Real g = -acc[i];
          G[m * ld + j] = g;
          lp[i] += (double)X[m * ld + j] * (double)g;
        }
      }
    }
  }
  // per chain: the 16 lanes of equal lane / 16 hold a wavefront's dims ...
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int msk = 1; msk < 16; msk <<= 1) lp[i] += __shfl_xor(lp[i], msk);
    if (jl == 0) lsh[wave * 16 + M::row(lane, i)] = lp[i];
  }
  __syncthreads();
  // ... and the wavefronts' sums are added in wavefront order
  if (threadIdx.x < 16) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lsh[w * 16 + threadIdx.x];
    const int64_t m = m0 + threadIdx.x;
    if (m < N) LP[m] = 0.5 * s;
  }
}

// The precision matrix in the state type, once per context.
template <class Real>
__global__ void k_dense_pack(const double *A, Real *out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (Real)A[i];
}

hipError_t launch_dense_pack(int prec, const LogregArgs &a, hipStream_t s) {
  const LrOffsets off = logreg_layout(prec == 0 ? 0 : 1, 0, a.d, a.N, a.ld, 1);
  const int64_t n = a.d * a.d;
  const dim3 grid((unsigned)((n + 255) / 256));
  const double *A = static_cast<const double *>(a.X);
  if (prec == 0)
    hipLaunchKernelGGL(k_dense_pack<double>, grid, dim3(256), 0, s, A, reinterpret_cast<double *>(a.scratch + off.total), n);
  else
    hipLaunchKernelGGL(k_dense_pack<float>, grid, dim3(256), 0, s, A, reinterpret_cast<float *>(a.scratch + off.total), n);
  return hipGetLastError();
}

hipError_t launch_dense_grad(int prec, const LogregArgs &a, hipStream_t s) {
  // 16 chains per workgroup, one wavefront per output tile up to 16
  const int64_t JT = (a.d + 15) / 16;
  const dim3 grid((unsigned)((a.N + 15) / 16)), block((unsigned)(64 * (JT < 16 ? JT : 16)));
  if (prec == 0)
    hipLaunchKernelGGL(k_dense_grad<double>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(k_dense_grad<float>, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace laps
