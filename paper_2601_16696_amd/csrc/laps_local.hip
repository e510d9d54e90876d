// Host dispatch of the per-chain kernels, and the two small helper kernels
// they rely on: the column sums of the per-dimension ensemble statistics and
// the per-dimension target constants.  The per-chain kernels themselves are
// instantiated per target in laps_local_{gauss,sv,phi4}.hip.
#include <mutex>
#include <unordered_map>

#include "laps_team.hpp"

namespace laps {

hipError_t grant_lds(const void *kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  static std::mutex mu;
  static std::unordered_map<const void *, size_t> granted;
  std::lock_guard<std::mutex> lock(mu);
  size_t &have = granted[kernel];
  if (bytes <= have) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) have = bytes;
  return e;
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

hipError_t launch_local(int kind, bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block,
                        size_t shmem, hipStream_t s) {
  if (kind == 0) return launch_local_gauss(dbl, Q, kk, a, grid, block, shmem, s);
  if (kind == 2) return launch_local_sv(dbl, Q, kk, a, grid, block, shmem, s);
  if (kind == 3) return launch_local_phi4(dbl, Q, kk, a, grid, block, shmem, s);
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
