// The sampler's counter-based random numbers as standalone entry points.
#include "laps.h"
#include "laps_internal.hpp"

namespace laps {

__global__ void k_philox_words(const uint64_t *ctr, uint64_t *out, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  philox4x64_10(c, seed, 0);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[4 * i + k] = c[k];
}

// one thread per (chain, oct)
template <class Real>
__global__ void k_philox_normals(uint64_t seed, int64_t n_chains, int64_t d, int64_t ld, uint64_t t, uint32_t tag,
                                 uint32_t sub, Real *out) {
  const int64_t octs = ld / 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_chains * octs) return;
  const int64_t m = i / octs, j = i - m * octs;
  Real z[8];
  normals8<Real>(seed, (uint64_t)m, (uint64_t)j, t, tag, sub, z);
#pragma unroll
  for (int k = 0; k < 8; ++k) out[m * ld + 8 * j + k] = (8 * j + k < d) ? z[k] : Real(0);
}

}  // namespace laps

extern "C" laps_status laps_philox_words(const uint64_t *ctr, uint64_t *out, int64_t n, uint64_t seed,
                                         void *stream) {
  if (!ctr || !out || n < 0) return LAPS_EINVAL;
  if (n == 0) return LAPS_OK;
  hipLaunchKernelGGL(laps::k_philox_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), ctr, out, n, seed);
  return hipGetLastError() == hipSuccess ? LAPS_OK : LAPS_EDEVICE;
}

extern "C" laps_status laps_philox_normals(uint64_t seed, int64_t n_chains, int64_t d, uint64_t t, uint32_t tag,
                                           uint32_t sub, int32_t prec, void *out, void *stream) {
  if (!out || n_chains < 0 || d < 1 || prec < 0 || prec > 2 || ((uintptr_t)out & 31)) return LAPS_EINVAL;
  const int64_t ld = laps_row_stride(d);
  const int64_t total = n_chains * (ld / 8);
  if (total == 0) return LAPS_OK;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (prec == LAPS_F64)
    hipLaunchKernelGGL(laps::k_philox_normals<double>, grid, dim3(256), 0, static_cast<hipStream_t>(stream), seed,
                       n_chains, d, ld, t, tag, sub, static_cast<double *>(out));
  else
    hipLaunchKernelGGL(laps::k_philox_normals<float>, grid, dim3(256), 0, static_cast<hipStream_t>(stream), seed,
                       n_chains, d, ld, t, tag, sub, static_cast<float *>(out));
  return hipGetLastError() == hipSuccess ? LAPS_OK : LAPS_EDEVICE;
}
