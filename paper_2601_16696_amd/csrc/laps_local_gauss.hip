// Per-chain kernel instances for the diagonal Gaussian target.
#include "laps_local.hpp"

namespace laps {

hipError_t launch_local_gauss(bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem,
                         hipStream_t s) {
  return launch_target<GaussTgt>(dbl, Q, kk, a, grid, block, shmem, s);
}

}  // namespace laps
