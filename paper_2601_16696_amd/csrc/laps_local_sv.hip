// Per-chain kernel instances for the stochastic-volatility target.
#include "laps_local.hpp"

namespace laps {

hipError_t launch_local_sv(bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem,
                         hipStream_t s) {
  return launch_target<SVTgt>(dbl, Q, kk, a, grid, block, shmem, s);
}

}  // namespace laps
