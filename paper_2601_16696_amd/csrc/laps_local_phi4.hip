// Per-chain kernel instances for the phi^4 lattice target.
#include "laps_local.hpp"

namespace laps {

hipError_t launch_local_phi4(bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem,
                             hipStream_t s) {
  // lattices whose rows are whole octs take the vectorised neighbour path;
  // other side lengths run one oct per lane
  if ((a.tn & 7) == 0) return launch_target<Phi4Tgt>(dbl, Q, kk, a, grid, block, shmem, s);
  if (Q != 1) return hipErrorInvalidValue;
  if (dbl) return launch_kind<double, 1, Phi4AnyTgt<double, 1>>(kk, a, grid, block, shmem, s);
  return launch_kind<float, 1, Phi4AnyTgt<float, 1>>(kk, a, grid, block, shmem, s);
}

}  // namespace laps
