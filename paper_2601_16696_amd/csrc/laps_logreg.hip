// Logistic regression target (placeholder until the matrix-core kernels land).
#include "laps_internal.hpp"

namespace laps {
int logreg_tile_chains(int) { return 64; }
size_t logreg_packed_bytes(int, int64_t, int64_t) { return 0; }
hipError_t launch_logreg_pack(int, const void *, void *, int64_t, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_logreg(int, KernelKind, const LogregArgs &, int, hipStream_t) { return hipErrorNotSupported; }
}  // namespace laps
