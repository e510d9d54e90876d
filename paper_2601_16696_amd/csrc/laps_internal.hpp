// Host/device argument blocks and launcher declarations shared by the
// translation units of the LAPS library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "laps_device.hpp"

namespace laps {

// Arguments of the per-chain kernels.  A team of T lanes owns one chain; lane
// r of a team owns the "octs" r + q T (q < Q) of the chain, i.e. the eight
// consecutive coordinates 8 (r + q T) .. 8 (r + q T) + 7, which is also the
// unit of one Philox block.  Rows have stride ld (a multiple of 8).
struct LocalArgs {
  void *x, *u, *g;
  double *logp, *delta, *acc;
  double *partials;        // [gridDim][4][ld]: sums of x-K, (x-K)^2, (x-K) g, g
  const double *shiftK;    // [ld] shift K (previous ensemble mean)
  DevHyper *hyp;
  const void *sigma;       // [ld] diagonal preconditioner (state type)
  const void *u0;          // optional initial velocities
  const void *aux;         // [ld] per-dim target constants (state type)
  const double *tdata;     // target data in double (SV returns y)
  int64_t tn;              // SV: T; phi4: L
  double tp0, tp1;         // phi4: m2, lambda
  int64_t N, d, ld;
  int T, tpw;
  uint64_t seed;
  int64_t max_total;
  int n_traj;
  double Lp_factor;
  int cache;               // store g and log p (1) or recompute them (0)
  int dyn;                 // 0 microcanonical velocity, 1 underdamped Langevin
  int stats;               // accumulate per-dim sums in the step kernel (1) or leave them to k_stats (0)
  double *logp_out;        // target eval: log p output
  void *g_out;             // target eval: gradient output (or null)
  // unadjusted step: normals written one step ahead by zn_blocks workgroups
  // appended to the launch, [2 slots][2 refreshes][N][ld] of the state type;
  // slot t % 2 holds step t's normals when zn_tag[t % 2] == t + 1
  void *zn;
  uint64_t *zn_tag;
  int zn_blocks;
  // MAMS transition: the next transition's normals written by zm_blocks
  // appended workgroups, [2 slots][2 n_traj + 1][N][ld]; slot (t / n_traj) % 2
  // holds the transition starting at t when zm_tag[slot] == t + 1
  void *zm;
  uint64_t *zm_tag;
  int zm_blocks;
};

// Arguments of the statistics / controller kernels.
struct CtlArgs {
  DevHyper *hyp;
  const double *partials;
  int G;                   // partial rows
  double *shiftK, *mean, *var, *m2, *Vii;
  double *ring, *wdelta;
  int64_t Tw;
  double *part2;           // [nb][4] per-block scalars
  int nb;
  const double *delta, *acc;
  int64_t N, d, ld;
  double C, alpha, eps0_factor, switch_tol, acc_tol, acc_target;
  double eps_fixed;  // > 0: unadjusted-phase step size held at this value
  int n_traj, eevpd_mode, switch_policy, integ;
  int64_t max_unadj, max_total;
  void *sigma;
  int sigma_double;
  // full-rank equipartition loss (probes > 0): positions and gradients of the
  // step, the probe dot products [N][P], per-chunk projections [NC][P][d] and
  // per-block squared norms [nbh]
  int probes, NC, nbh;
  uint64_t seed;
  const void *x, *g;
  double *pS, *pW, *pPart;
};

enum { FIN_INIT = 0, FIN_UNADJ = 1 };

// How write_partials stages a workgroup's per-dimension partial row through
// LDS (the four rows of a group hold 8 Q T doubles each):
//   2: teams of at most 32 lanes, every 32-lane half of every wavefront at once
//      (folded over its 16-lane rows only), within kPartialsHalves bytes;
//   1: every wavefront group's folded rows at once, within kPartialsOneRound;
//   0: one group's rows, the groups then added one after another.
constexpr size_t kPartialsOneRound = 16 * 1024, kPartialsHalves = 32 * 1024;
__host__ __device__ inline int partials_mode(int block, int T, int Q) {
  const int groups = block / (T < 64 ? 64 : T);
  const size_t rows = (size_t)4 * 8 * Q * T * sizeof(double);
  if (T <= 32 && (size_t)2 * groups * rows <= kPartialsHalves) return 2;
  if (groups > 1 && (size_t)groups * rows <= kPartialsOneRound) return 1;
  return 0;
}
// The LDS bytes of that staging.
__host__ __device__ inline size_t partials_lds_bytes(int block, int T, int Q) {
  const int groups = block / (T < 64 ? 64 : T);
  const size_t rows = (size_t)4 * 8 * Q * T * sizeof(double);
  const int mode = partials_mode(block, T, Q);
  return mode == 2 ? (size_t)2 * groups * rows : mode == 1 ? (size_t)groups * rows : rows;
}
// dimensions per workgroup of the statistics pass (its block count is
// ceil(d / fin_dims(d)))
__host__ __device__ inline int fin_dims(int64_t d) { return d <= 1024 ? 8 : 32; }
constexpr int kProbeChunk = 128;  // chains per partial projection of the full-rank loss

// Launchers (return hipSuccess or the launch error).
hipError_t launch_hyper_init(const CtlArgs &c, hipStream_t s);
hipError_t launch_finalize(const CtlArgs &c, int mode, hipStream_t s);
hipError_t launch_ctl_init(const CtlArgs &c, hipStream_t s);
hipError_t launch_switch(const CtlArgs &c, hipStream_t s);
hipError_t launch_ctl_adj(const CtlArgs &c, hipStream_t s);
hipError_t launch_ctl_unadj(const CtlArgs &c, hipStream_t s);
hipError_t launch_probes(const CtlArgs &c, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);

enum KernelKind { KK_INIT = 0, KK_UNADJ = 1, KK_MAMS_MN2 = 2, KK_MAMS_MN4 = 3, KK_EVAL = 4 };

// Local targets: kind is laps_target_kind (gauss, stochvol, phi4).
hipError_t launch_local(int kind, bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block,
                        size_t shmem, hipStream_t s);
hipError_t launch_local_gauss(bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem,
                              hipStream_t s);
hipError_t launch_local_sv(bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem,
                           hipStream_t s);
hipError_t launch_local_phi4(bool dbl, int Q, KernelKind kk, const LocalArgs &a, int grid, int block, size_t shmem,
                             hipStream_t s);
// Raises a kernel's dynamic LDS limit to at least `bytes` (no-op up to 64 KiB;
// gfx950 gives a workgroup up to 160 KiB).  Grants are remembered per kernel.
hipError_t grant_lds(const void *kernel, size_t bytes);
hipError_t launch_prep_aux(int kind, bool dbl, const void *src, void *aux, int64_t d, int64_t ld, hipStream_t s);
// Per-dimension ensemble sums of (x - K, (x - K)^2, (x - K) g, g) over CB
// chain blocks, one partial row per block (used when the step kernel does not
// accumulate them itself).
hipError_t launch_stats(bool dbl, const void *x, const void *g, const double *shiftK, double *partials, int64_t N,
                        int64_t d, int64_t ld, int CB, const DevHyper *hyp, hipStream_t s);

// Logistic regression.  The gradient kernels split the n data rows over S
// workgroup columns and write per-split partial sums (G = X^T r rows and
// sum_n [y z - softplus z]); the per-chain update kernels combine them.
struct LogregArgs {
  void *x, *u, *g;
  double *logp, *delta, *acc, *partials;
  const double *shiftK;
  DevHyper *hyp;
  const void *sigma;
  const void *u0;
  const void *X;           // LAPS_F64: double [n][d]; bf16 paths: uint16 bf16 bits [n][d]
  const double *y;         // [n] labels
  char *scratch;           // region laid out by logreg_layout()
  int64_t n, N, d, ld;
  int S, NB, KC, bps;      // row splits, 32-row blocks, 32-wide k chunks, blocks per split
  int T, tpw;              // team shape of the update kernels
  int dyn;                 // 0 microcanonical velocity, 1 underdamped Langevin
  uint64_t seed;
  int64_t max_total;
  int n_traj;
  double Lp_factor;
  int gate;                // 0: always; 1: unadjusted phase; 2: adjusted phase below max_total
  int mode, j, k, integ;   // update-kernel selector
  // integrator coefficients of the stage (set by the host per launch): b_0,
  // a_0, b_{k+1}, a_{k+1} and the stage count K
  double cb0, ca0, cbk, cak;
  int cK;
  int prior;               // 1: add the N(0, I) prior of logistic regression to the partial sums; 0: caller's log p
  int wy_term;             // 1: add theta . (X^T (y - 1/2)), left out of the bf16 gradient's split sums
  double *logp_out;        // LR_EVAL: log p output [N]
  void *g_out;             // LR_EVAL: gradient output [N][ld] (or null)
};

enum { LR_INIT = 0, LR_PRE = 1, LR_POST = 2, LR_MBEGIN = 3, LR_MSTEP = 4, LR_EVAL = 5 };

struct LrOffsets {
  size_t Xf, Xb, yf, wy, Gp, lp, x0, g0, sc, total;
};
__host__ __device__ inline size_t lr_al256(size_t v) { return (v + 255) / 256 * 256; }

__host__ __device__ inline LrOffsets logreg_layout(int prec, int64_t n, int64_t d, int64_t N, int64_t ld, int S) {
  const int64_t NB = (n + 31) / 32, KC = (d + 31) / 32;
  const size_t rs = prec == 0 ? 8 : 4;
  const bool bf = prec != 0;
  LrOffsets o{};
  size_t off = 0;
  o.Xf = off;
  off = lr_al256(off + (bf ? (size_t)NB * 2 * KC * 64 * 8 * 2 : 0));
  o.Xb = off;
  off = lr_al256(off + (bf ? (size_t)NB * 2 * KC * 64 * 8 * 2 : 0));
  o.yf = off;
  off = lr_al256(off + (bf ? (size_t)NB * 32 * 4 : 0));
  o.wy = off;
  off = lr_al256(off + (bf ? (size_t)ld * 8 : 0));
  o.Gp = off;
  off = lr_al256(off + (size_t)S * N * ld * rs);
  o.lp = off;
  off = lr_al256(off + (size_t)S * N * 8);
  o.x0 = off;
  off = lr_al256(off + (size_t)N * ld * rs);
  o.g0 = off;
  off = lr_al256(off + (size_t)N * ld * rs);
  o.sc = off;
  off = lr_al256(off + (size_t)4 * N * 8);
  o.total = off;
  return o;
}

// Row splits of the gradient launch: wgs workgroups aimed for (0: automatic).
void logreg_splits(int64_t n, int64_t N, int prec, int64_t d, int wgs, int &S, int &NB, int &bps);
hipError_t launch_logreg_pack(const LogregArgs &a, hipStream_t s);
hipError_t launch_logreg_grad(int prec, const LogregArgs &a, hipStream_t s);
// Q octs per lane (1..4) in teams of a.T <= 16 lanes.
hipError_t launch_logreg_update(int prec, int Q, const LogregArgs &a, int grid, int block, size_t shmem,
                                hipStream_t s);
// Dense-precision Gaussian: the precision matrix copied in the state type
// after the single partial-sum split of the scratch, and its gradient kernel.
hipError_t launch_dense_pack(int prec, const LogregArgs &a, hipStream_t s);
hipError_t launch_dense_grad(int prec, const LogregArgs &a, hipStream_t s);

}  // namespace laps
