// Host side of the C ABI declared in include/laps.h: argument validation,
// workspace carving, launch-shape selection and kernel enqueueing.  No device
// memory is allocated here and nothing synchronises except
// laps_ensemble_stats.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "laps.h"
#include "laps_internal.hpp"

using namespace laps;

struct laps_ctx {
  laps_config cfg;
  laps_target tg;
  void *x;
  hipStream_t stream;
  bool dbl;
  int64_t ld, Tw;
  // launch shape of the per-chain kernels; G = partial rows of the statistics
  int T, Q, tpw, block, G, nb, grid_full;
  bool split;
  size_t shmem, shmem_sig;
  int integ;
  bool adj_started;
  bool packed_ok;  // logistic regression: operand fragments of X packed
  bool is_static = false;  // context of laps_init_static: library storage, never deleted
  // workspace
  DevHyper *hyp;
  void *u, *g, *sigma, *aux, *packed;
  double *logp, *delta, *acc, *partials, *shiftK, *mean, *var, *m2, *Vii, *ring, *wdelta, *part2;
  double *pS, *pW, *pPart;  // full-rank loss scratch
  void *zn;                 // normals of the next unadjusted step (zn_blocks > 0)
  uint64_t *zn_tag;
  int zn_blocks;
  void *zm;                 // normals of the next MAMS transition (zm_blocks > 0)
  uint64_t *zm_tag;
  int zm_blocks;
  std::string err;
  // optional event pairs around the launches of one kernel (laps_kernel_log)
  int log_which = 0, log_every = 1;
  int64_t log_seen = 0;  // launches of the logged kernel so far
  std::vector<hipEvent_t> log_ev;
  size_t log_used = 0;
  ~laps_ctx() {
    for (hipEvent_t e : log_ev) (void)hipEventDestroy(e);
  }
};

static std::string g_last_global;

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

extern "C" int64_t laps_row_stride(int64_t d) { return round_up(d < 1 ? 1 : d, 8); }

extern "C" void laps_config_default(laps_config *c, int64_t n_chains, int64_t d) {
  memset(c, 0, sizeof(*c));
  c->n_chains = n_chains;
  c->d = d;
  c->prec = LAPS_F64;
  c->seed = 0;
  c->C = 0.025;
  c->alpha = 2.0;
  c->eps0_factor = 0.01;
  c->switch_tol = 0.01;
  c->window_frac = 0.2;
  c->acc_tol = 0.03;
  c->acc_target = 0.0;
  c->L_partial_factor = 1.25;
  c->n_steps_traj = 15;
  c->integrator_adj = 0;
  c->eevpd_mode = 1;
  c->switch_policy = 0;
  c->max_steps_unadj = 1000;
  c->max_steps_total = 2000;
}

namespace {

struct Shape {
  int T, Q, tpw, block, G, nb, grid_full;
  bool split;
  size_t shmem, shmem_sig;  // dynamic LDS without / with the preconditioner row
  bool ahead = true;        // normals computed ahead where the shape allows it (noise_blocks)
};

// Largest dimension of the targets run by the per-chain update kernels
// (callbacks, the dense Gaussian): teams of at most 16 lanes with up to 4 octs
// per lane.  Logistic regression stops at 128, where its matrix-core gradient
// kernels hold theta and the gradient tiles of a chain in registers.
constexpr int64_t kUpdateMaxD = 512;
constexpr int64_t kLogregMaxD = 128;

bool is_local(int kind) { return kind == LAPS_GAUSS_DIAG || kind == LAPS_STOCHVOL || kind == LAPS_PHI4; }

// Team shape of the per-chain kernels: the chain's ceil(d/8) octs over T
// lanes, Q octs per lane.  Short chains get one oct per lane (T the next power
// of two) and accumulate the per-dim sums in registers; longer chains take a
// whole wavefront (T = 64) with Q octs per lane, so that the per-chain scalar
// work is shared by 8 Q coordinates per lane; only chains longer than 64 lanes
// x Q_max octs use multi-wavefront teams.  FP64 state keeps up to 2 octs per
// lane in registers, FP32 up to 6.
bool local_shape(int kind, bool dbl, int64_t N, int64_t d, int team_lanes, Shape &s, int block_threads = 0) {
  const int64_t octs = (d + 7) / 8;
  // a phi^4 lattice whose rows are not whole octs runs one oct per lane
  const int64_t side = kind == LAPS_PHI4 ? (int64_t)llround(sqrt((double)d)) : 0;
  const int64_t qmax = (kind == LAPS_PHI4 && side % 8 != 0) ? 1 : (dbl ? 2 : 6);
  int64_t T;
  if (team_lanes > 0) {
    T = team_lanes;
    const bool pow2 = (T & (T - 1)) == 0;
    if (!((T <= 64 && pow2) || (T % 64 == 0 && T <= 512))) return false;
  } else if (octs <= 64) {
    T = 1;
    while (T < octs) T <<= 1;
  } else if (octs <= 64 * qmax) {
    T = 64;
  } else {
    T = 64 * ((octs + 64 * qmax - 1) / (64 * qmax));
    if (T > 512) return false;
  }
  const int64_t Q = (octs + T - 1) / T;
  if (Q > qmax) return false;
  s.T = (int)T;
  s.Q = (int)Q;
  s.split = !(Q == 1 && T <= 64);
  const int64_t ld = laps_row_stride(d);
  const size_t rs = dbl ? 8 : 4;
  const bool aux = kind != LAPS_PHI4;
  const bool stage = kind == LAPS_PHI4 || (kind == LAPS_STOCHVOL && T > 64);
  const size_t fixed = 2 * kRedSlots * sizeof(double) + (aux ? (size_t)ld * rs : 0);
  auto body = [&](int64_t blk) -> size_t {
    size_t b = stage ? (size_t)(blk / T) * ld * rs : 0;
    if (!s.split && blk > T) {
      const size_t pb = partials_lds_bytes((int)blk, (int)T, (int)Q);  // staging of the per-dim partial row
      if (pb > b) b = pb;
    }
    return b;
  };
  // Up to 256 threads per workgroup; fewer when the teams' chain copies would
  // take more than 56 KiB of LDS (which would cap the resident wavefronts).
  int64_t block = T <= 64 ? 256 : T;
  // workgroup size override (64, 128 or 256 threads) for teams inside a wavefront
  if (T <= 64 && (block_threads == 64 || block_threads == 128 || block_threads == 256)) block = block_threads;
  while (T <= 64 && block > T && block > 64 && fixed + body(block) + (size_t)ld * rs > 56 * 1024) block >>= 1;
  s.block = (int)block;
  s.tpw = (int)(block / T);
  const int64_t need = (N + s.tpw - 1) / s.tpw;
  s.grid_full = (int)need;
  if (s.split) {
    s.G = (int)(N < 64 ? N : 64);
  } else {
    // at most 512 workgroups (two per CU): each writes one partial row of the statistics
    const int64_t gmax = 512;
    s.G = (int)(need < gmax ? need : gmax);
  }
  s.shmem = fixed + body(block);
  s.shmem_sig = s.shmem + (size_t)ld * rs;
  s.nb = (int)((d + fin_dims(d) - 1) / fin_dims(d));
  return true;
}

bool shape_for(const laps_config *cfg, const laps_target *tg, Shape &s) {
  const bool dbl = cfg->prec == LAPS_F64;
  if (is_local(tg->kind))
    return local_shape(tg->kind, dbl, cfg->n_chains, cfg->d, cfg->team_lanes, s, cfg->block_threads);
  if (tg->kind == LAPS_LOGREG || tg->kind == LAPS_CALLBACK || tg->kind == LAPS_GAUSS_DENSE) {
    // per-chain update kernels: one oct per lane in teams of up to 16 lanes,
    // then 16-lane teams with Q = 2..4 octs per lane
    const int64_t octs = (cfg->d + 7) / 8;
    if (cfg->d > kUpdateMaxD) return false;
    int T = 1;
    while (T < octs && T < 16) T <<= 1;
    s.T = T;
    s.Q = (int)((octs + T - 1) / T);
    s.block = cfg->block_threads > 0 ? cfg->block_threads : 256;  // 64, 128 or 256 >= T
    s.tpw = s.block / T;
    s.G = (int)((cfg->n_chains + s.tpw - 1) / s.tpw);
    s.grid_full = s.G;
    s.split = false;
    s.shmem = 2 * kRedSlots * sizeof(double) + partials_lds_bytes(s.block, T, s.Q);
    s.shmem_sig = s.shmem;
    s.nb = (int)((cfg->d + fin_dims(cfg->d) - 1) / fin_dims(cfg->d));
    return true;
  }
  return false;
}

struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (size_t)round_up((int64_t)off, 256);
    const size_t at = off;
    off += bytes;
    return at;
  }
};

struct Layout {
  size_t hyp, u, g, logp, delta, acc, partials, shiftK, mean, var, m2, Vii, ring, wdelta, part2, sigma, aux, packed,
      pS, pW, pPart, zn, zn_tag, zm, zm_tag, total;
};

// Workgroups appended to an unadjusted-step launch to compute the next step's
// normals ahead (0: none).  FP64 state of the per-chain targets only (FP32
// normals use the hardware transcendentals and cost little), and only when
// the chain workgroups occupy at most half of the 1024 SIMDs, so that the
// appended ones run on compute units that would otherwise idle.
int noise_blocks(const laps_config *cfg, const laps_target *tg, const Shape &s) {
  if (!s.ahead || !is_local(tg->kind) || cfg->prec != LAPS_F64) return 0;
  const int64_t grid = s.split ? s.grid_full : s.G;
  if (grid * ((s.block + 63) / 64) > 512) return 0;
  const int64_t items = 2 * cfg->n_chains * ((cfg->d + 7) / 8);  // one thread per oct and refresh
  return (int)((items + s.block - 1) / s.block);
}

// Workgroups appended to a MAMS launch to compute the next transition's
// normals (0: none): on the same shapes as noise_blocks with one oct per lane
// (the kernel holds the next step's normals across the gradient stages only
// then), about 8 normals blocks per thread so that they finish well within
// the transition, and at most 512 workgroups in all.
int mams_noise_blocks(const laps_config *cfg, const laps_target *tg, const Shape &s) {
  if (noise_blocks(cfg, tg, s) == 0 || s.Q != 1 || cfg->n_steps_traj < 1) return 0;
  const int64_t items = (2 * (int64_t)cfg->n_steps_traj + 1) * cfg->n_chains * ((cfg->d + 7) / 8);
  const int64_t nb = (items + 8 * (int64_t)s.block - 1) / (8 * (int64_t)s.block);
  return s.grid_full + nb <= 512 ? (int)nb : 0;
}

int probe_chunks(int64_t N) { return (int)((N + kProbeChunk - 1) / kProbeChunk); }
int probe_blocks(int64_t d, int64_t P) { return (int)((d * P + 255) / 256); }

Layout layout(const laps_config *cfg, const laps_target *tg, const Shape &s) {
  const int64_t N = cfg->n_chains, d = cfg->d, ld = laps_row_stride(d);
  const size_t rs = cfg->prec == LAPS_F64 ? 8 : 4;
  int64_t Tw = (int64_t)llround(cfg->window_frac * (double)cfg->max_steps_total);
  if (Tw < 2) Tw = 2;
  Carve c;
  Layout L;
  L.hyp = c.take(sizeof(DevHyper));
  L.u = c.take((size_t)N * ld * rs);
  L.g = c.take((size_t)N * ld * rs);
  L.logp = c.take((size_t)N * 8);
  L.delta = c.take((size_t)N * 8);
  L.acc = c.take((size_t)N * 8);
  L.partials = c.take((size_t)s.G * 4 * ld * 8);
  L.shiftK = c.take((size_t)ld * 8);
  L.mean = c.take((size_t)ld * 8);
  L.var = c.take((size_t)ld * 8);
  L.m2 = c.take((size_t)ld * 8);
  L.Vii = c.take((size_t)ld * 8);
  L.ring = c.take((size_t)Tw * ld * 8);
  L.wdelta = c.take((size_t)ld * 8);
  L.part2 = c.take((size_t)s.nb * 4 * 8);
  L.sigma = c.take((size_t)ld * rs);
  L.aux = c.take((size_t)ld * rs);
  size_t lr = 0;
  if (tg->kind == LAPS_LOGREG) {
    int S, NB, bps;
    logreg_splits(tg->dims[0], N, cfg->prec, d, cfg->grad_workgroups, S, NB, bps);
    lr = logreg_layout(cfg->prec == LAPS_F64 ? 0 : 1, tg->dims[0], d, N, ld, S).total;
  } else if (tg->kind == LAPS_CALLBACK) {
    // one partial-sum "split": the callback's g and log p
    lr = logreg_layout(cfg->prec == LAPS_F64 ? 0 : 1, 0, d, N, ld, 1).total;
  } else if (tg->kind == LAPS_GAUSS_DENSE) {
    // one partial-sum split, then the precision matrix in the state type
    lr = logreg_layout(cfg->prec == LAPS_F64 ? 0 : 1, 0, d, N, ld, 1).total + (size_t)round_up(d * d * rs, 256);
  }
  L.packed = c.take(lr);
  const int64_t P = cfg->full_rank_probes;
  L.pS = c.take((size_t)N * P * 8);
  L.pW = c.take((size_t)probe_chunks(N) * P * d * 8);
  L.pPart = c.take((size_t)(P > 0 ? probe_blocks(d, P) : 0) * 8);
  const bool zn = noise_blocks(cfg, tg, s) > 0;
  L.zn = c.take(zn ? (size_t)4 * N * ld * rs : 0);
  L.zn_tag = c.take(zn ? 2 * sizeof(uint64_t) : 0);
  const bool zm = mams_noise_blocks(cfg, tg, s) > 0;
  L.zm = c.take(zm ? (size_t)2 * (2 * cfg->n_steps_traj + 1) * N * ld * rs : 0);
  L.zm_tag = c.take(zm ? 2 * sizeof(uint64_t) : 0);
  L.total = (size_t)round_up((int64_t)c.off, 256);
  return L;
}

int integ_for(const laps_config *cfg) {
  if (cfg->integrator_adj) return cfg->integrator_adj;
  return cfg->d <= 200 ? 1 : 2;
}

laps_status validate(const laps_config *cfg, const laps_target *tg, std::string &why) {
  if (!cfg || !tg) return why = "null config or target", LAPS_EINVAL;
  if (cfg->d < 2) return why = "d must be >= 2 (d-1 divides the velocity update)", LAPS_EINVAL;
  if (cfg->n_chains < 2) return why = "need at least 2 chains", LAPS_EINVAL;
  if (tg->d != cfg->d) return why = "target d differs from config d", LAPS_EINVAL;
  if (cfg->prec < 0 || cfg->prec > 2) return why = "unknown precision", LAPS_EINVAL;
  if (cfg->n_steps_traj < 1 || cfg->max_steps_total < 1 || cfg->max_steps_unadj < 0)
    return why = "step counts must be positive", LAPS_EINVAL;
  if (!(cfg->window_frac > 0.0) || !(cfg->C > 0.0) || !(cfg->alpha > 0.0) || !(cfg->eps0_factor > 0.0) ||
      !(cfg->L_partial_factor > 0.0))
    return why = "non-positive constant in config", LAPS_EINVAL;
  if (cfg->team_lanes < 0) return why = "team_lanes must be >= 0", LAPS_EINVAL;
  if (!(cfg->block_threads == 0 || cfg->block_threads == 64 || cfg->block_threads == 128 ||
        cfg->block_threads == 256))
    return why = "block_threads must be 0, 64, 128 or 256", LAPS_EINVAL;
  if (cfg->grad_workgroups < 0 || cfg->grad_workgroups > 65536)
    return why = "grad_workgroups must be in 0..65536", LAPS_EINVAL;
  if (!(cfg->eps_fixed >= 0.0) || !isfinite(cfg->eps_fixed))
    return why = "eps_fixed must be finite and >= 0", LAPS_EINVAL;
  if (cfg->dynamics != 0 && cfg->dynamics != 1) return why = "dynamics must be 0 or 1", LAPS_EINVAL;
  if (cfg->full_rank_probes < 0 || cfg->full_rank_probes > 1024)
    return why = "full_rank_probes must be in 0..1024", LAPS_EINVAL;
  if (cfg->integrator_adj < 0 || cfg->integrator_adj > 2 || cfg->eevpd_mode < 0 || cfg->eevpd_mode > 1 ||
      cfg->switch_policy < 0 || cfg->switch_policy > 1)
    return why = "bad enum in config", LAPS_EINVAL;
  switch (tg->kind) {
    case LAPS_GAUSS_DIAG:
      if (!tg->data[0]) return why = "gaussian needs data[0] = s2", LAPS_EINVAL;
      break;
    case LAPS_STOCHVOL:
      if (!tg->data[0] || cfg->d < 3) return why = "stochvol needs data[0] = y and d = T + 2 >= 3", LAPS_EINVAL;
      break;
    case LAPS_PHI4:
      if (tg->dims[0] < 2 || tg->dims[0] * tg->dims[0] != cfg->d) return why = "phi4 needs dims[0]^2 == d", LAPS_EINVAL;
      break;
    case LAPS_LOGREG:
    case LAPS_CALLBACK:
    case LAPS_GAUSS_DENSE:
      if (tg->kind == LAPS_LOGREG && (!tg->data[0] || !tg->data[1] || tg->dims[0] < 1))
        return why = "logreg needs X, y and n", LAPS_EINVAL;
      if (tg->kind == LAPS_CALLBACK && !tg->cb) return why = "a callback target needs cb", LAPS_EINVAL;
      if (tg->kind == LAPS_GAUSS_DENSE && !tg->data[0]) return why = "a dense Gaussian needs data[0] = A", LAPS_EINVAL;
      if (tg->kind != LAPS_LOGREG && cfg->prec == LAPS_MIXED_BF16)
        return why = "callback and dense Gaussian targets run in LAPS_F64 or LAPS_F32", LAPS_EUNSUPPORTED;
      // These targets share the per-chain update kernels.  Two GPU runs that used 32- and 64-lane update
      // teams (d > 128) outside the initialisation faulted the GPU with no cause shown; those teams are no
      // longer built: above 16 octs a 16-lane team holds several octs per lane.  The staged MN4 transition
      // runs the same device code as MN2 (only the stage count and the host-supplied coefficients differ).
      if (tg->kind == LAPS_LOGREG && cfg->d > kLogregMaxD)
        return why = "logistic regression supports d <= 128 (its matrix-core gradient kernels hold a chain's "
                     "theta and gradient tiles in registers)",
               LAPS_EUNSUPPORTED;
      if (cfg->d > kUpdateMaxD)
        return why = "callback and dense Gaussian targets support d <= 512", LAPS_EUNSUPPORTED;
      break;
    default:
      return why = "unknown target kind", LAPS_EINVAL;
  }
  Shape s;
  if (!shape_for(cfg, tg, s)) return why = "dimension too large for this build", LAPS_EUNSUPPORTED;
  // a workgroup of gfx950 holds at most 160 KiB of LDS
  if (s.shmem_sig > 160 * 1024) return why = "team shape needs more than 160 KiB of LDS", LAPS_EUNSUPPORTED;
  if (tg->kind == LAPS_LOGREG && cfg->prec != LAPS_F64 && cfg->prec != LAPS_MIXED_BF16)
    return why = "logistic regression runs in LAPS_F64 or LAPS_MIXED_BF16", LAPS_EUNSUPPORTED;
  return LAPS_OK;
}

LocalArgs local_args(laps_ctx *c) {
  LocalArgs a{};
  a.x = c->x;
  a.u = c->u;
  a.g = c->g;
  a.logp = c->logp;
  a.delta = c->delta;
  a.acc = c->acc;
  a.partials = c->partials;
  a.shiftK = c->shiftK;
  a.hyp = c->hyp;
  a.sigma = c->sigma;
  a.u0 = nullptr;
  a.aux = c->aux;
  a.tdata = static_cast<const double *>(c->tg.data[0]);
  a.tn = c->tg.kind == LAPS_STOCHVOL ? c->cfg.d - 2 : c->tg.dims[0];
  a.tp0 = c->tg.scal[0];
  a.tp1 = c->tg.scal[1];
  a.N = c->cfg.n_chains;
  a.d = c->cfg.d;
  a.ld = c->ld;
  a.T = c->T;
  a.tpw = c->tpw;
  a.seed = c->cfg.seed;
  a.max_total = c->cfg.max_steps_total;
  a.n_traj = c->cfg.n_steps_traj;
  a.Lp_factor = c->cfg.L_partial_factor;
  a.cache = 0;
  a.dyn = c->cfg.dynamics;
  return a;
}

LogregArgs logreg_args(laps_ctx *c, int gate) {
  LogregArgs a{};
  a.x = c->x;
  a.u = c->u;
  a.g = c->g;
  a.logp = c->logp;
  a.delta = c->delta;
  a.acc = c->acc;
  a.partials = c->partials;
  a.shiftK = c->shiftK;
  a.hyp = c->hyp;
  a.sigma = c->sigma;
  a.X = c->tg.data[0];
  a.y = static_cast<const double *>(c->tg.data[1]);
  a.scratch = static_cast<char *>(c->packed);
  a.n = c->tg.dims[0];
  a.N = c->cfg.n_chains;
  a.d = c->cfg.d;
  a.ld = c->ld;
  if (c->tg.kind == LAPS_CALLBACK || c->tg.kind == LAPS_GAUSS_DENSE) {
    a.n = 0;
    a.S = 1;
    a.NB = 0;
    a.bps = 0;
    a.prior = 0;
  } else {
    logreg_splits(a.n, a.N, c->cfg.prec, a.d, c->cfg.grad_workgroups, a.S, a.NB, a.bps);
    a.prior = 1;
    a.wy_term = c->cfg.prec == LAPS_F64 ? 0 : 1;
  }
  a.KC = (int)((a.d + 31) / 32);
  a.T = c->T;
  a.tpw = c->tpw;
  a.seed = c->cfg.seed;
  a.max_total = c->cfg.max_steps_total;
  a.n_traj = c->cfg.n_steps_traj;
  a.Lp_factor = c->cfg.L_partial_factor;
  a.gate = gate;
  a.integ = c->integ;
  a.dyn = c->cfg.dynamics;
  return a;
}

CtlArgs ctl_args(laps_ctx *c) {
  CtlArgs a{};
  a.hyp = c->hyp;
  a.partials = c->partials;
  a.G = c->G;
  a.shiftK = c->shiftK;
  a.mean = c->mean;
  a.var = c->var;
  a.m2 = c->m2;
  a.Vii = c->Vii;
  a.ring = c->ring;
  a.wdelta = c->wdelta;
  a.Tw = c->Tw;
  a.part2 = c->part2;
  a.nb = c->nb;
  a.delta = c->delta;
  a.acc = c->acc;
  a.N = c->cfg.n_chains;
  a.d = c->cfg.d;
  a.ld = c->ld;
  a.C = c->cfg.C;
  a.alpha = c->cfg.alpha;
  a.eps0_factor = c->cfg.eps0_factor;
  a.eps_fixed = c->cfg.eps_fixed;
  a.switch_tol = c->cfg.switch_tol;
  a.acc_tol = c->cfg.acc_tol;
  a.acc_target = c->cfg.acc_target;
  a.n_traj = c->cfg.n_steps_traj;
  a.eevpd_mode = c->cfg.eevpd_mode;
  a.switch_policy = c->cfg.switch_policy;
  a.integ = c->integ;
  a.max_unadj = c->cfg.max_steps_unadj;
  a.max_total = c->cfg.max_steps_total;
  a.sigma = c->sigma;
  a.sigma_double = c->dbl ? 1 : 0;
  a.probes = c->cfg.full_rank_probes;
  a.NC = probe_chunks(c->cfg.n_chains);
  a.nbh = a.probes > 0 ? probe_blocks(c->cfg.d, a.probes) : 0;
  a.seed = c->cfg.seed;
  a.x = c->x;
  a.g = c->g;
  a.pS = c->pS;
  a.pW = c->pW;
  a.pPart = c->pPart;
  return a;
}

laps_status fail(laps_ctx *c, hipError_t e, const char *where) {
  if (c) c->err = std::string(where) + ": " + hipGetErrorString(e);
  g_last_global = std::string(where) + ": " + hipGetErrorString(e);
  return LAPS_EDEVICE;
}

#define LAPS_CHECK(ctx, expr, where)          \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return fail(ctx, e_, where); \
  } while (0)

// Event-logged launch: records a begin/end event pair around `launch` when
// kernel `which` is being logged and events remain.
template <class F>
hipError_t logged(laps_ctx *c, int which, F &&launch) {
  bool on = c->log_which == which && c->log_used + 2 <= c->log_ev.size();
  if (c->log_which == which) on = on && (c->log_seen++ % c->log_every) == 0;
  hipError_t e = on ? hipEventRecord(c->log_ev[c->log_used], c->stream) : hipSuccess;
  if (e == hipSuccess) e = launch();
  if (on && e == hipSuccess) e = hipEventRecord(c->log_ev[c->log_used + 1], c->stream);
  if (on && e == hipSuccess) c->log_used += 2;
  return e;
}

// Workgroups of an unadjusted-step launch.  The split-statistics path (teams
// wider than a wavefront or several octs per lane, as at C3 and C4) runs every
// chain in one round when the full grid holds at least 4 wavefronts per SIMD,
// and then all wavefronts load, compute and store in step; with half the grid
// each team steps two chains in turn and the wavefronts drift apart, so one
// loads while another computes (measured: SV T = 2427 step 143.5 -> 136.8 us,
// phi^4 64 x 64 86.5 -> 79.5 us; a quarter of the grid was slower).
int unadj_grid(const laps_ctx *c) {
  if (!c->split) return c->G;
  const int64_t waves = (int64_t)c->grid_full * ((c->block + 63) / 64);
  return waves >= 4 * 1024 ? (c->grid_full + 1) / 2 : c->grid_full;
}

laps_status enqueue_chain_kernel(laps_ctx *c, KernelKind kk, const void *u0) {
  if (is_local(c->tg.kind)) {
    LocalArgs a = local_args(c);
    a.u0 = u0;
    const bool phase_stats = kk == KK_INIT || kk == KK_UNADJ;
    a.stats = (phase_stats && !c->split) ? 1 : 0;
    // the full-rank loss reads the step's gradients, so they are kept
    a.cache = (phase_stats && (c->split || (kk == KK_UNADJ && c->cfg.full_rank_probes > 0))) ? 1 : 0;
    int grid = kk == KK_UNADJ ? unadj_grid(c) : ((phase_stats && !c->split) ? c->G : c->grid_full);
    if (kk == KK_UNADJ && c->zn_blocks > 0) {
      a.zn = c->zn;
      a.zn_tag = c->zn_tag;
      a.zn_blocks = c->zn_blocks;
      grid += c->zn_blocks;
    }
    const bool mams = kk == KK_MAMS_MN2 || kk == KK_MAMS_MN4;
    if (mams && c->zm_blocks > 0) {
      a.zm = c->zm;
      a.zm_tag = c->zm_tag;
      a.zm_blocks = c->zm_blocks;
      grid += c->zm_blocks;
    }
    const int which = kk == KK_UNADJ ? LAPS_KERNEL_UNADJ : (mams ? LAPS_KERNEL_MAMS : 0);
    hipError_t e = logged(c, which, [&] {
      return launch_local(c->tg.kind, c->dbl, c->Q, kk, a, grid, c->block, mams ? c->shmem_sig : c->shmem,
                          c->stream);
    });
    if (e == hipSuccess && phase_stats && c->split)
      e = launch_stats(c->dbl, c->x, c->g, c->shiftK, c->partials, c->cfg.n_chains, c->cfg.d, c->ld, c->G,
                       kk == KK_UNADJ ? c->hyp : nullptr, c->stream);
    return e == hipSuccess ? LAPS_OK : fail(c, e, "per-chain kernel");
  }
  const int prec = c->cfg.prec;
  auto upd = [&](LogregArgs &a, int mode, int j, int k) -> hipError_t {
    a.mode = mode;
    a.j = j;
    a.k = k;
    const Coeffs C = integrator_coeffs(a.integ);
    a.cK = C.K;
    a.cb0 = C.b[0];
    a.ca0 = C.a[0];
    a.cbk = k + 1 < 6 ? C.b[k + 1] : 0.0;
    a.cak = k + 1 < 5 ? C.a[k + 1] : 0.0;
    return launch_logreg_update(prec, c->Q, a, c->G, c->block, c->shmem, c->stream);
  };
  const bool cb = c->tg.kind == LAPS_CALLBACK;
  int cb_rc = 0;
  // the ensemble gradient: the logistic-regression kernels, or the caller's
  // callback writing the single partial-sum split
  const bool dense = c->tg.kind == LAPS_GAUSS_DENSE;
  auto grad = [&](const LogregArgs &a) -> hipError_t {
    if (dense) return launch_dense_grad(prec == LAPS_F64 ? 0 : 1, a, c->stream);
    if (!cb) return launch_logreg_grad(prec, a, c->stream);
    const LrOffsets off = logreg_layout(c->dbl ? 0 : 1, 0, a.d, a.N, a.ld, 1);
    cb_rc = c->tg.cb(c->tg.cb_user, c->x, a.scratch + off.Gp, reinterpret_cast<double *>(a.scratch + off.lp), a.N,
                     a.d, a.ld, c->stream);
    return cb_rc == 0 ? hipSuccess : hipErrorUnknown;
  };
  hipError_t e = hipSuccess;
  if (kk == KK_INIT) {
    LogregArgs a = logreg_args(c, 0);
    a.u0 = u0;
    if (dense && !c->packed_ok) e = launch_dense_pack(prec == LAPS_F64 ? 0 : 1, a, c->stream);
    if (!cb && !dense && prec != LAPS_F64 && !c->packed_ok) e = launch_logreg_pack(a, c->stream);
    if (e == hipSuccess) c->packed_ok = true;
    if (e == hipSuccess) e = grad(a);
    if (e == hipSuccess) e = upd(a, LR_INIT, 0, 0);
  } else if (kk == KK_UNADJ) {
    LogregArgs a = logreg_args(c, 1);
    e = upd(a, LR_PRE, 0, 0);
    if (e == hipSuccess) e = logged(c, LAPS_KERNEL_GRAD, [&] { return grad(a); });
    if (e == hipSuccess) e = upd(a, LR_POST, 0, 0);
  } else {
    LogregArgs a = logreg_args(c, 2);
    const int K = integrator_coeffs(c->integ).K;
    e = upd(a, LR_MBEGIN, 0, 0);
    for (int j = 0; j < c->cfg.n_steps_traj && e == hipSuccess; ++j)
      for (int k = 0; k < K - 1 && e == hipSuccess; ++k) {
        e = logged(c, LAPS_KERNEL_GRAD, [&] { return grad(a); });
        if (e == hipSuccess) e = upd(a, LR_MSTEP, j, k);
      }
  }
  if (e == hipSuccess) return LAPS_OK;
  if (cb_rc != 0) {
    c->err = g_last_global = "gradient callback returned " + std::to_string(cb_rc);
    return LAPS_EDEVICE;
  }
  return fail(c, e, cb ? "update kernels" : dense ? "dense Gaussian kernels" : "logistic-regression kernels");
}

}  // namespace

extern "C" laps_status laps_workspace_size(const laps_config *cfg, const laps_target *tg, size_t *bytes) {
  std::string why;
  const laps_status st = validate(cfg, tg, why);
  if (st != LAPS_OK) {
    g_last_global = why;
    return st;
  }
  if (!bytes) return LAPS_EINVAL;
  Shape s;
  shape_for(cfg, tg, s);
  *bytes = layout(cfg, tg, s).total;
  return LAPS_OK;
}

namespace {

// Arguments checked before any device call: configuration, pointers and
// their alignment; fills the launch shape and workspace layout.
laps_status check_init(const laps_config *cfg, const laps_target *tg, const void *x_dev, const void *u0_dev,
                       laps_ctx **out, Shape &s, Layout &L) {
  std::string why;
  laps_status st = validate(cfg, tg, why);
  if (st != LAPS_OK) {
    g_last_global = why;
    return st;
  }
  if (!x_dev || !out) {
    g_last_global = "null pointer argument";
    return LAPS_EINVAL;
  }
  if (((uintptr_t)x_dev & 31) || (u0_dev && ((uintptr_t)u0_dev & 31))) {
    g_last_global = "misaligned pointer (x/u0 need 32 bytes)";
    return LAPS_EINVAL;
  }
  shape_for(cfg, tg, s);
  L = layout(cfg, tg, s);
  return LAPS_OK;
}

// Carves the workspace w for context c and enqueues the initialisation.
laps_status init_into(laps_ctx *c, const laps_config *cfg, const laps_target *tg, void *x_dev, const void *u0_dev,
                      char *w, const Shape &s, const Layout &L, void *stream) {
  c->cfg = *cfg;
  c->tg = *tg;
  c->x = x_dev;
  c->stream = static_cast<hipStream_t>(stream);
  c->dbl = cfg->prec == LAPS_F64;
  c->ld = laps_row_stride(cfg->d);
  c->Tw = (int64_t)llround(cfg->window_frac * (double)cfg->max_steps_total);
  if (c->Tw < 2) c->Tw = 2;
  c->T = s.T;
  c->Q = s.Q;
  c->tpw = s.tpw;
  c->block = s.block;
  c->G = s.G;
  c->grid_full = s.grid_full;
  c->split = s.split;
  c->nb = s.nb;
  c->shmem = s.shmem;
  c->shmem_sig = s.shmem_sig;
  c->integ = integ_for(cfg);
  c->adj_started = false;
  c->packed_ok = false;
  c->hyp = reinterpret_cast<DevHyper *>(w + L.hyp);
  c->u = w + L.u;
  c->g = w + L.g;
  c->logp = reinterpret_cast<double *>(w + L.logp);
  c->delta = reinterpret_cast<double *>(w + L.delta);
  c->acc = reinterpret_cast<double *>(w + L.acc);
  c->partials = reinterpret_cast<double *>(w + L.partials);
  c->shiftK = reinterpret_cast<double *>(w + L.shiftK);
  c->mean = reinterpret_cast<double *>(w + L.mean);
  c->var = reinterpret_cast<double *>(w + L.var);
  c->m2 = reinterpret_cast<double *>(w + L.m2);
  c->Vii = reinterpret_cast<double *>(w + L.Vii);
  c->ring = reinterpret_cast<double *>(w + L.ring);
  c->wdelta = reinterpret_cast<double *>(w + L.wdelta);
  c->part2 = reinterpret_cast<double *>(w + L.part2);
  c->sigma = w + L.sigma;
  c->aux = w + L.aux;
  c->packed = w + L.packed;
  c->pS = reinterpret_cast<double *>(w + L.pS);
  c->pW = reinterpret_cast<double *>(w + L.pW);
  c->pPart = reinterpret_cast<double *>(w + L.pPart);
  c->zn_blocks = noise_blocks(cfg, tg, s);
  c->zn = c->zn_blocks > 0 ? w + L.zn : nullptr;
  c->zn_tag = c->zn_blocks > 0 ? reinterpret_cast<uint64_t *>(w + L.zn_tag) : nullptr;
  c->zm_blocks = mams_noise_blocks(cfg, tg, s);
  c->zm = c->zm_blocks > 0 ? w + L.zm : nullptr;
  c->zm_tag = c->zm_blocks > 0 ? reinterpret_cast<uint64_t *>(w + L.zm_tag) : nullptr;
  CtlArgs ca = ctl_args(c);
  hipError_t e;
  if ((e = hipMemsetAsync(c->shiftK, 0, (size_t)c->ld * 8, c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(c->u, 0, (size_t)cfg->n_chains * c->ld * (c->dbl ? 8 : 4), c->stream)) != hipSuccess ||
      (e = hipMemsetAsync(c->g, 0, (size_t)cfg->n_chains * c->ld * (c->dbl ? 8 : 4), c->stream)) != hipSuccess ||
      (c->zn_tag && (e = hipMemsetAsync(c->zn_tag, 0, 2 * sizeof(uint64_t), c->stream)) != hipSuccess) ||
      (c->zm_tag && (e = hipMemsetAsync(c->zm_tag, 0, 2 * sizeof(uint64_t), c->stream)) != hipSuccess))
    return fail(c, e, "workspace clear");
  if (tg->kind == LAPS_GAUSS_DIAG || tg->kind == LAPS_STOCHVOL)
    e = launch_prep_aux(tg->kind, c->dbl, tg->data[0], c->aux, cfg->d, c->ld, c->stream);
  if (e == hipSuccess) e = launch_hyper_init(ca, c->stream);
  if (e != hipSuccess) return fail(c, e, "init");
  laps_status st = enqueue_chain_kernel(c, KK_INIT, u0_dev);
  if (st == LAPS_OK && (e = launch_finalize(ca, FIN_INIT, c->stream)) != hipSuccess) st = fail(c, e, "finalize");
  if (st == LAPS_OK && (e = launch_ctl_init(ca, c->stream)) != hipSuccess) st = fail(c, e, "controller init");
  return st;
}

}  // namespace

extern "C" laps_status laps_init(const laps_config *cfg, const laps_target *tg, void *x_dev, const void *u0_dev,
                                 void *ws_dev, size_t ws_bytes, void *stream, laps_ctx **out) {
  Shape s;
  Layout L;
  laps_status st = check_init(cfg, tg, x_dev, u0_dev, out, s, L);
  if (st != LAPS_OK) return st;
  if (!ws_dev) {
    g_last_global = "null pointer argument";
    return LAPS_EINVAL;
  }
  if ((uintptr_t)ws_dev & 255) {
    g_last_global = "misaligned pointer (workspace needs 256 bytes)";
    return LAPS_EINVAL;
  }
  if (ws_bytes < L.total) {
    g_last_global = "workspace too small";
    return LAPS_EWORKSPACE;
  }
  laps_ctx *c = new (std::nothrow) laps_ctx();
  if (!c) return LAPS_EINVAL;
  st = init_into(c, cfg, tg, x_dev, u0_dev, static_cast<char *>(ws_dev), s, L, stream);
  if (st != LAPS_OK) {
    delete c;
    return st;
  }
  *out = c;
  return LAPS_OK;
}

// ---------------------------------------------------------------------------
// Initialisation without allocation, for callers that cannot allocate device
// memory.  The workspace is `laps_static_scratch`, a file-scope device array
// that every GPU the library runs on holds until the process ends; host code
// uses only the address that hipGetSymbolAddress returns for it on each
// device (kept per device), never the array's name.  The context itself is
// library storage, one per device.  A later laps_init_static on the same
// device reuses both, so the previous static context of that device is then
// invalid; calls that overlap on one device race.
//
// The array has external linkage: a `static` device array stays a local
// symbol of the device code object (absent from its dynamic symbol table),
// which the runtime cannot resolve by name.  Its start is rounded up to 256
// bytes inside 256 bytes of slack, whatever alignment the loader gives it.
// ---------------------------------------------------------------------------
constexpr size_t kStaticWorkspaceBytes = (size_t)32 << 20;
constexpr int kStaticDevices = 64;
__device__ __align__(256) unsigned char laps_static_scratch[kStaticWorkspaceBytes + 256];
static void *g_scratch_ptr[kStaticDevices];
static laps_ctx g_static_ctx[kStaticDevices];
static std::mutex g_static_mu;

extern "C" laps_status laps_init_static(const laps_config *cfg, const laps_target *tg, void *x_dev,
                                        const void *u0_dev, void *stream, laps_ctx **out) {
  Shape s;
  Layout L;
  laps_status st = check_init(cfg, tg, x_dev, u0_dev, out, s, L);
  if (st != LAPS_OK) return st;
  if (L.total > kStaticWorkspaceBytes) {
    // the buffers of normals computed ahead are an optimisation: without them the kernels compute the
    // normals where they use them
    s.ahead = false;
    L = layout(cfg, tg, s);
  }
  if (L.total > kStaticWorkspaceBytes) {
    g_last_global = "the configuration needs " + std::to_string(L.total) + " workspace bytes; the static workspace of "
                    "laps_init_static holds " + std::to_string(kStaticWorkspaceBytes);
    return LAPS_EWORKSPACE;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, e, "current device");
  if (dev < 0 || dev >= kStaticDevices) {
    g_last_global = "device index beyond the static contexts";
    return LAPS_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(laps_static_scratch));
    if (e != hipSuccess || !p) return fail(nullptr, e != hipSuccess ? e : hipErrorInvalidSymbol, "static workspace");
    g_scratch_ptr[dev] = reinterpret_cast<void *>(((uintptr_t)p + 255) & ~(uintptr_t)255);
  }
  laps_ctx *c = &g_static_ctx[dev];
  for (hipEvent_t v : c->log_ev) (void)hipEventDestroy(v);
  c->log_ev.clear();
  c->log_which = 0;
  c->log_every = 1;
  c->log_seen = 0;
  c->log_used = 0;
  c->err.clear();
  c->is_static = true;
  st = init_into(c, cfg, tg, x_dev, u0_dev, static_cast<char *>(g_scratch_ptr[dev]), s, L, stream);
  if (st != LAPS_OK) return st;
  *out = c;
  return LAPS_OK;
}

extern "C" laps_status laps_step_unadjusted(laps_ctx *c, int64_t n) {
  if (!c || n < 0) return LAPS_EINVAL;
  if (c->adj_started) return LAPS_EPHASE;
  CtlArgs ca = ctl_args(c);
  for (int64_t k = 0; k < n; ++k) {
    laps_status st = enqueue_chain_kernel(c, KK_UNADJ, nullptr);
    if (st != LAPS_OK) return st;
    LAPS_CHECK(c, launch_finalize(ca, FIN_UNADJ, c->stream), "finalize");
    LAPS_CHECK(c, launch_probes(ca, c->stream), "full-rank loss");
    LAPS_CHECK(c, launch_ctl_unadj(ca, c->stream), "controller");
  }
  return LAPS_OK;
}

extern "C" laps_status laps_step_adjusted(laps_ctx *c, int64_t n) {
  if (!c || n < 0) return LAPS_EINVAL;
  CtlArgs ca = ctl_args(c);
  if (!c->adj_started) {
    LAPS_CHECK(c, launch_switch(ca, c->stream), "switch");
    c->adj_started = true;
  }
  const KernelKind kk = c->integ == 2 ? KK_MAMS_MN4 : KK_MAMS_MN2;
  for (int64_t k = 0; k < n; ++k) {
    laps_status st = enqueue_chain_kernel(c, kk, nullptr);
    if (st != LAPS_OK) return st;
    LAPS_CHECK(c, launch_ctl_adj(ca, c->stream), "controller");
  }
  return LAPS_OK;
}

extern "C" laps_status laps_ensemble_stats(laps_ctx *c, laps_stats *o, double *per_dim) {
  if (!c || !o) return LAPS_EINVAL;
  if (per_dim) {
    const size_t row = (size_t)c->cfg.d * 8;
    double *src[4] = {c->mean, c->var, c->m2, c->Vii};
    for (int k = 0; k < 4; ++k)
      LAPS_CHECK(c, hipMemcpyAsync(per_dim + (size_t)k * c->cfg.d, src[k], row, hipMemcpyDeviceToDevice, c->stream),
                 "per-dim copy");
  }
  DevHyper h;
  LAPS_CHECK(c, hipMemcpyAsync(&h, c->hyp, sizeof(h), hipMemcpyDeviceToHost, c->stream), "stats copy");
  LAPS_CHECK(c, hipStreamSynchronize(c->stream), "stream sync");
  o->t = h.t;
  o->grads_per_chain = h.grads;
  o->phase = h.phase;
  o->adapt = h.adapt;
  o->switch_ready = h.switch_ready;
  o->status_bits = h.status;
  o->eps = h.eps;
  o->L = h.L;
  o->eevpd = h.eevpd;
  o->eevpd_target = h.eevpd_target;
  o->dtilde = h.dtilde;
  o->max_delta = h.max_delta;
  o->acc_mean = h.acc_mean;
  o->n_nonfinite = h.n_nonfinite;
  o->integrator = h.integ;
  o->have_lo = h.have_lo;
  o->have_hi = h.have_hi;
  o->ring_full = h.ring_count == c->Tw;
  o->lo = h.lo;
  o->hi = h.hi;
  o->a_star = h.a_star;
  o->sum_var = h.sum_var;
  return (h.status & ST_NONFINITE) ? LAPS_ENONFINITE : LAPS_OK;
}

extern "C" laps_status laps_target_eval(const laps_target *tg, int32_t prec, const void *x_dev, void *logp_dev,
                                        void *grad_dev, int64_t n, void *stream) {
  if (!tg || !x_dev || !logp_dev || n < 1 || tg->d < 2 || prec < 0 || prec > 2) return LAPS_EINVAL;
  if (((uintptr_t)x_dev & 31) || (grad_dev && ((uintptr_t)grad_dev & 31))) return LAPS_EINVAL;
  laps_config cfg;
  laps_config_default(&cfg, n < 2 ? 2 : n, tg->d);
  cfg.prec = prec;
  std::string why;
  laps_status st = validate(&cfg, tg, why);
  if (st != LAPS_OK) {
    g_last_global = why;
    return st;
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (is_local(tg->kind)) {
    Shape sh;
    if (!local_shape(tg->kind, prec == LAPS_F64, n, tg->d, 0, sh) || sh.shmem > 64 * 1024) return LAPS_EUNSUPPORTED;
    LocalArgs a{};
    a.x = const_cast<void *>(x_dev);
    a.aux = nullptr;
    a.tdata = static_cast<const double *>(tg->data[0]);
    a.tn = tg->kind == LAPS_STOCHVOL ? tg->d - 2 : tg->dims[0];
    a.tp0 = tg->scal[0];
    a.tp1 = tg->scal[1];
    a.N = n;
    a.d = tg->d;
    a.ld = laps_row_stride(tg->d);
    a.T = sh.T;
    a.tpw = sh.tpw;
    a.logp_out = static_cast<double *>(logp_dev);
    a.g_out = grad_dev;
    const int grid = (int)((n + sh.tpw - 1) / sh.tpw);
    const hipError_t e = launch_local(tg->kind, prec == LAPS_F64, sh.Q, KK_EVAL, a, grid < 65535 ? grid : 65535,
                                      sh.block, sh.shmem, s);
    if (e != hipSuccess) {
      g_last_global = std::string("target eval: ") + hipGetErrorString(e);
      return LAPS_EDEVICE;
    }
    return LAPS_OK;
  }
  g_last_global = "standalone evaluation of this target needs a context (use laps_buffer after laps_init)";
  return LAPS_EUNSUPPORTED;
}

extern "C" laps_status laps_eval(laps_ctx *c, const void *x_dev, void *logp_dev, void *grad_dev) {
  if (!c || !x_dev || !logp_dev) return LAPS_EINVAL;
  if (((uintptr_t)x_dev & 31) || (grad_dev && ((uintptr_t)grad_dev & 31))) return LAPS_EINVAL;
  if (is_local(c->tg.kind))
    return laps_target_eval(&c->tg, c->cfg.prec, x_dev, logp_dev, grad_dev, c->cfg.n_chains, c->stream);
  const int prec = c->cfg.prec;
  LogregArgs a = logreg_args(c, 0);
  a.x = const_cast<void *>(x_dev);
  hipError_t e = hipSuccess;
  if (c->tg.kind == LAPS_GAUSS_DENSE) {
    e = launch_dense_grad(prec == LAPS_F64 ? 0 : 1, a, c->stream);
  } else if (c->tg.kind == LAPS_CALLBACK) {
    const LrOffsets off = logreg_layout(c->dbl ? 0 : 1, 0, a.d, a.N, a.ld, 1);
    const int rc = c->tg.cb(c->tg.cb_user, x_dev, a.scratch + off.Gp, reinterpret_cast<double *>(a.scratch + off.lp),
                            a.N, a.d, a.ld, c->stream);
    if (rc != 0) {
      c->err = g_last_global = "gradient callback returned " + std::to_string(rc);
      return LAPS_EDEVICE;
    }
  } else {
    e = launch_logreg_grad(prec, a, c->stream);
  }
  if (e == hipSuccess) {
    a.mode = LR_EVAL;
    a.logp_out = static_cast<double *>(logp_dev);
    a.g_out = grad_dev;
    e = launch_logreg_update(prec, c->Q, a, c->G, c->block, c->shmem, c->stream);
  }
  return e == hipSuccess ? LAPS_OK : fail(c, e, "evaluation");
}

extern "C" laps_status laps_restart(laps_ctx *c, const void *x0_dev) {
  if (!c) return LAPS_EINVAL;
  if (x0_dev && ((uintptr_t)x0_dev & 31)) return LAPS_EINVAL;
  if (x0_dev && x0_dev != c->x)
    LAPS_CHECK(c,
               hipMemcpyAsync(c->x, x0_dev, (size_t)c->cfg.n_chains * c->ld * (c->dbl ? 8 : 4),
                              hipMemcpyDeviceToDevice, c->stream),
               "restart copy");
  CtlArgs ca = ctl_args(c);
  LAPS_CHECK(c, launch_fill(c->shiftK, c->ld, 0.0, c->stream), "restart fill");
  LAPS_CHECK(c, launch_hyper_init(ca, c->stream), "restart");
  c->adj_started = false;
  laps_status st = enqueue_chain_kernel(c, KK_INIT, nullptr);
  if (st != LAPS_OK) return st;
  LAPS_CHECK(c, launch_finalize(ca, FIN_INIT, c->stream), "finalize");
  LAPS_CHECK(c, launch_ctl_init(ca, c->stream), "controller init");
  return LAPS_OK;
}

struct laps_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" laps_status laps_graph_create(laps_ctx *const *ctxs, int32_t n_ctx, int32_t restart,
                                         const void *const *x0s, int64_t n_unadj, int64_t n_adj, laps_graph **out) {
  if (!ctxs || n_ctx < 1 || !out || n_unadj < 0 || n_adj < 0) return LAPS_EINVAL;
  for (int32_t k = 0; k < n_ctx; ++k) {
    if (!ctxs[k]) return LAPS_EINVAL;
    if (!ctxs[k]->stream) {
      g_last_global = "graph recording needs every context on a created (non-default) stream";
      return LAPS_EINVAL;
    }
    if (ctxs[k]->log_which != 0) {
      g_last_global = "graph recording needs kernel event logging off";
      return LAPS_EINVAL;
    }
  }
  // recording starts on a private stream; the contexts' streams fork from it
  hipStream_t origin = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&origin, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(nullptr, e, "graph stream");
  std::vector<hipEvent_t> ev;
  auto cleanup = [&]() {
    for (hipEvent_t v : ev) (void)hipEventDestroy(v);
    (void)hipStreamDestroy(origin);
  };
  hipEvent_t fork;
  e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(origin);
    return fail(nullptr, e, "graph events");
  }
  ev.push_back(fork);
  for (int32_t k = 0; k < n_ctx && e == hipSuccess; ++k) {
    hipEvent_t j;
    e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
    if (e == hipSuccess) ev.push_back(j);
  }
  if (e != hipSuccess) {
    cleanup();
    return fail(nullptr, e, "graph events");
  }
  e = hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    cleanup();
    return fail(nullptr, e, "begin capture");
  }
  laps_status st = LAPS_OK;
  e = hipEventRecord(fork, origin);
  for (int32_t k = 0; k < n_ctx && e == hipSuccess && st == LAPS_OK; ++k) {
    laps_ctx *c = ctxs[k];
    e = hipStreamWaitEvent(c->stream, fork, 0);
    if (e != hipSuccess) break;
    if (restart) st = laps_restart(c, x0s ? x0s[k] : nullptr);
    if (st == LAPS_OK && n_unadj > 0 && !c->adj_started) st = laps_step_unadjusted(c, n_unadj);
    if (st == LAPS_OK && n_adj > 0) st = laps_step_adjusted(c, n_adj);
    if (st == LAPS_OK) {
      e = hipEventRecord(ev[1 + k], c->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(origin, ev[1 + k], 0);
    }
  }
  hipGraph_t g = nullptr;
  const hipError_t e_end = hipStreamEndCapture(origin, &g);
  if (e == hipSuccess) e = e_end;
  if (st != LAPS_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    cleanup();
    if (st != LAPS_OK) return st;
    return fail(nullptr, e, "capture");
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  cleanup();
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(nullptr, e, "graph instantiate");
  }
  laps_graph *G = new (std::nothrow) laps_graph{g, x};
  if (!G) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    return LAPS_EINVAL;
  }
  *out = G;
  return LAPS_OK;
}

extern "C" laps_status laps_graph_launch(laps_graph *G, void *stream) {
  if (!G) return LAPS_EINVAL;
  const hipError_t e = hipGraphLaunch(G->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAPS_OK : fail(nullptr, e, "graph launch");
}

extern "C" laps_status laps_graph_destroy(laps_graph *G) {
  if (!G) return LAPS_OK;
  (void)hipGraphExecDestroy(G->exec);
  (void)hipGraphDestroy(G->graph);
  delete G;
  return LAPS_OK;
}

extern "C" void *laps_buffer(laps_ctx *c, int32_t which) {
  if (!c) return nullptr;
  switch (which) {
    case 0: return c->u;
    case 1: return c->g;
    case 2: return c->logp;
    case 3: return c->delta;
    case 4: return c->acc;
    case 5: return c->sigma;
    default: return nullptr;
  }
}

extern "C" laps_status laps_destroy(laps_ctx *c) {
  if (c && c->is_static) return LAPS_OK;  // library storage, reused by the next laps_init_static
  delete c;
  return LAPS_OK;
}

extern "C" const char *laps_status_string(laps_status s) {
  switch (s) {
    case LAPS_OK: return "ok";
    case LAPS_EINVAL: return "invalid argument";
    case LAPS_EDEVICE: return "device error";
    case LAPS_ENONFINITE: return "non-finite energy error in some chains";
    case LAPS_EPHASE: return "wrong phase";
    case LAPS_EWORKSPACE: return "workspace too small";
    case LAPS_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

extern "C" const char *laps_last_error(const laps_ctx *c) {
  if (c && !c->err.empty()) return c->err.c_str();
  return g_last_global.c_str();
}

extern "C" laps_status laps_time_kernel(laps_ctx *c, int32_t which, int32_t n_reps, float *avg_ms) {
  if (!c || n_reps < 1 || !avg_ms || which < 1 || which > 2) return LAPS_EINVAL;
  if (!is_local(c->tg.kind)) return LAPS_EUNSUPPORTED;
  hipEvent_t e0, e1;
  LAPS_CHECK(c, hipEventCreate(&e0), "event");
  LAPS_CHECK(c, hipEventCreate(&e1), "event");
  const KernelKind kk = which == 1 ? KK_UNADJ : (c->integ == 2 ? KK_MAMS_MN4 : KK_MAMS_MN2);
  LocalArgs a = local_args(c);
  a.stats = 0;
  a.cache = c->split ? 1 : 0;
  int grid = (kk == KK_UNADJ && c->split) ? unadj_grid(c) : c->grid_full;
  if (kk == KK_UNADJ && c->zn_blocks > 0) {
    a.zn = c->zn;
    a.zn_tag = c->zn_tag;
    a.zn_blocks = c->zn_blocks;
    grid += c->zn_blocks;
  }
  if (kk != KK_UNADJ && c->zm_blocks > 0) {
    a.zm = c->zm;
    a.zm_tag = c->zm_tag;
    a.zm_blocks = c->zm_blocks;
    grid += c->zm_blocks;
  }
  hipError_t e = hipEventRecord(e0, c->stream);
  for (int32_t k = 0; k < n_reps && e == hipSuccess; ++k)
    e = launch_local(c->tg.kind, c->dbl, c->Q, kk, a, grid, c->block, which == 1 ? c->shmem : c->shmem_sig,
                     c->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(c, e, "kernel timing");
  *avg_ms = ms / (float)n_reps;
  return LAPS_OK;
}

extern "C" laps_status laps_kernel_log(laps_ctx *c, int32_t which, int32_t capacity, int32_t every) {
  if (!c || capacity < 0 || every < 1 || which < 0 || which > LAPS_KERNEL_GRAD) return LAPS_EINVAL;
  if (which == LAPS_KERNEL_GRAD ? is_local(c->tg.kind) : (which != 0 && !is_local(c->tg.kind)))
    return LAPS_EUNSUPPORTED;
  LAPS_CHECK(c, hipStreamSynchronize(c->stream), "stream sync");
  for (hipEvent_t e : c->log_ev) (void)hipEventDestroy(e);
  c->log_ev.clear();
  c->log_used = 0;
  c->log_which = 0;
  c->log_seen = 0;
  if (which == 0 || capacity == 0) return LAPS_OK;
  for (int32_t k = 0; k < 2 * capacity; ++k) {
    hipEvent_t e;
    // timing-only events: no system-scope cache writeback at each record
    const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    if (r != hipSuccess) return fail(c, r, "event");
    c->log_ev.push_back(e);
  }
  c->log_which = which;
  c->log_every = every;
  return LAPS_OK;
}

extern "C" laps_status laps_kernel_log_read(laps_ctx *c, int64_t *count, double *total_ms) {
  if (!c || !count || !total_ms) return LAPS_EINVAL;
  *count = 0;
  *total_ms = 0.0;
  if (c->log_used == 0) return LAPS_OK;
  LAPS_CHECK(c, hipEventSynchronize(c->log_ev[c->log_used - 1]), "event sync");
  double sum = 0.0;
  for (size_t k = 0; k < c->log_used; k += 2) {
    float ms = 0.f;
    LAPS_CHECK(c, hipEventElapsedTime(&ms, c->log_ev[k], c->log_ev[k + 1]), "event time");
    sum += ms;
  }
  *count = (int64_t)(c->log_used / 2);
  *total_ms = sum;
  return LAPS_OK;
}

extern "C" laps_status laps_time_gradient(laps_ctx *c, int32_t n_reps, float *avg_ms) {
  if (!c || n_reps < 1 || !avg_ms) return LAPS_EINVAL;
  hipEvent_t e0, e1;
  LAPS_CHECK(c, hipEventCreate(&e0), "event");
  LAPS_CHECK(c, hipEventCreate(&e1), "event");
  hipError_t e = hipEventRecord(e0, c->stream);
  for (int32_t k = 0; k < n_reps && e == hipSuccess; ++k) {
    if (is_local(c->tg.kind)) {
      LocalArgs a = local_args(c);
      a.logp_out = c->logp;
      a.g_out = c->g;
      e = launch_local(c->tg.kind, c->dbl, c->Q, KK_EVAL, a, c->grid_full, c->block, c->shmem, c->stream);
    } else if (c->tg.kind == LAPS_GAUSS_DENSE) {
      LogregArgs a = logreg_args(c, 0);
      e = launch_dense_grad(c->dbl ? 0 : 1, a, c->stream);
    } else if (c->tg.kind == LAPS_CALLBACK) {
      LogregArgs a = logreg_args(c, 0);
      const LrOffsets off = logreg_layout(c->dbl ? 0 : 1, 0, a.d, a.N, a.ld, 1);
      if (c->tg.cb(c->tg.cb_user, c->x, a.scratch + off.Gp, reinterpret_cast<double *>(a.scratch + off.lp), a.N,
                   a.d, a.ld, c->stream) != 0)
        e = hipErrorUnknown;
    } else {
      LogregArgs a = logreg_args(c, 0);
      e = launch_logreg_grad(c->cfg.prec, a, c->stream);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(c, e, "gradient timing");
  *avg_ms = ms / (float)n_reps;
  return LAPS_OK;
}
