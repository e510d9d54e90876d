"""Reference second moments of the stochastic-volatility posterior (the
benchmark's synthetic series: T = 2427, d = 2429) for the bias metric of
section "Bias" (b^2 = (E[x_i^2] - E_p[x_i^2])^2 / Var_p[x_i^2]), written by the
FP64 oracle only.

Eight independent oracle ensembles (128 chains each, own seeds) run the full
method: the unadjusted phase with the automatic switch, then MAMS transitions
(MN4, since d > 200); after 100 transitions of burn-in, the positions of the
next 200 transitions are pooled.  E_p[x_i^2] and Var_p[x_i^2] come from the
pooled samples, their Monte Carlo standard errors from the spread of the
eight ensembles' estimates.  As a stationarity check, the estimates from the
first and the second 100 kept transitions are compared.

The two hyperparameters s and r mix slowly.  Longer oracle runs settle at
E[s^2] = 7.17-7.18 (7.08 here), while 4096-chain ensembles settle near 7.6,
so the reference is not used to time the bias.

    python tests/golden/stochvol_moments.py   # ~15 minutes on 8 cores
writes tests/golden/stochvol_T2427_moments.json.
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N_WORKERS, CHAINS, BURN, KEEP = 8, 128, 100, 200
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stochvol_T2427_moments.json")


def _worker(k):
    from oracle import oracle as orc
    from paper_2601_16696_amd import workloads
    w = workloads.stochvol()
    x0 = np.asarray(w["x0"])[k * CHAINS:(k + 1) * CHAINS]
    e = orc.Ensemble(orc.Target.from_workload(w), CHAINS, 7000 + k,
                     max_steps_unadj=1000, max_steps_total=1000 + 15 * (BURN + KEEP + 5))
    e.init(x0)
    e.step_unadjusted(1000)
    n_unadj = int(e.stats()["t"])
    e.do_switch()
    d = w["d"]
    s2 = np.zeros((2, d))
    s4 = np.zeros((2, d))
    acc = []
    for j in range(BURN + KEEP):
        e.step_adjusted(1)
        acc.append(e.stats()["acc_mean"])
        if j >= BURN:
            half = 0 if j < BURN + KEEP // 2 else 1
            x2 = e.array("x") ** 2
            s2[half] += x2.sum(0)
            s4[half] += (x2 * x2).sum(0)
    n = CHAINS * KEEP // 2
    return s2 / n, s4 / n, float(np.mean(acc[BURN:])), n_unadj


def main():
    with Pool(N_WORKERS) as p:
        res = p.map(_worker, range(N_WORKERS))
    m2 = np.array([r[0] for r in res])  # [worker][half][d]
    m4 = np.array([r[1] for r in res])
    e2 = m2.mean((0, 1))
    var2 = m4.mean((0, 1)) - e2 ** 2
    per_worker = m2.mean(1)
    se = per_worker.std(0, ddof=1) / np.sqrt(N_WORKERS)
    halves = m2.mean(0)  # [half][d]
    se_half = m2.std(0, ddof=1) / np.sqrt(N_WORKERS)
    z_halves = np.abs(halves[0] - halves[1]) / np.sqrt(se_half[0] ** 2 + se_half[1] ** 2)
    out = dict(
        workload="stochvol_T2427 (workloads.stochvol defaults)",
        source="FP64 oracle, %d ensembles x %d chains, automatic switch, %d burn-in + %d pooled MAMS transitions each"
               % (N_WORKERS, CHAINS, BURN, KEEP),
        E_x2=e2.tolist(), Var_x2=var2.tolist(), se_E_x2=se.tolist(),
        max_se_over_std=float(np.max(se / np.sqrt(var2))),
        halves_z_median=float(np.median(z_halves)), halves_z_max=float(np.max(z_halves)),
        acceptance=[r[2] for r in res], unadjusted_steps=[r[3] for r in res])
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, "max se/std", out["max_se_over_std"], "halves z median/max",
          out["halves_z_median"], out["halves_z_max"], "acc", out["acceptance"], "switch at", out["unadjusted_steps"])


if __name__ == "__main__":
    main()
