"""Reference second moments of the logistic-regression posterior (the
benchmark's synthetic data set: X 5000 x 100, N(0, I) prior) for the bias
metric of section "Bias" (b^2 = (E[x_i^2] - E_p[x_i^2])^2 / Var_p[x_i^2]),
written by the FP64 oracle only.

Eight independent oracle ensembles (64 chains each, own seeds) run the full
method: the unadjusted phase with the automatic switch, then MAMS transitions;
after 20 transitions of burn-in (the step-size bisection settles within a
few), the positions of the next 60 transitions are pooled.  E_p[x_i^2] and
Var_p[x_i^2] come from the pooled samples; the spread of the eight
ensembles' estimates gives their Monte Carlo standard errors.

    python tests/golden/logreg_moments.py   # ~2 minutes on 8 cores
writes tests/golden/logreg_n5000_d100_moments.json.
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N_WORKERS, CHAINS, BURN, KEEP = 8, 64, 20, 60
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "logreg_n5000_d100_moments.json")


def _worker(k):
    from oracle import oracle as orc
    from paper_2601_16696_amd import workloads
    w = workloads.logreg()
    x0 = np.asarray(w["x0"])[k * CHAINS:(k + 1) * CHAINS]
    e = orc.Ensemble(orc.Target.from_workload(w), CHAINS, 5000 + k,
                     max_steps_unadj=1000, max_steps_total=1000 + 15 * (BURN + KEEP + 5))
    e.init(x0)
    e.step_unadjusted(1000)
    e.do_switch()
    s2 = np.zeros(w["d"])
    s4 = np.zeros(w["d"])
    acc = []
    for j in range(BURN + KEEP):
        e.step_adjusted(1)
        acc.append(e.stats()["acc_mean"])
        if j >= BURN:
            x2 = e.array("x") ** 2
            s2 += x2.sum(0)
            s4 += (x2 * x2).sum(0)
    n = CHAINS * KEEP
    return s2 / n, s4 / n, float(np.mean(acc[BURN:])), int(e.stats()["grads_per_chain"])


def main():
    with Pool(N_WORKERS) as p:
        res = p.map(_worker, range(N_WORKERS))
    m2 = np.array([r[0] for r in res])
    m4 = np.array([r[1] for r in res])
    e2 = m2.mean(0)
    var2 = m4.mean(0) - e2 ** 2
    se = m2.std(0, ddof=1) / np.sqrt(N_WORKERS)
    out = dict(
        workload="logreg_n5000_d100 (workloads.logreg defaults)",
        source="FP64 oracle, %d ensembles x %d chains, %d burn-in + %d pooled MAMS transitions each"
               % (N_WORKERS, CHAINS, BURN, KEEP),
        E_x2=e2.tolist(), Var_x2=var2.tolist(), se_E_x2=se.tolist(),
        max_se_over_std=float(np.max(se / np.sqrt(var2))),
        acceptance=[r[2] for r in res], grads_per_chain=res[0][3])
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT, "max se/std", out["max_se_over_std"])


if __name__ == "__main__":
    main()
