"""Ablation sweeps of the hyperparameters and of the dynamics (appendix
"Ablation studies" and the step-size comparison of the appendix on the adaptive
step size) on targets with closed-form second moments, run through the
library's sampler.

The paper's metric is the number of gradient calls per chain until the squared
bias of the second moments first drops below 0.01 (b^2_max; b^2_avg for the
sweep over the number of chains M), reported relative to the best point of each
grid.  b^2_i = (E_M[x_i^2] - s2_i)^2 / (2 s2_i^2), with s2_i the target's exact
variance of x_i (section "Bias" of the benchmarks): the diagonal Gaussian gives
s2 directly, the rotated ill-conditioned one the diagonal of its covariance.

Every configuration is an independent run of the product path; b^2 is taken
with torch from the positions after each unadjusted step and each MAMS
transition (measurement only, outside the method).

    python -m paper_2601_16696_amd.ablation --target gauss --out sweeps.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import laps, workloads

THRESHOLD = 0.01


def _target(name: str, n_chains: int = 1024):
    if name == "gauss":
        w = workloads.gaussian(n_chains=n_chains)
        return w, w["sigma2"]
    if name == "ill":
        w = workloads.ill_gaussian(n_chains=n_chains)
        return w, w["cov_diag"]
    raise ValueError(f"unknown target {name}")


def grads_to_bias(w: dict, s2, prec="f64", threshold: float = THRESHOLD, which: str = "max",
                  max_unadj: int = 1000, max_total: int = 4000, unadjusted_only: bool = False,
                  stop_at_hit: bool = True, **cfg) -> dict:
    """One LAPS run of workload w, stepped one unadjusted step / one MAMS
    transition at a time; returns the first point where b^2_<which> drops
    below threshold (gradients per chain, steps of each phase), the smallest
    b^2 seen, and the run's final step size.  unadjusted_only keeps the run in
    the unadjusted phase (no switch)."""
    torch = laps._torch()
    c = dict(switch_policy=0, max_steps_unadj=max_unadj, max_steps_total=max_total)
    if unadjusted_only:
        c.update(switch_policy=1, max_steps_unadj=max_total)
    c.update(cfg)
    s = laps.Sampler(w, prec, **c)
    s2t = torch.as_tensor(np.asarray(s2), device=s.x.device, dtype=torch.float64)

    def b2():
        x = s.positions().to(torch.float64)
        b = ((x * x).mean(0) - s2t) ** 2 / (2.0 * s2t * s2t)
        v = torch.stack([b.max(), b.mean()]).cpu().numpy()
        return float(v[0]), float(v[1])

    col = 0 if which == "max" else 1
    n_u = n_a = 0
    hit = None
    best = math.inf
    switch = None
    while True:
        st = s.stats()
        if st["t"] >= c["max_steps_total"]:
            break
        if st["phase"] == 0:
            if unadjusted_only and n_u >= c["max_steps_unadj"]:
                break
            s.step_unadjusted(1)
            n_u += 1
        else:
            if unadjusted_only:
                break
            if switch is None:
                switch = dict(grads_per_chain=st["grads_per_chain"], eps=st["eps"], t=st["t"])
            s.step_adjusted(1)
            n_a += 1
        v = b2()
        best = min(best, v[col])
        if hit is None and v[col] < threshold:
            st = s.stats()
            hit = dict(grads_per_chain=int(st["grads_per_chain"]), n_unadj=n_u, n_adj=n_a, phase=int(st["phase"]))
            if stop_at_hit:
                break
    st = s.stats()
    out = dict(reached=hit is not None, min_b2=best, final_eps=st["eps"], final_grads=int(st["grads_per_chain"]),
               switch=switch)
    if hit:
        out.update(hit)
    del s
    return out


def _relative(rows: list) -> list:
    done = [r["grads_per_chain"] for r in rows if r["reached"]]
    best = min(done) if done else None
    for r in rows:
        r["relative"] = (r["grads_per_chain"] / best) if (best and r["reached"]) else None
    return rows


def sweep(target: str = "gauss", prec="f64", log=None) -> dict:
    """The grids of the ablation appendix on one closed-form target (the
    defaults C = 0.025, alpha = 2, acceptance 0.7 / 0.9, 15 steps per
    trajectory, automatic switch, M = 1024 are in every grid)."""
    w, s2 = _target(target)
    out = {"target": w["name"], "precision": prec, "threshold": THRESHOLD}

    def run(label, **kw):
        t0 = time.perf_counter()
        try:
            r = grads_to_bias(kw.pop("w", w), kw.pop("s2", s2), prec, **kw)
        except laps.LapsError as e:  # a configuration the library refuses for this target
            r = dict(reached=False, min_b2=math.nan, refused=str(e))
        r["seconds"] = time.perf_counter() - t0
        if log:
            print(f"{target} {label}: {r.get('grads_per_chain')} grads (reached {r['reached']}, "
                  f"min b2 {r['min_b2']:.3g})", file=log, flush=True)
        return r

    out["C"] = _relative([dict(C=v, **run(f"C={v}", C=v)) for v in (0.005, 0.01, 0.025, 0.05, 0.1, 0.2)])
    out["alpha"] = _relative([dict(alpha=v, **run(f"alpha={v}", alpha=v)) for v in (0.5, 1.0, 2.0, 4.0, 8.0)])
    acc = []
    for integ, name in ((1, "MN2"), (2, "MN4")):
        for a in (0.5, 0.6, 0.7, 0.8, 0.9, 0.95):
            acc.append(dict(integrator=name, acc_target=a,
                            **run(f"{name} a*={a}", integrator_adj=integ, acc_target=a)))
    out["acc_target"] = _relative(acc)
    out["steps_per_trajectory"] = _relative([dict(n_steps_traj=v, **run(f"traj={v}", n_steps_traj=v))
                                             for v in (5, 10, 15, 20, 30)])
    unadj = [dict(max_steps_unadj="automatic", **run("switch=auto"))]
    for n in (10, 50, 100, 200, 500, 1000):
        unadj.append(dict(max_steps_unadj=n, **run(f"switch@{n}", switch_policy=1, max_unadj=n)))
    out["unadjusted_steps"] = _relative(unadj)
    chains = []
    for M in (64, 128, 256, 512, 1024, 2048, 4096):
        wm, s2m = _target(target, n_chains=M)
        chains.append(dict(n_chains=M, **run(f"M={M}", w=wm, s2=s2m, which="avg")))
    out["n_chains"] = _relative(chains)
    # adaptive vs fixed step size, unadjusted dynamics only
    ref = run("adaptive (unadjusted only)", unadjusted_only=True, max_total=2000, stop_at_hit=False)
    eps_ref = ref["final_eps"]
    fixed = [dict(eps="adaptive", **ref)]
    for f in (0.25, 0.5, 1.0, 2.0, 4.0):
        fixed.append(dict(eps=f * eps_ref, eps_over_adaptive_final=f,
                          **run(f"eps={f}x", unadjusted_only=True, max_total=2000, stop_at_hit=False,
                                eps_fixed=f * eps_ref)))
    out["fixed_eps"] = _relative(fixed)
    # microcanonical vs underdamped Langevin dynamics, the rest of the scheme unchanged
    out["dynamics"] = _relative([dict(dynamics=name, **run(f"dynamics={name}", dynamics=v))
                                 for v, name in ((0, "microcanonical"), (1, "langevin"))])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--target", default="gauss", choices=["gauss", "ill"])
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"])
    ap.add_argument("--out", default=None, help="JSON file for the results (default: stdout)")
    a = ap.parse_args(argv)
    laps.lib()
    res = sweep(a.target, a.prec, log=sys.stderr)
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    else:
        print(text)


if __name__ == "__main__":
    main()
