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
transition (measurement only, outside the method).  By default the grid
points run as one batched workload: up to 16 samplers advance together, each
on its own stream, one move per round.

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


class _Run:
    """One configuration of a batched sweep: its own sampler on its own stream,
    advanced one unadjusted step or MAMS transition per round with the same
    decisions as grads_to_bias (the run is deterministic, so its results equal
    the sequential driver's)."""

    def __init__(self, w, s2, prec, threshold=THRESHOLD, which="max", max_unadj=1000, max_total=4000,
                 unadjusted_only=False, stop_at_hit=True, **cfg):
        torch = laps._torch()
        self.c = dict(switch_policy=0, max_steps_unadj=max_unadj, max_steps_total=max_total)
        if unadjusted_only:
            self.c.update(switch_policy=1, max_steps_unadj=max_total)
        self.c.update(cfg)
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.s = laps.Sampler(w, prec, **self.c)
            self.s2t = torch.as_tensor(np.asarray(s2), device=self.s.x.device, dtype=torch.float64)
        self.threshold, self.col = threshold, 0 if which == "max" else 1
        self.unadjusted_only, self.stop_at_hit = unadjusted_only, stop_at_hit
        self.n_u = self.n_a = 0
        self.hit, self.switch, self.best = None, None, math.inf
        self.st = self.s.stats()
        self.done = False
        self.pending = None

    def issue(self):
        """Enqueues the next move and its bias on the run's stream (no host sync)."""
        torch = laps._torch()
        st = self.st
        if st["t"] >= self.c["max_steps_total"]:
            self.done = True
            return
        if st["phase"] == 0:
            if self.unadjusted_only and self.n_u >= self.c["max_steps_unadj"]:
                self.done = True
                return
            self.s.step_unadjusted(1)
            self.n_u += 1
        else:
            if self.unadjusted_only:
                self.done = True
                return
            if self.switch is None:
                self.switch = dict(grads_per_chain=st["grads_per_chain"], eps=st["eps"], t=st["t"])
            self.s.step_adjusted(1)
            self.n_a += 1
        with torch.cuda.stream(self.stream):
            x = self.s.positions().to(torch.float64)
            b = ((x * x).mean(0) - self.s2t) ** 2 / (2.0 * self.s2t * self.s2t)
            self.pending = torch.stack([b.max(), b.mean()])

    def collect(self):
        """Reads the bias of the move just issued and decides whether the run goes on."""
        if self.done or self.pending is None:
            return
        torch = laps._torch()
        with torch.cuda.stream(self.stream):  # the copy waits for the run's stream, not the default one
            v = self.pending.cpu().numpy()
        self.pending = None
        self.best = min(self.best, float(v[self.col]))
        self.st = self.s.stats()
        if self.hit is None and float(v[self.col]) < self.threshold:
            self.hit = dict(grads_per_chain=int(self.st["grads_per_chain"]), n_unadj=self.n_u, n_adj=self.n_a,
                            phase=int(self.st["phase"]))
            if self.stop_at_hit:
                self.done = True

    def result(self) -> dict:
        st = self.s.stats()
        out = dict(reached=self.hit is not None, min_b2=self.best, final_eps=st["eps"],
                   final_grads=int(st["grads_per_chain"]), switch=self.switch)
        if self.hit:
            out.update(self.hit)
        return out


def grads_to_bias_many(specs: list, prec="f64", concurrent: int = 16) -> list:
    """grads_to_bias for many configurations at once: up to `concurrent` runs
    advance together, each on its own stream, one move per round, and the host
    waits once per round for all of them.  specs: dicts of grads_to_bias'
    arguments (w, s2 and the keyword arguments).  A configuration the library
    refuses gives dict(reached=False, min_b2=nan, refused=message)."""
    torch = laps._torch()
    results = [None] * len(specs)
    for lo in range(0, len(specs), concurrent):
        runs = {}
        for k in range(lo, min(lo + concurrent, len(specs))):
            sp = dict(specs[k])
            try:
                runs[k] = _Run(sp.pop("w"), sp.pop("s2"), prec, **sp)
            except laps.LapsError as e:
                results[k] = dict(reached=False, min_b2=math.nan, refused=str(e))
        active = list(runs.values())
        while active:
            for r in active:
                r.issue()
            for r in active:
                r.collect()
            active = [r for r in active if not r.done]
        for k, r in runs.items():
            results[k] = r.result()
        del runs, active
        torch.cuda.synchronize()
    return results


def _relative(rows: list) -> list:
    done = [r["grads_per_chain"] for r in rows if r["reached"]]
    best = min(done) if done else None
    for r in rows:
        r["relative"] = (r["grads_per_chain"] / best) if (best and r["reached"]) else None
    return rows


def sweep(target: str = "gauss", prec="f64", log=None, batched: bool = True) -> dict:
    """The grids of the ablation appendix on one closed-form target (the
    defaults C = 0.025, alpha = 2, acceptance 0.7 / 0.9, 15 steps per
    trajectory, automatic switch, M = 1024 are in every grid).  batched runs
    the grid points together (grads_to_bias_many); otherwise one after the
    other (grads_to_bias); the results are the same."""
    w, s2 = _target(target)
    out = {"target": w["name"], "precision": prec, "threshold": THRESHOLD, "batched": batched}
    t_all = time.perf_counter()

    def run_all(items):
        """items: (label, row fields, grads_to_bias keyword arguments); returns the rows."""
        specs = []
        for _, _, kw in items:
            kw = dict(kw)
            specs.append(dict(w=kw.pop("w", w), s2=kw.pop("s2", s2), **kw))
        if batched:
            res = grads_to_bias_many(specs, prec)
        else:
            res = []
            for sp in specs:
                sp = dict(sp)
                t0 = time.perf_counter()
                try:
                    r = grads_to_bias(sp.pop("w"), sp.pop("s2"), prec, **sp)
                except laps.LapsError as e:  # a configuration the library refuses for this target
                    r = dict(reached=False, min_b2=math.nan, refused=str(e))
                r["seconds"] = time.perf_counter() - t0
                res.append(r)
        rows = []
        for (label, fields, _), r in zip(items, res):
            if log:
                print(f"{target} {label}: {r.get('grads_per_chain')} grads (reached {r['reached']}, "
                      f"min b2 {r['min_b2']:.3g})", file=log, flush=True)
            rows.append(dict(fields, **r))
        return rows

    groups = {}
    items = []

    def add(group, label, fields, **kw):
        groups.setdefault(group, []).append(len(items))
        items.append((label, fields, kw))

    for v in (0.005, 0.01, 0.025, 0.05, 0.1, 0.2):
        add("C", f"C={v}", dict(C=v), C=v)
    for v in (0.5, 1.0, 2.0, 4.0, 8.0):
        add("alpha", f"alpha={v}", dict(alpha=v), alpha=v)
    for integ, name in ((1, "MN2"), (2, "MN4")):
        for a in (0.5, 0.6, 0.7, 0.8, 0.9, 0.95):
            add("acc_target", f"{name} a*={a}", dict(integrator=name, acc_target=a), integrator_adj=integ,
                acc_target=a)
    for v in (5, 10, 15, 20, 30):
        add("steps_per_trajectory", f"traj={v}", dict(n_steps_traj=v), n_steps_traj=v)
    add("unadjusted_steps", "switch=auto", dict(max_steps_unadj="automatic"))
    for n in (10, 50, 100, 200, 500, 1000):
        add("unadjusted_steps", f"switch@{n}", dict(max_steps_unadj=n), switch_policy=1, max_unadj=n)
    for M in (64, 128, 256, 512, 1024, 2048, 4096):
        wm, s2m = _target(target, n_chains=M)
        add("n_chains", f"M={M}", dict(n_chains=M), w=wm, s2=s2m, which="avg")
    # microcanonical vs underdamped Langevin dynamics, the rest of the scheme unchanged
    for v, name in ((0, "microcanonical"), (1, "langevin")):
        add("dynamics", f"dynamics={name}", dict(dynamics=name), dynamics=v)
    # adaptive vs fixed step size, unadjusted dynamics only (the fixed values need the adaptive run's final eps)
    add("fixed_eps", "adaptive (unadjusted only)", dict(eps="adaptive"), unadjusted_only=True, max_total=2000,
        stop_at_hit=False)
    rows = run_all(items)
    for g, idx in groups.items():
        out[g] = [rows[i] for i in idx]
    eps_ref = out["fixed_eps"][0]["final_eps"]
    fixed = [(f"eps={f}x", dict(eps=f * eps_ref, eps_over_adaptive_final=f),
              dict(unadjusted_only=True, max_total=2000, stop_at_hit=False, eps_fixed=f * eps_ref))
             for f in (0.25, 0.5, 1.0, 2.0, 4.0)]
    out["fixed_eps"] += run_all(fixed)
    for g in ("C", "alpha", "acc_target", "steps_per_trajectory", "unadjusted_steps", "n_chains", "fixed_eps",
              "dynamics"):
        out[g] = _relative(out[g])
    out["wall_seconds"] = time.perf_counter() - t_all
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--target", default="gauss", choices=["gauss", "ill"])
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"])
    ap.add_argument("--out", default=None, help="JSON file for the results (default: stdout)")
    ap.add_argument("--sequential", action="store_true", help="one configuration after the other")
    a = ap.parse_args(argv)
    laps.lib()
    res = sweep(a.target, a.prec, log=sys.stderr, batched=not a.sequential)
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    else:
        print(text)


if __name__ == "__main__":
    main()
