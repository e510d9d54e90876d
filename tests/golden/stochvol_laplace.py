"""Reference second moments of the stochastic-volatility posterior (the
benchmark's synthetic series: T = 2427, d = 2429) for the bias metric of
section "Bias" (b^2 = (E[x_i^2] - E_p[x_i^2])^2 / Var_p[x_i^2]), from the
Laplace method of oracle/sv_laplace.py: the hyperparameters (s, r) on a
161 x 161 grid, the latent series given (s, r) by the Gaussian at its
conditional mode.  No sampler is involved, so the reference does not depend
on how fast any sampler mixes in the slow direction s.

    python tests/golden/stochvol_laplace.py   # ~2 minutes on one core
writes tests/golden/stochvol_T2427_laplace.json.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stochvol_T2427_laplace.json")
S = np.linspace(-4.7, -0.7, 161)
R = np.linspace(0.2, 4.2, 161)


def main():
    from oracle import sv_laplace
    from paper_2601_16696_amd import workloads
    w = workloads.stochvol(n_chains=2)
    out = sv_laplace.posterior_moments(w["y"], S, R)
    res = dict(workload="stochvol_T2427 (workloads.stochvol defaults)",
               source="Laplace method (oracle/sv_laplace.py): (s, r) on a 161 x 161 grid over "
                      "[-4.7, -0.7] x [0.2, 4.2], h | s, r Gaussian at the conditional mode",
               E_x2=out["E_x2"].tolist(), Var_x2=out["Var_x2"].tolist(), E_s=out["E_s"], E_r=out["E_r"],
               grid_edge_mass=out["grid_edge_mass"])
    with open(OUT, "w") as f:
        json.dump(res, f)
    print("wrote", OUT, "E[s^2]", out["E_x2"][-2], "E[r^2]", out["E_x2"][-1], "edge", out["grid_edge_mass"])


if __name__ == "__main__":
    main()
