"""The C ABI driven from plain C (paper_2601_16696_amd/csrc/laps_capi_run.c:
the HIP runtime's C API and include/laps.h, no Python or torch in that
process): a small full run on the diagonal Gaussian whose final positions,
step count, phase and step size match the oracle's on the same inputs."""
import os
import subprocess

import numpy as np
import pytest

from paper_2601_16696_amd import workloads

pytestmark = pytest.mark.gpu

PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2601_16696_amd")
BIN = os.path.join(PKG, "laps_capi_run")


def test_c_consumer_matches_oracle(tmp_path):
    from oracle import oracle as orc
    assert os.path.exists(BIN), "build the library first (it builds the C consumer too)"
    w = workloads.gaussian(n_chains=100, d=100)
    N, d = w["n_chains"], w["d"]
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    np.concatenate([np.asarray(w["sigma2"], dtype=np.float64).ravel(),
                    np.asarray(w["x0"], dtype=np.float64).ravel()]).tofile(inp)
    print("running", BIN, N, d, flush=True)
    r = subprocess.run([BIN, inp, out, str(N), str(d), str(w["seed"])], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    raw = np.fromfile(out, dtype=np.float64)
    x_gpu, tail = raw[:N * d].reshape(N, d), raw[N * d:]
    e = orc.Ensemble(orc.Target.from_workload(w), N, w["seed"], switch_policy=1, max_steps_unadj=12,
                     max_steps_total=12 + 15 * 3)
    e.init(w["x0"])
    e.step_unadjusted(12)
    e.do_switch()
    e.step_adjusted(3)
    st = e.stats()
    assert tail[0] == st["t"] == 12 + 45 and tail[1] == st["phase"] == 2
    assert abs(tail[2] - st["eps"]) <= 1e-9 * st["eps"]
    xo = e.array("x")
    err = np.linalg.norm(x_gpu - xo, axis=1) / np.linalg.norm(xo, axis=1)
    assert np.max(err) < 1e-10, np.max(err)
