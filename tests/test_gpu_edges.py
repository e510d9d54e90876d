"""Degenerate and minimal cases on the GPU against the oracle: the smallest
valid ensembles (2 or 3 chains) and dimensions of every target family (d = 2
Gaussian, logistic regression with one observation, stochastic volatility
with T = 1, the 2 x 2 lattice, the 2-D dense Gaussian), zero-step calls, and
the phase rules of the entry points."""
import numpy as np
import pytest

from paper_2601_16696_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    from paper_2601_16696_amd import laps
    laps.lib()
    return laps


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle
    return oracle


def _rel_rows(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


CASES = {
    "gauss_d2_N2": lambda: workloads.gaussian(n_chains=2, d=2, x0_scale=1.0),
    "gauss_d2_N3": lambda: workloads.gaussian(n_chains=3, d=2, x0_scale=1.0),
    "logreg_n1_d2": lambda: workloads.logreg(n_chains=3, n=1, d=2),
    "stochvol_T1": lambda: workloads.stochvol(n_chains=2, T=1),
    "phi4_side2": lambda: workloads.phi4(n_chains=2, side=2),
    "dense_d2": lambda: workloads.ill_gaussian(n_chains=2, d=2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_minimal_sizes_match_oracle(gpu, orc, name):
    """Small d puts delta = h |g| / (d - 1) in the regime where the velocity
    map's energy is ill-conditioned in e.u, so positions are compared at 1e-8
    after 8 unadjusted steps (with the GPU's step sizes replayed) and 2
    transitions."""
    w = CASES[name]()
    cfg = dict(switch_policy=1, max_steps_unadj=8, max_steps_total=8 + 15 * 2, integrator_adj=1)
    o = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], **cfg)
    o.init(w["x0"])
    s = gpu.Sampler(w, "f64", **cfg)
    for _ in range(8):
        sg = s.stats()
        o.set_hyper(sg["eps"], sg["L"])
        o.step_unadjusted(1)
        s.step_unadjusted(1)
    so, sg = o.stats(), s.stats()
    assert sg["t"] == so["t"] == 8 and sg["phase"] == so["phase"] == 1
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.max(err) < 1e-8, np.max(err)
    for _ in range(2):
        o.set_hyper(s.stats()["eps"], 0.0)
        o.step_adjusted(1)
        s.step_adjusted(1)
    so, sg = o.stats(), s.stats()
    assert sg["t"] == so["t"] and sg["phase"] == so["phase"] == 2
    acc_o, acc_g = o.array("acc"), s.buffer("acc").cpu().numpy()
    same = np.abs(acc_o - acc_g) < 1e-6
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.all(err[same] < 1e-8), err


def test_zero_steps_and_phase_rules(gpu):
    w = workloads.gaussian(n_chains=5, d=7, x0_scale=1.0)
    s = gpu.Sampler(w, "f64", switch_policy=1, max_steps_unadj=3, max_steps_total=3 + 15)
    x0 = s.positions().clone()
    s.step_unadjusted(0)
    s.step_adjusted(0)  # the switch itself, no transition
    st = s.stats()
    assert st["t"] == 0 and st["phase"] == 2
    import torch
    assert torch.equal(s.positions(), x0)
    with pytest.raises(gpu.LapsError) as e:
        s.step_unadjusted(1)  # after the adjusted phase has started
    assert e.value.status == gpu.EPHASE
    s.step_adjusted(3)  # transitions start at t = 0 and 15 (< 18) and run; the third starts at 30 >= 18
    st = s.stats()
    assert st["t"] == 30 and st["phase"] == 2


def test_steps_after_the_automatic_switch_are_no_ops(gpu):
    w = workloads.gaussian(n_chains=16, d=5, x0_scale=1.0)
    s = gpu.Sampler(w, "f64", switch_policy=1, max_steps_unadj=4)
    s.step_unadjusted(4)
    x = s.positions().clone()
    s.step_unadjusted(6)
    st = s.stats()
    import torch
    assert st["t"] == 4 and st["phase"] == 1 and torch.equal(s.positions(), x)


# The largest dimensions the per-chain kernels take: FP64 keeps at most 2 octs
# per lane on 512-lane teams (d = 8192); FP32 up to 6, bounded by the MAMS
# kernel's LDS (the per-dim constants and the preconditioner, two rows of d
# floats, within 160 KiB: d = 20000)
@pytest.mark.parametrize("prec,d,N", [("f64", 8192, 6), ("f32", 20000, 4)])
def test_maximum_dimension(gpu, orc, prec, d, N):
    w = workloads.gaussian(n_chains=N, d=d, seed_data=1020, seed_x0=2020, seed_rng=3020, x0_scale=1.0)
    cfg = dict(switch_policy=1, max_steps_unadj=5, max_steps_total=5 + 15)
    o = orc.Ensemble(orc.Target.from_workload(w), N, w["seed"], **cfg)
    o.init(w["x0"])
    s = gpu.Sampler(w, prec, **cfg)
    for _ in range(5):
        sg = s.stats()
        o.set_hyper(sg["eps"], sg["L"])
        o.step_unadjusted(1)
        s.step_unadjusted(1)
    tol = 1e-10 if prec == "f64" else 1e-4
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.max(err) < tol, np.max(err)
    o.set_hyper(s.stats()["eps"], 0.0)
    o.step_adjusted(1)
    s.step_adjusted(1)
    assert s.stats()["t"] == o.stats()["t"] == 20
    acc_o, acc_g = o.array("acc"), s.buffer("acc").cpu().numpy()
    same = np.abs(acc_o - acc_g) < (1e-8 if prec == "f64" else 1e-3)
    assert same.mean() >= 0.5
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.all(err[same] < tol), err
