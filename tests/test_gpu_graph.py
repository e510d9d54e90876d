"""Restart and batched graph replays against eager runs on the GPU.

A restart must reproduce the run that laps_init starts bit for bit; a graph
of run segments of several samplers, each on its own stream, must reproduce
the eager runs of the same samplers bit for bit on every replay, with the
program's own eager work and synchronisations between replays."""
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


def _run(s, n_unadj, n_adj):
    s.step_unadjusted(n_unadj)
    s.step_adjusted(n_adj)


def test_restart_reproduces_fresh_run(gpu):
    import torch
    w = workloads.gaussian(n_chains=96, d=37)
    cfg = dict(switch_policy=1, max_steps_unadj=12, max_steps_total=12 + 15 * 3)
    s = gpu.Sampler(w, "f64", **cfg)
    x0 = s.x.clone()
    _run(s, 12, 2)
    ref = s.x.clone()
    st_ref = s.stats()
    s.restart(x0[:, :w["d"]])
    _run(s, 12, 2)
    torch.cuda.synchronize()
    assert torch.equal(s.x, ref)
    st = s.stats()
    assert st["eps"] == st_ref["eps"] and st["t"] == st_ref["t"] and st["acc_mean"] == st_ref["acc_mean"]


def test_segment_graphs_replay_eager_runs(gpu):
    import torch
    specs = [(workloads.gaussian(n_chains=80, d=45), "f32"),
             (workloads.logreg(n_chains=70, n=300, d=20), "bf16"),
             (workloads.stochvol(n_chains=40, T=150), "f64")]
    cfg = dict(switch_policy=1, max_steps_unadj=14, max_steps_total=14 + 15 * 4)
    streams = [torch.cuda.Stream() for _ in specs]
    samplers, x0s = [], []
    for (w, prec), st in zip(specs, streams):
        with torch.cuda.stream(st):
            s = gpu.Sampler(w, prec, **cfg)
            x0s.append(s.x.clone())
        samplers.append(s)
    torch.cuda.synchronize()
    # eager reference runs, each on its own stream
    refs = []
    for s, st, x0 in zip(samplers, streams, x0s):
        with torch.cuda.stream(st):
            s.restart(x0[:, :s.d])
            _run(s, 14, 3)
    torch.cuda.synchronize()
    refs = [s.x.clone() for s in samplers]
    # the same runs as three segment graphs: restart + 9 steps | 5 steps + switch + 2 | 1 transition
    g1 = gpu.RunGraph(samplers, 9, 0, restart=True, x0s=x0s)
    g2 = gpu.RunGraph(samplers, 5, 2)
    g3 = gpu.RunGraph(samplers, 0, 1)
    for rep in range(3):
        g1.launch()
        g2.launch()
        g3.launch()
        torch.cuda.synchronize()
        for k, (s, ref) in enumerate(zip(samplers, refs)):
            assert torch.equal(s.x, ref), (rep, k, float((s.x - ref).abs().max()))
        # eager work between replays
        junk = torch.randn(1000, device="cuda:0").sum()
        for s in samplers:
            _ = s.stats()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)


@pytest.mark.parametrize("spec", [("gauss", "unadj"), ("logreg", "grad")])
def test_kernel_log_counts_launches(gpu, spec):
    """The event log brackets every launch of the chosen kernel inside the
    steps that follow (one per unadjusted step; for logistic regression also
    the MAMS trajectory's gradients), leaves the run's results unchanged, and
    graph recording refuses a logging context."""
    import torch
    name, which = spec
    w = workloads.gaussian(n_chains=64, d=30) if name == "gauss" else workloads.logreg(n_chains=64, n=200, d=20)
    prec = "f64" if name == "gauss" else "bf16"
    cfg = dict(switch_policy=1, max_steps_unadj=10, max_steps_total=10 + 15 * 2, integrator_adj=1)
    ref = gpu.Sampler(w, prec, **cfg)
    _run(ref, 10, 1)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = gpu.Sampler(w, prec, **cfg)
    s.kernel_log(which, 100)
    with pytest.raises(gpu.LapsError):
        gpu.RunGraph([s], 1, 0)
    _run(s, 10, 1)
    n, ms = s.kernel_log_read()
    # MN2 takes two gradients per integrator step of the 15-step trajectory
    assert n == (10 if which == "unadj" else 10 + 2 * 15)
    assert ms > 0.0
    s.kernel_log(which, 0)
    assert s.kernel_log_read() == (0, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(s.x, ref.x)
    # one launch in three: the first, the fourth, ...
    s.restart(torch.as_tensor(w["x0"], device="cuda:0").to(s.x.dtype))
    s.kernel_log(which, 100, 3)
    _run(s, 10, 1)
    n3, _ = s.kernel_log_read()
    assert n3 == (n + 2) // 3
    s.kernel_log(which, 0)
