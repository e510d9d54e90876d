"""laps_init_static: the initialisation for callers that cannot allocate
device memory, whose workspace is the library's static device array.  Its
runs are compared with laps_init on a caller workspace, bit for bit (the same
kernels on the same inputs), on two calls in a row on one device, the second
with a smaller input, so the second reuses the array and the context the
first left behind."""
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
    st = [s.stats()]
    s.step_adjusted(n_adj)
    st.append(s.stats())
    return st, s.positions().cpu().numpy().copy()


CASES = [
    # the larger input first: bf16 logistic regression, 192 chains, 8 row splits
    (lambda: workloads.logreg(n_chains=192, n=2000, d=100), "bf16", 12, 2),
    # then a smaller one: FP64 diagonal Gaussian, 40 chains, d = 37
    (lambda: workloads.gaussian(n_chains=40, d=37), "f64", 10, 2),
]


def test_static_workspace_matches_caller_workspace(gpu):
    import torch
    for k, (make, prec, n_unadj, n_adj) in enumerate(CASES):
        w = make()
        cfg = dict(switch_policy=1, max_steps_unadj=n_unadj, max_steps_total=n_unadj + 15 * n_adj)
        ref = gpu.Sampler(w, prec, **cfg)
        st_ref, x_ref = _run(ref, n_unadj, n_adj)
        s = gpu.Sampler(w, prec, static_workspace=True, **cfg)
        assert s.ws is None
        st, x = _run(s, n_unadj, n_adj)
        torch.cuda.synchronize()
        assert np.array_equal(x, x_ref), (k, np.max(np.abs(x - x_ref)))
        for a, b in zip(st, st_ref):
            for key in ("t", "grads_per_chain", "phase", "eps", "L", "dtilde", "eevpd", "acc_mean", "n_nonfinite"):
                assert a[key] == b[key], (k, key, a[key], b[key])
        assert st[-1]["phase"] == 2 and st[-1]["n_nonfinite"] == 0
        del s, ref


def test_static_workspace_without_normals_ahead_matches_caller_workspace(gpu):
    """An FP64 configuration of the C1 size (1024 chains, d = 100) needs about
    59 MB with the buffers of normals computed ahead, more than the 32 MiB
    static array; laps_init_static then drops those buffers and its kernels
    compute the normals where they use them.  The caller-workspace run keeps
    them, so the comparison also checks that both ways of getting the normals
    give the same run bit for bit."""
    import torch
    w = workloads.gaussian(n_chains=1024, d=100)
    cfg = dict(switch_policy=1, max_steps_unadj=30, max_steps_total=30 + 15 * 3)
    ref = gpu.Sampler(w, "f64", **cfg)
    assert ref.ws.numel() * ref.ws.element_size() > 32 << 20
    st_ref, x_ref = _run(ref, 30, 3)
    s = gpu.Sampler(w, "f64", static_workspace=True, **cfg)
    assert s.ws is None
    st, x = _run(s, 30, 3)
    torch.cuda.synchronize()
    assert np.array_equal(x, x_ref), np.max(np.abs(x - x_ref))
    for a, b in zip(st, st_ref):
        for key in ("t", "grads_per_chain", "phase", "eps", "L", "dtilde", "eevpd", "acc_mean", "n_nonfinite"):
            assert a[key] == b[key], (key, a[key], b[key])
    assert st[-1]["phase"] == 2 and st[-1]["n_nonfinite"] == 0
    del s, ref


def test_static_workspace_refuses_oversized_configurations(gpu):
    w = workloads.stochvol(n_chains=4096)
    with pytest.raises(gpu.LapsError, match="static workspace"):
        gpu.Sampler(w, "f32", static_workspace=True, switch_policy=1, max_steps_unadj=10)
