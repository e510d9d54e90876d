"""GPU parity of the logistic-regression target (the matrix-core path).

FP64 (plain vector-ALU gradient): positions within 1e-10 per chain of the
oracle after unadjusted steps and MAMS transitions.

bf16 mixed (v_mfma_f32_16x16x32_bf16, float accumulation, FP32 state, FP64
energy and reductions): X is bf16-exact by construction and theta enters as a
bf16 hi + lo pair, so on identical states every z_n is off by at most
2^-17 sum_i |X_ni theta_i| plus float accumulation; the residual r enters the
second product rounded to bf16 (2^-9 relative).  The tests check log p and
the gradient against those bounds on identical states, and a replayed run
against the oracle.  Sizes are ragged in every tiled dimension: N not a
multiple of 64 chains, n not a multiple of 32 rows, d not a multiple of 8/32.
"""
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


def _w(N=100, n=300, d=37, seed=11):
    return workloads.logreg(n_chains=N, n=n, d=d, seed_data=1000 + seed, seed_x0=2000 + seed)


def _oracle(orc, w, **cfg):
    e = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], **cfg)
    e.init(w["x0"])
    return e


def _rel_rows(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


# Logistic regression above d = 128 is refused by the library (its gradient kernels hold a chain's theta
# in registers up to 128 coordinates; the refusal is tested on the CPU in test_abi.py).  These shapes also
# ran in the two GPU faults whose cause is not found, so they stay off the GPU.
WIDE = pytest.mark.skip(reason="logistic regression with d > 128 is refused by the library; these shapes ran in "
                               "GPU faults whose cause is not found")


@pytest.mark.parametrize("shape", [(100, 300, 37), (64, 32, 100), (130, 5000, 100),
                                   pytest.param((40, 77, 300), marks=WIDE)])
def test_gradient_at_init_f64(gpu, orc, shape):
    N, n, d = shape
    w = _w(N, n, d)
    s = gpu.Sampler(w, "f64", integrator_adj=1)
    s.stats()
    g = s.buffer("g").cpu().numpy()
    lp = s.buffer("logp").cpu().numpy()
    ot = orc.Target.from_workload(w)
    ref = [ot.logp_grad(x) for x in w["x0"]]
    lref = np.array([r[0] for r in ref])
    gref = np.array([r[1] for r in ref])
    assert np.max(np.abs(lp - lref) / np.maximum(np.abs(lref), 1.0)) < 1e-12
    assert np.max(_rel_rows(g, gref)) < 1e-12


# (n, d) of the batched mix's logistic targets reach every k-chunk count of the
# staged (d <= 128) and direct-load gradient kernels; fewer chains, with n
# shortened where the oracle would be slow
C5_LR = [(48, 1000, 20), (40, 1534, 29), (36, 2354, 43), (24, 3611, 64), (20, 2000, 94),
         pytest.param((16, 1200, 138), marks=WIDE), pytest.param((12, 800, 204), marks=WIDE),
         pytest.param((8, 600, 300), marks=WIDE)]
MN2 = dict(integrator_adj=1)


@pytest.mark.parametrize("shape", [(100, 300, 37), (64, 32, 100), (130, 5000, 100),
                                   pytest.param((40, 77, 300), marks=WIDE)] + C5_LR)
def test_gradient_at_init_bf16_error_bounds(gpu, orc, shape):
    N, n, d = shape
    w = _w(N, n, d)
    s = gpu.Sampler(w, "bf16", **MN2)
    s.stats()
    th = np.asarray(w["x0"], dtype=np.float32).astype(np.float64)  # the FP32 state
    g = s.buffer("g").cpu().numpy().astype(np.float64)
    lp = s.buffer("logp").cpu().numpy()
    X, y = w["X"], w["y"]
    ot = orc.Target.from_workload(w)
    for m in range(N):
        l_ref, g_ref = ot.logp_grad(th[m])
        z = X @ th[m]
        zabs = np.abs(X) @ np.abs(th[m])
        dz = 2.0**-17 * zabs + 2.0**-22 * zabs * 2  # hi/lo residual + float accumulation
        sig = 1 / (1 + np.exp(-z))
        # log p = theta . X^T (y - 1/2) (FP64) + sum_n f(z_n), f(z) = -|z|/2 - log(1 + e^{-|z|}),
        # |f'(z)| = |sigmoid(z) - 1/2|: the z error enters through f only
        bound_l = np.sum(np.abs(sig - 0.5) * dz + 0.25 * dz**2) + 1e-6 * np.sum(np.abs(z) + 1.0)
        assert abs(lp[m] - l_ref) <= bound_l, (m, lp[m] - l_ref, bound_l)
        # residual rounding to bf16 (and its dependence on z) bounds the gradient error
        dr = 2.0**-9 * np.abs(y - sig) + 0.25 * dz + 1e-7
        bound_g = np.abs(X).T @ dr + 1e-5 * (np.abs(X).T @ np.abs(y - sig)) + 1e-6 * np.abs(th[m])
        assert np.all(np.abs(g[m] - g_ref) <= bound_g), (m, np.max(np.abs(g[m] - g_ref) / bound_g))


@pytest.mark.parametrize("block_threads", [0, 64, 128])
def test_unadjusted_and_adjusted_f64(gpu, orc, block_threads):
    w = _w(100, 300, 37)
    cfg = dict(switch_policy=1, max_steps_unadj=15, max_steps_total=400, block_threads=block_threads)
    o = _oracle(orc, w, **cfg)
    s = gpu.Sampler(w, "f64", **cfg)
    for k in range(15):
        o.step_unadjusted(1)
        s.step_unadjusted(1)
        so, sg = o.stats(), s.stats()
        for key in ("eps", "L", "dtilde"):
            assert abs(sg[key] - so[key]) <= 1e-9 * abs(so[key]), (k, key, sg[key], so[key])
    x = s.positions().cpu().numpy()
    assert np.max(_rel_rows(x, o.array("x"))) < 1e-10
    assert so["phase"] == sg["phase"] == 1
    for k in range(3):
        o.step_adjusted(1)
        s.step_adjusted(1)
        so, sg = o.stats(), s.stats()
        assert abs(sg["acc_mean"] - so["acc_mean"]) < 1e-8, (k, sg["acc_mean"], so["acc_mean"])
        assert abs(sg["eps"] - so["eps"]) <= 1e-9 * so["eps"]
        assert sg["t"] == so["t"] and sg["grads_per_chain"] == so["grads_per_chain"]
    x = s.positions().cpu().numpy()
    assert np.max(_rel_rows(x, o.array("x"))) < 1e-10
    np.testing.assert_allclose(s.buffer("acc").cpu().numpy(), o.array("acc"), rtol=0, atol=1e-8)


def test_mixed_replayed_against_oracle(gpu, orc):
    """bf16 gradients steer the velocity; with the oracle replaying the GPU's
    eps and L, positions stay within 2e-3 relative per chain over 10 steps and
    the energy errors agree to the log p error bound."""
    w = _w(100, 300, 37)
    cfg = dict(switch_policy=1, max_steps_unadj=1000)
    o = _oracle(orc, w, **cfg)
    s = gpu.Sampler(w, "bf16", **cfg)
    for k in range(10):
        sg = s.stats()
        o.set_hyper(sg["eps"], sg["L"])
        o.step_unadjusted(1)
        s.step_unadjusted(1)
    x = s.positions().cpu().numpy()
    err = _rel_rows(x, o.array("x"))
    assert np.max(err) < 2e-3, np.max(err)
    dl = s.buffer("delta").cpu().numpy() - o.array("delta")
    assert np.max(np.abs(dl)) < 5e-2, np.max(np.abs(dl))


def test_mixed_adjusted_runs_and_accepts(gpu, orc):
    w = _w(256, 500, 64, seed=3)
    s = gpu.Sampler(w, "bf16", switch_policy=1, max_steps_unadj=200, max_steps_total=200 + 15 * 12)
    s.step_unadjusted(200)
    s.step_adjusted(12)
    st = s.stats()
    assert st["phase"] == 2 and st["n_nonfinite"] == 0
    assert abs(st["acc_mean"] - 0.7) < 0.15
    assert np.all(np.isfinite(s.positions().cpu().numpy()))


@pytest.mark.parametrize("shape", [(100, 300, 37), (96, 1000, 100)])
def test_mixed_transitions_against_oracle_on_identical_states(gpu, orc, shape):
    """The bf16 adjusted phase (MN2 MAMS transitions, the bulk of the
    logistic-regression run's gradients) against the FP64 oracle.  Before
    every transition the oracle takes the GPU's positions (its FP32 state,
    exactly), its step size and, at the switch, its preconditioner; the
    oracle's own FP64 log p and gradient at those positions start its
    trajectory.  Per transition: the step counter is identical; chains with
    the same Metropolis decision agree to 5e-3 relative (their trajectories
    are steered by bf16 gradients, r rounded to 2^-9, for 15 steps); the
    energy errors agree within 0.1 with a median below 0.02 (measured up to
    0.05: the difference is mostly log p at the two sides' slightly different
    endpoints, since each side's Delta is the exact energy error of its own
    reversible map, while Delta itself spreads over ~1 at acceptance 0.7);
    decisions flip only where the uniform lies between the two sides'
    acceptance probabilities, for at most 10% of the chains."""
    import torch
    N, n, d = shape
    w = _w(N, n, d, seed=21)
    n_adj = 4
    cfg = dict(switch_policy=1, max_steps_unadj=10, max_steps_total=10 + 15 * n_adj)
    o = _oracle(orc, w, **cfg)
    s = gpu.Sampler(w, "bf16", **cfg)
    ot = orc.Target.from_workload(w)
    for _ in range(10):
        sg = s.stats()
        o.set_hyper(sg["eps"], sg["L"])
        o.step_unadjusted(1)
        s.step_unadjusted(1)
    o.do_switch()
    worst_dD, worst_x, flips_total = 0.0, 0.0, 0
    for k in range(n_adj):
        sg = s.stats()
        assert sg["t"] == o.stats()["t"] == 10 + 15 * k
        xk = s.positions().cpu().numpy().astype(np.float64)
        s.step_adjusted(1)
        torch.cuda.synchronize()
        sig = s.buffer("sigma").cpu().numpy().astype(np.float64)
        lg = [ot.logp_grad(r) for r in xk]
        o.set_array("x", xk)
        o.set_array("g", np.array([r[1] for r in lg]))
        o.set_array("logp", np.array([r[0] for r in lg]))
        o.set_array("sigma", sig)
        o.set_hyper(sg["eps"], sg["L"])
        o.mams_move()
        o.adj_control()
        sg2, so = s.stats(), o.stats()
        assert sg2["t"] == so["t"] == 10 + 15 * (k + 1) and sg2["n_nonfinite"] == 0
        dg, do = s.buffer("delta").cpu().numpy(), o.array("delta")
        dD = np.abs(dg - do)
        worst_dD = max(worst_dD, float(dD.max()))
        assert np.max(dD) < 0.1 and np.median(dD) < 0.02, (k, np.max(dD), np.median(dD))
        xg, xo = s.positions().cpu().numpy().astype(np.float64), o.array("x")
        acc_g = np.any(xg != xk, axis=1)
        acc_o = np.any(xo != xk, axis=1)
        flip = acc_g != acc_o
        flips_total += int(flip.sum())
        # a flip needs the uniform between e^{-Delta_gpu} and e^{-Delta_oracle}
        U = np.array([orc.mh_uniform(w["seed"], m, 10 + 15 * k) for m in range(N)])
        lo = np.minimum(np.exp(-dg), np.exp(-do))
        hi = np.maximum(np.exp(-dg), np.exp(-do))
        assert np.all((U[flip] >= lo[flip]) & (U[flip] < hi[flip]))
        same = ~flip
        # rejected on both sides: restored to the identical start
        assert np.array_equal(xg[same & ~acc_g], xk[same & ~acc_g])
        both = same & acc_g
        if np.any(both):
            err = _rel_rows(xg[both], xo[both])
            worst_x = max(worst_x, float(err.max()))
            assert np.max(err) < 5e-3, (k, np.max(err))
    assert flips_total <= max(2, 0.1 * N * n_adj), flips_total
    print(f"bf16 MAMS vs FP64 oracle (N={N}, n={n}, d={d}): max |dDelta| {worst_dD:.2e}, "
          f"max rel x err {worst_x:.2e}, decision flips {flips_total}/{N * n_adj}")


@pytest.mark.parametrize("prec", ["f64", "bf16"])
@pytest.mark.parametrize("shape", [
    (40, 150, 100), (70, 300, 37),
    pytest.param((40, 150, 204), marks=pytest.mark.skip(
        reason="the logistic-regression MN4 transition at d = 204 faulted the GPU (illegal memory access) with "
               "no cause shown; the library refuses logistic regression with d > 128"))])
def test_fourth_order_transitions(gpu, orc, prec, shape):
    """The MN4 integrator in the adjusted phase (the automatic choice above
    d = 200, asked for explicitly here): five gradient stages per step
    through the per-chain update kernel.  FP64 runs free (both controllers
    their own) with eps within 1e-9 and positions within 3e-10: the two
    transitions take 150 gradient stages per chain, each summed in another
    order by the matrix-core kernel than by the oracle (~1e-15 relative), and
    the step sizes of the free controllers differ in the last digits (the
    MN2 tests, with two stages per step instead of five, hold 1e-10).  bf16
    with the oracle replaying eps."""
    N, n, d = shape
    w = _w(N, n, d, seed=5)
    cfg = dict(switch_policy=1, max_steps_unadj=8, max_steps_total=8 + 15 * 3, integrator_adj=2)
    o = _oracle(orc, w, **cfg)
    s = gpu.Sampler(w, prec, **cfg)
    replay = prec != "f64"
    for _ in range(8):
        if replay:
            sg = s.stats()
            o.set_hyper(sg["eps"], sg["L"])
        o.step_unadjusted(1)
        s.step_unadjusted(1)
    for k in range(2):
        if replay and k > 0:
            o.set_hyper(s.stats()["eps"], 0.0)
        o.step_adjusted(1)
        s.step_adjusted(1)
        so, sg = o.stats(), s.stats()
        assert so["integrator"] == sg["integrator"] == 2 and so["t"] == sg["t"]
        assert sg["n_nonfinite"] == 0
        if not replay:
            assert abs(sg["eps"] - so["eps"]) <= 1e-9 * so["eps"], (k, sg["eps"], so["eps"])
    x, xo = s.positions().cpu().numpy(), o.array("x")
    err = _rel_rows(x, xo)
    if prec == "f64":
        assert np.max(err) < 3e-10, np.max(err)
        np.testing.assert_allclose(s.buffer("acc").cpu().numpy(), o.array("acc"), rtol=0, atol=1e-8)
    else:
        # chains whose accept decision flips between the two (U within the bf16 energy error) are excluded
        assert np.mean(err > 1e-2) <= 0.1 and np.max(err[err <= 1e-2]) < 2e-3, (np.mean(err > 1e-2), np.max(err))
