"""GPU parity: the HIP path against the FP64 CPU oracle on identical seeded
inputs, through the C ABI.

Integer work (Philox words) must match bit for bit.  Floating point: FP64
state within 1e-10 relative per chain after the runs below, FP32 state within
1e-4 (the oracle then replays the GPU's eps and L so that FP32 rounding is not
fed back through the controller); per-step scalars within 1e-9 relative in
FP64, except where a quantity is a near-cancelling difference of log densities
(the energy error and EEVPD), whose tolerance scales with |log p|.  Sizes span several
workgroups, ragged last octs (d not a multiple of 8), ragged chain tiles, and
single-wave, multi-team and multi-wave team shapes.
"""
import numpy as np
import pytest

from paper_2601_16696_amd import workloads

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "gpu tests need a GPU"
    from paper_2601_16696_amd import laps
    laps.lib()
    return laps


def _oracle(orc, w, **cfg):
    e = orc.Ensemble(orc.Target.from_workload(w), w["n_chains"], w["seed"], **cfg)
    e.init(w["x0"])
    return e


def _rel_rows(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def _close(a, b, tol):
    return abs(a - b) <= tol * max(abs(b), 1e-300)


# ------------------------------------------------------------------ RNG
def test_philox_words_bit_exact(gpu, orc):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**63, size=(513, 4), dtype=np.int64).astype(np.uint64)
    ctr[0] = 0
    ctr[1] = 2**64 - 1
    got = gpu.philox_words(ctr, 3001)
    ref = np.array([orc.philox4x64_10(c, [3001, 0]) for c in ctr])
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 3e-6)])
def test_normal_stream(gpu, orc, prec, tol):
    d = 101
    z = gpu.philox_normals(77, 9, d, 12, 2, 3, prec).cpu().numpy()
    ref = np.array([orc.normals(77, m, 12, 2, 3, d) for m in range(9)])
    assert np.max(np.abs(z - ref) / (1 + np.abs(ref))) < tol


# ------------------------------------------------------------------ targets
def _small_workloads():
    return {
        "gauss": workloads.gaussian(n_chains=100, d=100),
        "stochvol": workloads.stochvol(n_chains=37, T=200),
        "phi4": workloads.phi4(n_chains=50, side=12),
        "phi4_multiwave": workloads.phi4(n_chains=20, side=32),
        "gauss_d3": workloads.gaussian(n_chains=70, d=3, x0_scale=1.0),
        # dimensions of the batched mix's Gaussians, fewer chains
        "gauss_d10": workloads.gaussian(n_chains=90, d=10, seed_data=1005, seed_x0=2005, seed_rng=3005, x0_scale=1.0),
        "gauss_d440": workloads.gaussian(n_chains=96, d=440, seed_data=1010, seed_x0=2010, seed_rng=3010),
        "gauss_d938": workloads.gaussian(n_chains=64, d=938, seed_data=1011, seed_x0=2011, seed_rng=3011),
        "gauss_d2000": workloads.gaussian(n_chains=48, d=2000, seed_data=1012, seed_x0=2012, seed_rng=3012),
        # the benchmark lattice (side 64) with few chains: FP64 MAMS needs 66 KiB of LDS
        "phi4_L64": workloads.phi4(n_chains=20, side=64, seed_x0=2013, seed_rng=3013),
    }


# Team shapes of the per-chain kernels, forced through team_lanes so that the
# small sizes above reach every code path: several octs per lane (Q > 1, the
# column-sum statistics), octs wrapping across lanes in the neighbour exchange,
# the whole-oct lattice rows (side a multiple of 8) and multi-wavefront teams.
SHAPES = {
    # name: (workload, {precision: team_lanes})
    "gauss": ("gauss", {"f64": 0, "f32": 0}),                        # 16 lanes x 1 oct
    "gauss_q2": ("gauss", {"f64": 8, "f32": 4}),                     # 2 / 4 octs per lane
    "stochvol": ("stochvol", {"f64": 0, "f32": 0}),                  # 32 lanes x 1 oct
    "stochvol_q": ("stochvol", {"f64": 16, "f32": 8}),               # 2 / 4 octs per lane
    "stochvol_multiwave": ("stochvol", {"f64": 128, "f32": 128}),    # two wavefronts per chain
    "phi4": ("phi4", {"f64": 0, "f32": 0}),                          # side 12: per-site neighbours
    "phi4_rows": ("phi4_multiwave", {"f64": 0, "f32": 0}),           # side 32: 64 lanes x 2 octs
    "phi4_rows_q": ("phi4_multiwave", {"f64": 64, "f32": 32}),       # 2 / 4 octs per lane
    "phi4_multiwave": ("phi4_multiwave", {"f64": 128, "f32": 128}),  # two wavefronts per chain
    "gauss_d3": ("gauss_d3", {"f64": 0, "f32": 0}),
    "gauss_d10": ("gauss_d10", {"f64": 0, "f32": 0}),                # 2 lanes x 1 oct
    "gauss_d440": ("gauss_d440", {"f64": 0, "f32": 0}),              # 64 lanes x 1 oct, in-register sums
    "gauss_d938": ("gauss_d938", {"f64": 0, "f32": 0}),              # 64 lanes x 2 octs
    "gauss_d2000": ("gauss_d2000", {"f64": 0, "f32": 0}),            # 64 x 4 (FP32), 128 x 2 (FP64)
    "phi4_L64": ("phi4_L64", {"f64": 0, "f32": 0}),                  # 128 x 4 (FP32), 256 x 2 (FP64)
}


# shapes whose oracle replays the GPU's (eps, L) in FP64 too (see test_unadjusted_steps)
REPLAY = ("gauss_d440", "gauss_d938", "gauss_d2000", "phi4_L64")


def _shape(name, prec):
    wname, lanes = SHAPES[name]
    return _small_workloads()[wname], {"team_lanes": lanes[prec]}


@pytest.mark.parametrize("name", ["gauss", "stochvol", "phi4", "phi4_multiwave", "gauss_d3"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_target_eval(gpu, orc, name, prec):
    import torch
    w = _small_workloads()[name]
    tgt = gpu.Target(w, prec)
    x = torch.as_tensor(w["x0"], device="cuda:0")
    lp, g = tgt.eval(x)
    torch.cuda.synchronize()
    ot = orc.Target.from_workload(w)
    ref = [ot.logp_grad(r) for r in w["x0"]]
    lref = np.array([r[0] for r in ref])
    gref = np.array([r[1] for r in ref])
    tol = 1e-12 if prec == "f64" else 2e-5
    lp = lp.cpu().numpy()
    assert np.max(np.abs(lp - lref) / np.maximum(np.abs(lref), 1.0)) < tol
    g = g.cpu().numpy()
    assert np.max(_rel_rows(g, gref)) < tol


# ------------------------------------------------------------------ steps
def _delta_tol(o, prec, s=None):
    """Elementwise tolerance of the energy error Delta = (log p before - log p
    after) + B energies.  Its rounding error scales with |log p| (the terms
    nearly cancel); and since eps is computed from the near-cancelling EEVPD of
    earlier steps, the two step sizes differ at ~1e-11 relative, which Delta
    (a low power of eps) carries as a relative part."""
    d_o = o.array("delta")
    lp = np.max(np.abs(o.array("logp"))) + 1.0
    rel = 1e-8 if prec == "f64" else 1e-4
    if s is not None:
        so, sg = o.stats(), s.stats()
        rel = max(rel, 50.0 * abs(sg["eps"] - so["eps"]) / so["eps"])
    return (1e-12 if prec == "f64" else 2e-6) * lp + rel * np.abs(d_o)


def _run_pair(gpu, orc, w, prec, n_unadj, replay, per_step=None, **cfg):
    """Runs oracle and GPU side by side.  replay=True makes the oracle take the
    GPU's (eps, L) before every step, which isolates the per-chain maps from
    controller feedback (used for the FP32 state against the FP64 oracle)."""
    o = _oracle(orc, w, **cfg)
    s = gpu.Sampler(w, prec, **cfg)
    so, sg = o.stats(), s.stats()
    assert _close(sg["eps"], so["eps"], 1e-12) and _close(sg["L"], so["L"], TOL[prec])
    for k in range(n_unadj):
        if replay:
            sg = s.stats()
            o.set_hyper(sg["eps"], sg["L"])
        o.step_unadjusted(1)
        s.step_unadjusted(1)
        if per_step:
            per_step(k, o, s)
    return o, s


def _compare_x(o, s, prec):
    x = s.positions().cpu().numpy()
    err = _rel_rows(x, o.array("x"))
    assert np.max(err) < TOL[prec], np.max(err)


@pytest.mark.parametrize("name", list(SHAPES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unadjusted_steps(gpu, orc, name, prec):
    w, shape = _shape(name, prec)
    # The batched mix's larger Gaussian shapes (d = 440 ... 2000) from the cold start keep many chains in the
    # ill-conditioned large-delta regime, whose energy errors feed the step-size controller; the
    # oracle replays the GPU's (eps, L) there, so that the per-chain maps of these team shapes are
    # compared by themselves (the controller is compared on the other shapes).  The side-64 lattice
    # likewise: there a relative change of 1e-15 in the start moves the oracle's own EEVPD target by
    # ~1e-10 within six steps, so last-digit differences of the GPU's arithmetic reach 1e-9
    replay = prec == "f32" or name in REPLAY

    # d = 3: delta = h |g| / (d-1) is large, where the velocity energy
    # (d-1) log(cosh delta + c sinh delta) is ill-conditioned in c = e.u, so
    # only the positions are compared, at 1e-8
    per_step_delta = name != "gauss_d3"

    def check(k, o, s):
        so, sg = o.stats(), s.stats()
        assert sg["t"] == so["t"] and sg["phase"] == so["phase"]
        d_o = o.array("delta")
        d_g = s.buffer("delta").cpu().numpy()
        tol = _delta_tol(o, prec, s)
        atol = np.max(tol)
        if per_step_delta:
            # a few chains per step can sit where the velocity energy is ill-conditioned in
            # e.u (large delta with e.u near -1): allow 2% of them (at least 4 chains) up to
            # 100x the bound; the larger cold-started Gaussians (d >= 440, 2% of whose
            # variances are 1e-2 with starts of scale 10) keep more chains in that regime
            # over the first steps, so 10% there
            ratio = np.abs(d_g - d_o) / tol
            allow = 0.1 if name in ("gauss_d440", "gauss_d938", "gauss_d2000") else max(0.02, 4.0 / len(ratio))
            assert np.mean(ratio > 1) <= allow and np.max(ratio) < 100, (k, np.mean(ratio > 1), np.max(ratio))
        if not replay:
            # EEVPD inherits the conditioning of Delta plus the drift of eps (Delta ~ eps^3)
            rms = np.sqrt(np.mean(d_o**2)) + 1e-300
            e_tol = 1e-9 + 3 * atol / rms
            if per_step_delta:
                assert _close(sg["eevpd"], so["eevpd"], e_tol), (k, sg["eevpd"], so["eevpd"], e_tol)
            for key in ("L", "dtilde", "eevpd_target", "eps"):
                assert _close(sg[key], so[key], 1e-9 if per_step_delta else 1e-7), (k, key, sg[key], so[key])
        else:
            for key in ("L", "dtilde"):
                assert _close(sg[key], so[key], TOL[prec]), (k, key, sg[key], so[key])

    o, s = _run_pair(gpu, orc, w, prec, 30, replay, per_step=check, switch_policy=1, max_steps_unadj=1000, **shape)
    tol = TOL[prec] if per_step_delta or prec == "f32" else 1e-8
    x = s.positions().cpu().numpy()
    assert np.max(_rel_rows(x, o.array("x"))) < tol, np.max(_rel_rows(x, o.array("x")))
    u = s.buffer("u").cpu().numpy()
    # with few dimensions each refresh and velocity update moves the unit vector u by a larger
    # fraction, so rounding differences in u grow faster over the 30 steps
    u_tol = tol * (10 if w["d"] <= 10 else 1)
    assert np.max(_rel_rows(u, o.array("u"))) < u_tol, np.max(_rel_rows(u, o.array("u")))


@pytest.mark.parametrize("name", ["gauss", "gauss_q2", "stochvol", "stochvol_q", "stochvol_multiwave", "phi4",
                                  "phi4_rows", "phi4_rows_q", "phi4_multiwave", "gauss_d10", "gauss_d440",
                                  "gauss_d938", "gauss_d2000", "phi4_L64"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjusted_transitions(gpu, orc, name, prec):
    """MAMS transitions after a fixed switch.  Chains whose accept decision
    differs between GPU and oracle (U within rounding of e^{-Delta}) are
    counted; FP64 allows none."""
    w, shape = _shape(name, prec)
    # FP32 state, and the larger cold-started Gaussians (see test_unadjusted_steps): the oracle
    # replays the GPU's step sizes
    replay = prec == "f32" or name in REPLAY
    o, s = _run_pair(gpu, orc, w, prec, 12, replay, switch_policy=1, max_steps_unadj=12, max_steps_total=400,
                     **shape)
    assert o.stats()["phase"] == s.stats()["phase"] == 1
    flipped = np.zeros(w["n_chains"], dtype=bool)
    for k in range(4):
        if replay and k > 0:
            o.set_hyper(s.stats()["eps"], 0.0)
        o.step_adjusted(1)
        s.step_adjusted(1)
        so, sg = o.stats(), s.stats()
        assert so["integrator"] == sg["integrator"] and so["t"] == sg["t"]
        acc_o, acc_g = o.array("acc"), s.buffer("acc").cpu().numpy()
        if k == 0:
            np.testing.assert_allclose(s.buffer("sigma").cpu().numpy(), o.array("sigma"), rtol=TOL[prec])
        x_o, x_g = o.array("x"), s.positions().cpu().numpy()
        err = _rel_rows(x_g, x_o)
        flipped |= err > 1e-2
        assert np.max(np.abs(acc_g - acc_o)[~flipped]) < (1e-8 if prec == "f64" else 2e-3)
        if not replay:
            assert _close(sg["acc_mean"], so["acc_mean"], 1e-8), (k, sg["acc_mean"], so["acc_mean"])
            assert _close(sg["eps"], so["eps"], 1e-9)
    if prec == "f64":
        assert not flipped.any()
    else:
        assert flipped.mean() <= 0.05, flipped.mean()
    err = _rel_rows(s.positions().cpu().numpy(), o.array("x"))
    assert np.max(err[~flipped]) < TOL[prec], np.max(err[~flipped])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_large_delta_first_steps(gpu, orc, prec):
    """d = 3 from the N(0, 10^2) cold start: |delta| reaches ~1600 on the second
    step, where the velocity map needs its cosh-divided form.  Compared over
    the first three steps, before the strongly sensitive dynamics of this
    regime amplify rounding differences."""
    w = workloads.gaussian(n_chains=70, d=3)
    o, s = _run_pair(gpu, orc, w, prec, 3, prec == "f32", switch_policy=1)
    d_o, d_g = o.array("delta"), s.buffer("delta").cpu().numpy()
    assert np.all(np.isfinite(d_g)) and np.all(np.isfinite(d_o))
    assert np.all(np.abs(d_g - d_o) <= _delta_tol(o, prec) * (1 if prec == "f64" else 50))
    x = s.positions().cpu().numpy()
    # this regime amplifies rounding differences strongly (gradients ~1e3 act on steps of ~3)
    assert np.max(_rel_rows(x, o.array("x"))) < (1e-8 if prec == "f64" else TOL[prec])


def test_window_and_automatic_switch(gpu, orc):
    # short window (round(0.2 * 40) = 8 steps) so the ring fills inside the test
    w = workloads.gaussian(n_chains=64, d=20, x0_scale=1.0)
    cfg = dict(switch_policy=0, max_steps_unadj=35, max_steps_total=40, switch_tol=0.5)
    o = _oracle(orc, w, **cfg)
    s = gpu.Sampler(w, "f64", **cfg)
    for k in range(40):
        o.step_unadjusted(1)
        s.step_unadjusted(1)
        so, sg = o.stats(), s.stats()
        assert so["phase"] == sg["phase"] and so["t"] == sg["t"], k
        if so["ring_full"]:
            assert _close(sg["max_delta"], so["max_delta"], 1e-10), (k, sg["max_delta"], so["max_delta"])
    assert so["t"] < 35 and so["phase"] == 1  # the fluctuation rule fired before the cap


def test_phase_rules(gpu, orc):
    w = workloads.gaussian(n_chains=16, d=10)
    s = gpu.Sampler(w, "f64", switch_policy=1, max_steps_unadj=5, max_steps_total=40)
    s.step_unadjusted(9)  # the last four are predicated no-ops on the device
    st = s.stats()
    assert st["t"] == 5 and st["phase"] == 1
    s.step_adjusted(10)  # 15 steps per transition: those starting at t = 5, 20, 35 < 40 run
    st = s.stats()
    assert st["phase"] == 2 and st["t"] == 50
    with pytest.raises(gpu.LapsError) as ei:
        s.step_unadjusted(1)
    assert ei.value.status == gpu.EPHASE


def test_nonfinite_chain_flagged_and_rejected(gpu, orc):
    w = workloads.gaussian(n_chains=32, d=12)
    x0 = w["x0"].copy()
    x0[5, 3] = np.nan
    s = gpu.Sampler(w, "f64", x0=x0, switch_policy=1, max_steps_unadj=0)
    s.step_adjusted(1)
    st = s.stats()
    assert st["n_nonfinite"] >= 1 and (st["status_bits"] & 1) and st["status"] == gpu.ENONFINITE
    assert s.buffer("acc").cpu().numpy()[5] == 0.0
    x = s.positions().cpu().numpy()
    assert np.all(np.isfinite(np.delete(x, 5, axis=0)))
