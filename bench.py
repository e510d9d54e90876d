#!/usr/bin/env python3
"""Throughput of the LAPS hot path on one MI355X.

One benchmark step is one full LAPS run (Algorithm "LAPS Pseudocode") over one
synthetic workload, chains cold-started from the prior or the workload's x0:
initialisation, 1000 unadjusted steps (leapfrog, 1 gradient each), the switch,
and 67 MAMS transitions (15 integrator steps each).  Every phase runs in the
library's HIP kernels; positions are resident in HBM before the timed region.

Default workload: Bayesian logistic regression (X 5000 x 100 N(0,1) rounded to
bf16, weights N(0, 1/d), Bernoulli labels, N(0, I) prior), 4096 chains, bf16
matrix-core gradient with FP32 state.  Others: --workload gauss (diagonal
Gaussian d = 100, 1024 chains, FP64), stochvol (T = 2427, 4096 chains, FP32),
phi4 (64 x 64 lattice, 2048 chains, FP32), ill_gauss (randomly rotated
ill-conditioned Gaussian d = 100, dense precision on the matrix cores, 1024
chains, FP64), batched (16 targets, 46018 chains, run concurrently from
recorded segment graphs).

value = chain-gradient evaluations per second over the timed runs.
roofline: the dominant kernel, one launch in ten inside the timed runs bracketed
by HIP events on the stream it runs on (logistic regression: the gradient kernel against the bf16 matrix-core peak,
4 n d flops per chain-gradient; per-chain targets: the unadjusted step kernel
against HBM, its rows of x, u (and g) read and written once per chain).
time_to_bias: wall-clock and gradients per chain until the squared bias of
the second moments b^2_max first drops below 0.01 on the diagonal Gaussian
(closed-form moments), FP64 and FP32 state; the same on the rotated
ill-conditioned Gaussian, and on the logistic-regression posterior (bf16 and
plain FP64 GPU paths, reference moments from the FP64 oracle); with
--workload stochvol or phi4, on those posteriors in FP32 and FP64 state
(reference moments from the Laplace method over the hyperparameter grid, and
from the FP64 oracle).
cpu_baseline: the FP64 CPU oracle on a bounded sample of the same workload.
f64_gpu: the same run with the plain FP64 path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "chain-grad evals/s & time to bias b²<0.01, mixed/batched vs plain FP64 GPU"
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the bf16 gradient kernel on the logistic-regression workload, from FETCH_SIZE
# and WRITE_SIZE counters scaled by what they read for a plain copy of known size; kept with the counter
# summary under profiles/ and reset to None whenever the kernel changes.
LR_GRAD_TRAFFIC_BYTES = 35.09e6
# Instructions per launch of the same kernel (SQ_INSTS_VALU, which includes the MFMA instructions,
# SQ_INSTS_MFMA and SQ_INSTS_VALU_TRANS_F32, mean per dispatch), kept with the counter summary under
# profiles/ and reset to None whenever the kernel changes: they give the vector-ALU ceiling reported
# next to the matrix-core one.
LR_GRAD_INSTS = {"valu": 5710817, "mfma": 994048, "trans": 687360}
SIMDS, CLOCK_HZ = 1024, 2.4e9  # 256 CUs x 4 SIMDs at 2.4 GHz
# Vector instructions (SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F32) per launch of the per-chain step kernels,
# from the counter summary under profiles/; reset to None whenever a kernel changes.
STEP_INSTS = {
    "stochvol": {"unadj": (30373889, 909313), "mams": (945985857, 27885571)},
    "phi4": {"unadj": (20598784, 571392), "mams": (552036857, 9981952)},
}


def _valu_ceiling(valu, trans, kernel_ms, mfma=0):
    """Vector-ALU issue time of a launch spread over every SIMD (a wave64 vector instruction occupies a
    SIMD 4 cycles, a transcendental 16, an MFMA instruction, counted in valu, none of the vector ALU)
    against the kernel's duration."""
    cyc = (valu - mfma) * 4 + trans * 12
    t_valu = cyc / (SIMDS * CLOCK_HZ)
    t_k = kernel_ms * 1e-3
    return {"bound": "alu", "achieved": cyc / t_k / 1e9, "peak": SIMDS * CLOCK_HZ / 1e9,
            "unit": "G SIMD-cycles/s of vector-ALU issue", "frac": t_valu / t_k, "valu_issue_us": t_valu * 1e6}
N_UNADJ, N_ADJ = 1000, 67
# the dominant kernel's launches bracketed by HIP events inside the timed runs: one in LOG_EVERY
LOG_EVERY = int(os.environ.get("LAPS_BENCH_LOG_EVERY", "10"))


def _run_once(s, x0, n_unadj, n_adj):
    s.restart(x0)  # device-side cold start from x0, same workspace
    s.step_unadjusted(n_unadj)
    s.step_adjusted(n_adj)


WORKLOADS = {
    # name: (generator, default precision)
    "logreg": ("logreg", "bf16"),
    "gauss": ("gaussian", "f64"),
    "stochvol": ("stochvol", "f32"),
    "phi4": ("phi4", "f32"),
    "ill_gauss": ("ill_gaussian", "f64"),
    "batched": ("batched_mix", "mixed"),
}


def _cfg(n_unadj=N_UNADJ, n_adj=N_ADJ):
    return dict(switch_policy=1, max_steps_unadj=n_unadj, max_steps_total=n_unadj + 15 * n_adj)


def gpu_throughput(w, prec, steps, warmup, n_unadj=N_UNADJ, n_adj=N_ADJ, log=None, **extra):
    """Timed full runs.  log names a kernel ("grad" or "unadj") whose every
    launch inside the timed runs is bracketed by HIP events on the sampler's
    stream; its mean duration is returned as kernel_ms."""
    import torch
    from paper_2601_16696_amd import laps
    s = laps.Sampler(w, prec, **_cfg(n_unadj, n_adj), **extra)
    x0 = torch.as_tensor(w["x0"], device="cuda:0").to(s.x.dtype)
    for _ in range(warmup):
        _run_once(s, x0, n_unadj, n_adj)
    if log:
        # every LOG_EVERY-th launch (at most 5 gradients per integrator step of a 15-step trajectory)
        s.kernel_log(log, steps * (n_unadj + 75 * n_adj) // LOG_EVERY + 1, LOG_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _run_once(s, x0, n_unadj, n_adj)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel = None
    if log:
        n_launch, tot_ms = s.kernel_log_read()
        s.kernel_log(log, 0)
        kernel = dict(launches=n_launch, ms=tot_ms / max(n_launch, 1))
    st = s.stats()
    grad_ms = s.time_gradient(50)
    ms = (t1 - t0) / steps * 1e3
    grads = st["grads_per_chain"] * w["n_chains"]
    return dict(ms=ms, value=grads / (ms * 1e-3), stats=st, grad_ms=grad_ms, kernel=kernel, sampler=s)


def step_kernel_times(w, prec, n_reps=20):
    """HIP-event times of the unadjusted step kernel and the fused MAMS
    transition kernel alone, on a fresh sampler of the same workload (per-chain
    targets only)."""
    import torch
    from paper_2601_16696_amd import laps
    s = laps.Sampler(w, prec, **_cfg(40, 20))
    s.step_unadjusted(20)
    unadj = s.time_kernel("unadj", n_reps)
    s.step_unadjusted(20)
    s.step_adjusted(1)
    adj = s.time_kernel("adj", max(2, n_reps // 4))
    torch.cuda.synchronize()
    return unadj, adj


def measured_peaks():
    """Achievable peaks on this GPU, measured with library code: a streaming copy of 2 GiB (larger than
    the 256 MB last-level cache), read + write bytes over time, and a bf16 GEMM of 8192^3 through
    torch.matmul (hipBLASLt), 2 M N K flops over time; the best of 20 timed launches each."""
    import torch
    def best(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return min(ts)
    n = 1 << 29  # floats: 2 GiB per buffer
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    t_copy = best(lambda: b.copy_(a))
    del a, b
    m = 8192
    x = torch.randn(m, m, dtype=torch.bfloat16, device="cuda:0")
    y = torch.randn(m, m, dtype=torch.bfloat16, device="cuda:0")
    t_gemm = best(lambda: torch.matmul(x, y))
    del x, y
    torch.cuda.empty_cache()
    return {"hbm_copy_GBs": 2 * 4 * n / t_copy / 1e9, "copy_bytes": 2 * 4 * n,
            "bf16_gemm_TFLOPs": 2 * m ** 3 / t_gemm / 1e12, "gemm_shape": [m, m, m]}


def _oracle_slice(args):
    """One oracle process on its own slice of the chains (a worker of cpu_baseline_all_cores)."""
    name, k, n_chains, n_unadj, n_adj = args
    from oracle import oracle as orc
    from paper_2601_16696_amd import workloads
    w = getattr(workloads, name)()
    lo = (k * n_chains) % w["n_chains"]
    sub = dict(w)
    sub["x0"] = np.asarray(w["x0"])[lo:lo + n_chains]
    sub["n_chains"] = n_chains
    t0 = time.perf_counter()
    e = orc.Ensemble(orc.Target.from_workload(sub), n_chains, w["seed"] + k, switch_policy=1,
                     max_steps_unadj=n_unadj, max_steps_total=n_unadj + 15 * n_adj)
    e.init(sub["x0"])
    e.step_unadjusted(n_unadj)
    e.step_adjusted(n_adj)
    return e.stats()["grads_per_chain"] * n_chains, time.perf_counter() - t0


def cpu_baseline_all_cores(gen, n_chains=256, n_unadj=10, n_adj=1, procs=16):
    """The oracle as it stands on all host cores: procs independent processes (a fresh interpreter each,
    nothing of the GPU), each running the oracle on its own slice of n_chains chains with its own
    ensemble statistics; throughput = all chain-gradients over the slowest process's time."""
    import multiprocessing as mp
    procs = max(1, min(procs, os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_slice, [(gen, k, n_chains, n_unadj, n_adj) for k in range(procs)])
    grads = sum(r[0] for r in res)
    t = max(r[1] for r in res)
    return dict(value=grads / t, unit="chain-grad evals/s", cores=procs, kind="oracle",
                sample=f"{procs} processes x {n_chains} chains (distinct slices of {gen}), init + {n_unadj} "
                       f"unadjusted steps + {n_adj} MAMS transition each ({grads} chain-gradients, slowest process "
                       f"{t:.1f} s, single-threaded FP64 per process)")


CPU_SAMPLE = {  # about 10 s of single-threaded oracle work on the same workload
    "logreg": dict(n_chains=256, n_unadj=10, n_adj=1),
    "gauss": dict(n_chains=1024, n_unadj=600, n_adj=4),
    "stochvol": dict(n_chains=512, n_unadj=20, n_adj=1),
    "phi4": dict(n_chains=512, n_unadj=20, n_adj=1),
    "ill_gauss": dict(n_chains=1024, n_unadj=1000, n_adj=8),
}


def cpu_baseline(w, n_chains=256, n_unadj=10, n_adj=1):
    from oracle import oracle as orc
    n_chains = min(n_chains, w["n_chains"])
    sub = dict(w)
    sub["x0"] = w["x0"][:n_chains]
    sub["n_chains"] = n_chains
    t0 = time.perf_counter()
    e = orc.Ensemble(orc.Target.from_workload(sub), n_chains, w["seed"], switch_policy=1, max_steps_unadj=n_unadj,
                     max_steps_total=n_unadj + 15 * n_adj)
    e.init(sub["x0"])
    e.step_unadjusted(n_unadj)
    e.step_adjusted(n_adj)
    dt = time.perf_counter() - t0
    grads = e.stats()["grads_per_chain"] * n_chains
    return dict(value=grads / dt, unit="chain-grad evals/s", cores=1, kind="oracle",
                sample=f"first {n_chains} chains of {w['name']}, init + {n_unadj} unadjusted steps + {n_adj} MAMS "
                       f"transition ({grads} chain-gradients in {dt:.1f} s, single-threaded FP64)")


# --------------------------------------------------------------------------- time to bias
def _bias_reference(target):
    """Workload and the exact E[x_i^2], Var[x_i^2] of its target: closed forms
    for the two Gaussians (zero mean: E = s2, Var = 2 s2^2), the FP64
    oracle's reference moments for logistic regression, and the Laplace-method
    reference (oracle/sv_laplace.py, no sampler involved) for stochastic
    volatility, and the FP64 oracle's site-pooled reference for phi^4 (every
    site alike by translation invariance)."""
    from paper_2601_16696_amd import workloads
    if target in ("logreg", "stochvol", "phi4"):
        name = {"logreg": "logreg_n5000_d100_moments.json", "stochvol": "stochvol_T2427_laplace.json",
                "phi4": "phi4_L64_moments.json"}[target]
        ref = json.load(open(os.path.join(ROOT, "tests", "golden", name)))
        w = getattr(workloads, target)()
        return w, np.array(ref["E_x2"]), np.array(ref["Var_x2"])
    w = workloads.gaussian() if target == "gauss" else workloads.ill_gaussian()
    s2 = np.asarray(w["sigma2"] if target == "gauss" else w["cov_diag"])
    return w, s2, 2.0 * s2 * s2


def time_to_bias(prec, threshold=0.01, target="gauss", n_adj=N_ADJ):
    """The paper's automatic switch on a target with known second moments:
    the diagonal Gaussian ("gauss"), the rotated ill-conditioned one ("ill")
    or the logistic-regression posterior ("logreg", 4096 chains, reference
    moments from the FP64 oracle).  Walks the run step by step (untimed)
    computing b^2_i = (E[x_i^2] - E_p[x_i^2])^2 / Var_p[x_i^2] (section "Bias")
    from the ensemble after every unadjusted step and every transition, finds
    the first crossing of b^2_max < threshold, then times a fresh identical
    run truncated there (the run is deterministic for its seed)."""
    import torch
    from paper_2601_16696_amd import laps
    w, e_ref, v_ref = _bias_reference(target)
    cfg = dict(switch_policy=0, max_steps_unadj=N_UNADJ, max_steps_total=N_UNADJ + 15 * n_adj)
    s = laps.Sampler(w, prec, **cfg)
    e_t = torch.as_tensor(e_ref, device="cuda:0", dtype=torch.float64)
    v_t = torch.as_tensor(v_ref, device="cuda:0", dtype=torch.float64)

    def b2(argmax=False):
        x = s.positions().to(torch.float64)
        b = ((x * x).mean(0) - e_t) ** 2 / v_t
        if argmax:
            return float(b.max()), float(b.mean()), int(b.argmax())
        return float(b.max()), float(b.mean())

    n_u = n_a = 0
    hit = None
    below = after = 0
    while True:
        st = s.stats()
        if st["t"] >= cfg["max_steps_total"]:
            break
        if st["phase"] == 0 and n_u < N_UNADJ:
            s.step_unadjusted(1)
            n_u += 1
        else:
            s.step_adjusted(1)
            n_a += 1
        bmax, bavg = b2()
        if hit is not None:
            after += 1
            below += bmax < threshold
        elif bmax < threshold:
            st = s.stats()
            hit = dict(n_unadj=n_u, n_adj=n_a, t=st["t"], grads_per_chain=st["grads_per_chain"], b2_max=bmax,
                       b2_avg=bavg, phase_at_crossing=st["phase"])
    final = b2(argmax=True)
    out = dict(precision=prec, reached=hit is not None, b2_max_final=final[0], b2_avg_final=final[1],
               b2_argmax_final=final[2], unadjusted_steps_run=n_u)
    if hit is None:
        return out
    out.update(hit)
    out["fraction_of_later_points_below"] = below / max(after, 1)
    # timed re-run to the crossing
    s.restart(torch.as_tensor(w["x0"], device="cuda:0").to(s.x.dtype))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if hit["n_unadj"]:
        s.step_unadjusted(hit["n_unadj"])
    if hit["n_adj"]:
        s.step_adjusted(hit["n_adj"])
    torch.cuda.synchronize()
    out["ms"] = (time.perf_counter() - t0) * 1e3
    out["b2_max_rerun"] = b2()[0]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="logreg", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default=None, choices=["bf16", "f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-bias", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured copy and GEMM peaks")
    ap.add_argument("--full-rank-compare", type=int, default=0, metavar="P",
                    help="also time the same runs with the full-rank loss from P probes and report the ratio")
    ap.add_argument("--cpu-procs", type=int, default=16, help="oracle processes of the all-cores baseline (0: none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_16696_amd import laps, workloads
    laps.lib()
    gen, default_prec = WORKLOADS[args.workload]

    if args.workload == "batched":
        # The concurrent replay of the 16-target mix from segment graphs faulted the GPU (an illegal
        # memory access) on its first run and no cause has been shown; its logistic targets with d > 128
        # are refused by the library since, so the mix is not run.
        print("bench.py --workload batched is disabled: its graph replay of the 16-target mix faulted the GPU "
              "and the cause is not found", file=sys.stderr)
        sys.exit(3)

    prec = args.prec or default_prec
    w = getattr(workloads, gen)()
    N, d = w["n_chains"], w["d"]
    nonlocal_target = args.workload in ("logreg", "ill_gauss")
    r = gpu_throughput(w, prec, args.steps, args.warmup, log="grad" if nonlocal_target else "unadj")
    kern = r["kernel"]
    if args.workload == "logreg":
        n = w["X"].shape[0]
        work = 4.0 * n * d * N  # flops of X theta and X^T r per ensemble gradient
        peak = PEAK_BF16_TFLOPS if prec == "bf16" else 78.6
        achieved = work / (kern["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma" if prec == "bf16" else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": LR_GRAD_TRAFFIC_BYTES if prec == "bf16" else None,
                "traffic_unit": "bytes per launch",
                "kernel": "k_lr_grad_bf16_pipe<4, 7>" if prec == "bf16" else "k_lr_grad_f64", "kernel_ms": kern["ms"],
                "launches_timed": kern["launches"], "isolated_kernel_ms": r["grad_ms"],
                "algorithmic_flops_per_launch": work}
        if prec == "bf16" and LR_GRAD_INSTS:
            vc = _valu_ceiling(LR_GRAD_INSTS["valu"], LR_GRAD_INSTS["trans"], kern["ms"], LR_GRAD_INSTS["mfma"])
            t_mfma = LR_GRAD_INSTS["mfma"] * 16 / (SIMDS * CLOCK_HZ)  # 16 cycles per 16x16x32 bf16 MFMA
            vc["mfma_issue_us"] = t_mfma * 1e6
            vc["frac_of_valu_plus_mfma_in_series"] = (vc["valu_issue_us"] * 1e-6 + t_mfma) / (kern["ms"] * 1e-3)
            roof["valu_ceiling"] = vc
        precision = ("bf16 matrix-core gradient, fp32 state, fp64 energy error and reductions"
                     if prec == "bf16" else "fp64 throughout")
        extra = {"n": n}
    elif args.workload == "ill_gauss":
        work = 2.0 * d * d * N  # flops of A x per ensemble gradient
        peak = 78.6 if prec == "f64" else 157.3  # dense matrix-core FP64 / FP32
        achieved = work / (kern["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None, "kernel": f"k_dense_grad<{'double' if prec == 'f64' else 'float'}>",
                "kernel_ms": kern["ms"], "launches_timed": kern["launches"], "isolated_kernel_ms": r["grad_ms"],
                "algorithmic_flops_per_launch": work}
        precision = "fp64 throughout" if prec == "f64" else "fp32 state, fp64 energy error and reductions"
        extra = {"condition_number": w["cond"]}
    else:
        rs = 8 if prec == "f64" else 4
        unadj_ms, adj_ms = step_kernel_times(w, prec)
        # algorithmic bytes of one unadjusted step: x and u read and written once per chain (4 rows);
        # the stochastic-volatility and phi^4 kernels also keep g in HBM (2 more rows), an implementation
        # choice reported apart and not counted
        work = float(4 * rs * d * N)
        kept_g = float(2 * rs * d * N) if args.workload != "gauss" else 0.0
        achieved = work / (kern["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None, "kernel": "k_unadj (unadjusted step)",
                "kernel_ms": kern["ms"], "launches_timed": kern["launches"], "isolated_kernel_ms": unadj_ms,
                "algorithmic_bytes_per_launch": work, "kept_gradient_bytes_per_launch": kept_g,
                "adjusted_transition_kernel_ms": adj_ms, "gradient_only_ms": r["grad_ms"]}
        insts = STEP_INSTS.get(args.workload) if prec == "f32" else None
        if insts:
            roof["valu_ceiling"] = _valu_ceiling(*insts["unadj"], kern["ms"])
            roof["adjusted_transition_valu_ceiling"] = _valu_ceiling(*insts["mams"], adj_ms)
        precision = "fp64 throughout" if prec == "f64" else "fp32 state, fp64 energy error and reductions"
        extra = {}
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "chain-grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": dict({
            "workload": f"{w['name']}: full LAPS run, {N_UNADJ} unadjusted steps + {N_ADJ} MAMS transitions",
            "chains": N, "d": d, "precision": precision,
            "grads_per_chain": r["stats"]["grads_per_chain"], "parallelism": "single GPU"}, **extra),
        "roofline": roof,
        "final_state": {"acc_mean": r["stats"]["acc_mean"], "eps": r["stats"]["eps"], "t": r["stats"]["t"],
                        "n_nonfinite": r["stats"]["n_nonfinite"]},
    }
    del r["sampler"]
    torch.cuda.empty_cache()
    if not args.no_f64 and prec != "f64":
        r64 = gpu_throughput(w, "f64", 1, 0)
        line["f64_gpu"] = {"value": r64["value"], "ms_per_step": r64["ms"], "gradient_ms": r64["grad_ms"],
                           "speedup_of_mixed": line["value"] / r64["value"]}
        del r64["sampler"]
    if not args.no_bias and args.workload == "logreg":
        line["time_to_bias"] = {"workload": "gaussian_diag_d100_N1024 (closed-form moments), automatic switch",
                                "criterion": "first step with b2_max < 0.01",
                                "f64": time_to_bias("f64"), "f32": time_to_bias("f32")}
        line["time_to_bias_ill_conditioned"] = {
            "workload": "ill_gaussian_d100_N1024: randomly rotated Gaussian, covariance eigenvalues ~ Gamma(0.5, 1) "
                        "(condition ~1e5), closed-form moments, automatic switch",
            "criterion": "first step with b2_max < 0.01",
            "paper_laps_grads_context": 308,
            "f64": time_to_bias("f64", target="ill"), "f32": time_to_bias("f32", target="ill")}
        lb, l64 = time_to_bias("bf16", target="logreg"), time_to_bias("f64", target="logreg")
        line["time_to_bias_logistic"] = {
            "workload": "logreg_n5000_d100_N4096, automatic switch; E_p[x_i^2] and Var_p[x_i^2] from the FP64 oracle "
                        "(8 x 64 chains, 60 pooled MAMS transitions each; tests/golden/logreg_n5000_d100_moments.json)",
            "criterion": "first step with b2_max < 0.01",
            "bf16": lb, "f64": l64,
            "speedup_of_mixed": (l64["ms"] / lb["ms"]) if lb.get("ms") and l64.get("ms") else None,
            "grads_per_chain_at_crossing": {"bf16": lb.get("grads_per_chain"), "f64": l64.get("grads_per_chain")}}
    if not args.no_bias and args.workload == "stochvol":
        l32 = time_to_bias("f32", target="stochvol", n_adj=400)
        l64 = time_to_bias("f64", target="stochvol", n_adj=400)
        line["time_to_bias_stochvol"] = {
            "workload": "stochvol_T2427_N4096, automatic switch; E_p[x_i^2] and Var_p[x_i^2] from the Laplace method "
                        "over a (s, r) grid (oracle/sv_laplace.py; tests/golden/stochvol_T2427_laplace.json)",
            "criterion": "first step with b2_max < 0.01", "paper_laps_grads_context": 1325,
            "f32": l32, "f64": l64,
            "speedup_of_f32": (l64["ms"] / l32["ms"]) if l32.get("ms") and l64.get("ms") else None}
    if not args.no_bias and args.workload == "phi4":
        l32, l64 = time_to_bias("f32", target="phi4"), time_to_bias("f64", target="phi4")
        line["time_to_bias_phi4"] = {
            "workload": "phi4_L64_N2048, automatic switch; E_p[x_i^2] and Var_p[x_i^2] from the FP64 oracle, all sites "
                        "pooled (tests/golden/phi4_L64_moments.json)",
            "criterion": "first step with b2_max < 0.01", "f32": l32, "f64": l64,
            "speedup_of_f32": (l64["ms"] / l32["ms"]) if l32.get("ms") and l64.get("ms") else None}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, **CPU_SAMPLE[args.workload])
        if args.cpu_procs > 0:
            line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(gen, procs=args.cpu_procs,
                                                                    **CPU_SAMPLE[args.workload])
    if args.full_rank_compare > 0:
        rf = gpu_throughput(w, prec, args.steps, args.warmup, full_rank_probes=args.full_rank_compare)
        del rf["sampler"]
        line["full_rank_loss"] = {
            "probes": args.full_rank_compare, "ms_per_step_diagonal": r["ms"], "ms_per_step_full_rank": rf["ms"],
            "run_time_ratio": rf["ms"] / r["ms"],
            "note": "section 'Equipartition condition' (full-rank form); the paper's Table 4 gives full-rank / "
                    "diagonal run-time ratios of 0.95-1.10 on its targets (context only)"}
    if not args.no_peaks:
        pk = measured_peaks()
        line["measured_peaks"] = pk
        if roof["unit"] == "TFLOP/s" and roof["bound"] == "mfma" and prec == "bf16":
            roof["frac_of_measured_peak"] = roof["achieved"] / pk["bf16_gemm_TFLOPs"]
        elif roof["unit"] == "GB/s":
            roof["frac_of_measured_peak"] = roof["achieved"] / pk["hbm_copy_GBs"]
    print(json.dumps(line))


if __name__ == "__main__":
    main()
