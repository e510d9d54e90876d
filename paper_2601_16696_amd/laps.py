"""Thin Python binding of the LAPS C ABI (include/laps.h).

Argument marshalling only: every step of the sampler runs in the HIP kernels
of liblaps_hip.so.  PyTorch provides device memory and the stream.  There is
no CPU fallback: without the built library every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblaps_hip.so")

OK, EINVAL, EDEVICE, ENONFINITE, EPHASE, EWORKSPACE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
F64, F32, MIXED_BF16 = 0, 1, 2
GAUSS_DIAG, LOGREG, STOCHVOL, PHI4, CALLBACK, GAUSS_DENSE = 0, 1, 2, 3, 4, 5
PRECISIONS = {"f64": F64, "f32": F32, "bf16": MIXED_BF16, F64: F64, F32: F32, MIXED_BF16: MIXED_BF16}
KINDS = {"gauss": GAUSS_DIAG, "logreg": LOGREG, "stochvol": STOCHVOL, "phi4": PHI4, "callback": CALLBACK,
         "gauss_dense": GAUSS_DENSE}
# laps_grad_cb: (user, x_dev, g_dev, logp_dev, n_chains, d, ld, stream) -> int
GRAD_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p)


class LapsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"LAPS status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int64), ("d", ctypes.c_int64), ("prec", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("C", ctypes.c_double), ("alpha", ctypes.c_double),
                ("eps0_factor", ctypes.c_double), ("switch_tol", ctypes.c_double),
                ("window_frac", ctypes.c_double), ("acc_tol", ctypes.c_double), ("acc_target", ctypes.c_double),
                ("L_partial_factor", ctypes.c_double), ("n_steps_traj", ctypes.c_int32),
                ("integrator_adj", ctypes.c_int32), ("eevpd_mode", ctypes.c_int32),
                ("switch_policy", ctypes.c_int32), ("max_steps_unadj", ctypes.c_int64),
                ("max_steps_total", ctypes.c_int64), ("team_lanes", ctypes.c_int32), ("full_rank_probes", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("grad_workgroups", ctypes.c_int32),
                ("eps_fixed", ctypes.c_double), ("dynamics", ctypes.c_int32)]


class TargetS(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("d", ctypes.c_int64), ("data", ctypes.c_void_p * 4),
                ("dims", ctypes.c_int64 * 4), ("scal", ctypes.c_double * 4), ("cb", ctypes.c_void_p),
                ("cb_user", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("grads_per_chain", ctypes.c_int64), ("phase", ctypes.c_int32),
                ("adapt", ctypes.c_int32), ("switch_ready", ctypes.c_int32), ("status_bits", ctypes.c_int32),
                ("eps", ctypes.c_double), ("L", ctypes.c_double), ("eevpd", ctypes.c_double),
                ("eevpd_target", ctypes.c_double), ("dtilde", ctypes.c_double), ("max_delta", ctypes.c_double),
                ("acc_mean", ctypes.c_double), ("n_nonfinite", ctypes.c_int64), ("integrator", ctypes.c_int32),
                ("have_lo", ctypes.c_int32), ("have_hi", ctypes.c_int32), ("ring_full", ctypes.c_int32),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("a_star", ctypes.c_double),
                ("sum_var", ctypes.c_double)]


EXPORTS = ["laps_config_default", "laps_row_stride", "laps_workspace_size", "laps_init", "laps_init_static",
           "laps_step_unadjusted",
           "laps_step_adjusted", "laps_ensemble_stats", "laps_target_eval", "laps_eval", "laps_philox_words",
           "laps_philox_normals", "laps_time_gradient", "laps_time_kernel", "laps_kernel_log",
           "laps_kernel_log_read", "laps_restart", "laps_graph_create",
           "laps_graph_launch", "laps_graph_destroy", "laps_buffer", "laps_destroy", "laps_status_string",
           "laps_last_error"]

_lib = None


def lib():
    """Loads the built HIP library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LapsError(EUNSUPPORTED, f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                                      "(python -m paper_2601_16696_amd.build)")
    # torch first: its HIP runtime then provides the soname libamdhip64.so.7
    # that the library links, so the process holds one runtime, not two.
    _torch()
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, U64, U32, D = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32,
                                ctypes.c_double)
    sig = {
        "laps_config_default": (None, [P, I64, I64]),
        "laps_row_stride": (I64, [I64]),
        "laps_workspace_size": (I32, [P, P, P]),
        "laps_init": (I32, [P, P, P, P, P, ctypes.c_size_t, P, P]),
        "laps_init_static": (I32, [P, P, P, P, P, P]),
        "laps_step_unadjusted": (I32, [P, I64]),
        "laps_step_adjusted": (I32, [P, I64]),
        "laps_ensemble_stats": (I32, [P, P, P]),
        "laps_target_eval": (I32, [P, I32, P, P, P, I64, P]),
        "laps_eval": (I32, [P, P, P, P]),
        "laps_philox_words": (I32, [P, P, I64, U64, P]),
        "laps_philox_normals": (I32, [U64, I64, I64, U64, U32, U32, I32, P, P]),
        "laps_time_gradient": (I32, [P, I32, P]),
        "laps_time_kernel": (I32, [P, I32, I32, P]),
        "laps_kernel_log": (I32, [P, I32, I32, I32]),
        "laps_kernel_log_read": (I32, [P, P, P]),
        "laps_restart": (I32, [P, P]),
        "laps_graph_create": (I32, [P, I32, I32, P, I64, I64, P]),
        "laps_graph_launch": (I32, [P, P]),
        "laps_graph_destroy": (I32, [P]),
        "laps_buffer": (P, [P, I32]),
        "laps_destroy": (I32, [P]),
        "laps_status_string": (ctypes.c_char_p, [I32]),
        "laps_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st: int, ctx=None):
    if st != OK:
        msg = lib().laps_last_error(ctx).decode() if ctx is not None else lib().laps_last_error(None).decode()
        raise LapsError(st, f"{lib().laps_status_string(st).decode()} ({msg})")


def row_stride(d: int) -> int:
    return lib().laps_row_stride(d)


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _state_dtype(prec: int):
    torch = _torch()
    return torch.float64 if prec == F64 else torch.float32


def bf16_bits(a: np.ndarray) -> np.ndarray:
    """Upper 16 bits of float32 values that are already bf16-exact."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


class Target:
    """Device-resident target description (keeps its tensors alive)."""

    def __init__(self, w: dict, prec, device="cuda:0"):
        torch = _torch()
        self.prec = PRECISIONS[prec]
        self.kind = KINDS[w["kind"]]
        self.d = int(w["d"])
        self.keep = []
        s = TargetS()
        s.kind = self.kind
        s.d = self.d
        if self.kind == GAUSS_DIAG:
            t = torch.as_tensor(np.asarray(w["sigma2"], dtype=np.float64), device=device)
            self.keep.append(t)
            s.data[0] = t.data_ptr()
        elif self.kind == STOCHVOL:
            t = torch.as_tensor(np.asarray(w["y"], dtype=np.float64), device=device)
            self.keep.append(t)
            s.data[0] = t.data_ptr()
            s.dims[0] = int(w["y"].shape[0])
        elif self.kind == PHI4:
            s.dims[0] = int(w["side"])
            s.scal[0] = float(w["m2"])
            s.scal[1] = float(w["lam"])
        elif self.kind == LOGREG:
            X = np.asarray(w["X"])
            if self.prec == F64:
                tX = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float64), device=device)
            else:
                tX = torch.as_tensor(bf16_bits(X).view(np.int16), device=device)
            ty = torch.as_tensor(np.asarray(w["y"], dtype=np.float64), device=device)
            self.keep += [tX, ty]
            s.data[0] = tX.data_ptr()
            s.data[1] = ty.data_ptr()
            s.dims[0] = int(X.shape[0])
        elif self.kind == GAUSS_DENSE:
            t = torch.as_tensor(np.ascontiguousarray(w["prec"], dtype=np.float64), device=device)
            self.keep.append(t)
            s.data[0] = t.data_ptr()
        elif self.kind == CALLBACK:
            self._set_callback(w["fn"])
            s.cb = ctypes.cast(self._cb, ctypes.c_void_p)
        self.s = s

    def _set_callback(self, fn):
        """fn(x, g, logp) is called with torch views of the library's buffers
        (x, g: [N, ld] in the state type; logp: [N] float64) on the stream the
        library names, and must write g[:, :d] = grad log p(x) and logp.  The
        views alias device memory registered in self.buffers (the sampler's
        positions and workspace)."""
        import traceback
        self.buffers = []

        def view(ptr, shape, dtype):
            torch = _torch()
            nbytes = int(np.prod(shape)) * torch.empty((), dtype=dtype).element_size()
            for t in self.buffers:
                base = t.data_ptr()
                size = t.numel() * t.element_size()
                if base <= ptr and ptr + nbytes <= base + size:
                    off = ptr - base
                    return t.reshape(-1).view(torch.uint8)[off:off + nbytes].view(dtype).view(shape)
            raise RuntimeError("callback pointer outside the registered buffers")

        def tramp(user, xp, gp, lpp, n, d, ld, stream):
            try:
                torch = _torch()
                dt = _state_dtype(self.prec)
                x, g = view(xp, (n, ld), dt), view(gp, (n, ld), dt)
                lp = view(lpp, (n,), torch.float64)
                st = torch.cuda.ExternalStream(stream) if stream else torch.cuda.default_stream()
                with torch.cuda.stream(st):
                    fn(x, g, lp)
                return 0
            except Exception:
                traceback.print_exc()
                return 1

        self._cb = GRAD_CB(tramp)

    def eval(self, x, grad: bool = True, stream=None):
        """log p [n] (float64) and gradient [n, d] for rows of x ([n, d] or padded [n, ld])."""
        torch = _torch()
        ld = row_stride(self.d)
        dt = _state_dtype(self.prec)
        n = x.shape[0]
        if x.shape[1] != ld or x.dtype != dt or not x.is_contiguous():
            xp = torch.zeros((n, ld), dtype=dt, device=x.device)
            xp[:, :self.d] = x[:, :self.d].to(dt)
        else:
            xp = x
        lp = torch.empty(n, dtype=torch.float64, device=x.device)
        g = torch.empty((n, ld), dtype=dt, device=x.device) if grad else None
        st = lib().laps_target_eval(ctypes.byref(self.s), self.prec, ctypes.c_void_p(xp.data_ptr()),
                                    ctypes.c_void_p(lp.data_ptr()),
                                    ctypes.c_void_p(g.data_ptr()) if grad else None, n, _stream_ptr(stream))
        _check(st)
        return lp, (g[:, :self.d] if grad else None)


class Sampler:
    """One LAPS ensemble on the current GPU.

    w: workload dict (see workloads.py); x0: [N, d] initial positions.
    cfg keywords override the paper's defaults (laps_config fields)."""

    def __init__(self, w: dict, prec="f64", x0=None, seed=None, device="cuda:0", u0=None, static_workspace=False,
                 **cfg):
        torch = _torch()
        self.prec = PRECISIONS[prec]
        self.target = Target(w, self.prec, device)
        x0 = w["x0"] if x0 is None else x0
        N, d = int(x0.shape[0]), int(w["d"])
        self.N, self.d = N, d
        self.ld = row_stride(d)
        c = Config()
        lib().laps_config_default(ctypes.byref(c), N, d)
        c.prec = self.prec
        c.seed = int(w.get("seed", 0) if seed is None else seed)
        for k, v in cfg.items():
            if not hasattr(c, k):
                raise TypeError(f"unknown config field {k}")
            setattr(c, k, v)
        self.cfg = c
        dt = _state_dtype(self.prec)
        self.x = torch.zeros((N, self.ld), dtype=dt, device=device)
        self.x[:, :d] = torch.as_tensor(np.asarray(x0), device=device).to(dt)
        self.u0 = None
        if u0 is not None:
            self.u0 = torch.zeros((N, self.ld), dtype=dt, device=device)
            self.u0[:, :d] = torch.as_tensor(np.asarray(u0), device=device).to(dt)
        nbytes = ctypes.c_size_t(0)
        _check(lib().laps_workspace_size(ctypes.byref(c), ctypes.byref(self.target.s), ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        # static_workspace: laps_init_static, the library's own device array (no workspace tensor)
        self.static_workspace = bool(static_workspace)
        self.ws = None if self.static_workspace else torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        if self.target.kind == CALLBACK:
            self.target.buffers += [t for t in (self.x, self.ws) if t is not None]
        self.per_dim = torch.empty((4, d), dtype=torch.float64, device=device)
        self.ctx = ctypes.c_void_p()
        self._init()

    def _init(self):
        u0 = ctypes.c_void_p(self.u0.data_ptr()) if self.u0 is not None else None
        if self.static_workspace:
            st = lib().laps_init_static(ctypes.byref(self.cfg), ctypes.byref(self.target.s),
                                        ctypes.c_void_p(self.x.data_ptr()), u0, _stream_ptr(), ctypes.byref(self.ctx))
        else:
            st = lib().laps_init(ctypes.byref(self.cfg), ctypes.byref(self.target.s), ctypes.c_void_p(self.x.data_ptr()),
                                 u0, ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, _stream_ptr(),
                                 ctypes.byref(self.ctx))
        _check(st)

    def reinit(self, x0):
        """Starts a fresh run from x0 (a device tensor [N, d]) in the same memory."""
        if self.ctx:
            lib().laps_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()
        self.x[:, :self.d].copy_(x0)
        self._init()

    def restart(self, x0=None):
        """Enqueues a fresh run from x0 (device tensor [N, d]; None keeps the
        current positions) without reallocating: the state laps_init leaves."""
        if x0 is not None:
            self.x[:, :self.d].copy_(x0)
        _check(lib().laps_restart(self.ctx, None), self.ctx)

    def time_kernel(self, which: str, n_reps: int = 20) -> float:
        """Mean milliseconds of the unadjusted step kernel ("unadj") or the
        fused adjusted transition kernel ("adj") alone (per-chain targets)."""
        ms = ctypes.c_float(0.0)
        _check(lib().laps_time_kernel(self.ctx, {"unadj": 1, "adj": 2}[which], n_reps, ctypes.byref(ms)), self.ctx)
        return ms.value

    KERNELS = {"unadj": 1, "adj": 2, "grad": 3}

    def kernel_log(self, which: str, capacity: int, every: int = 1):
        """Records HIP events around every `every`-th launch of one kernel of
        the following steps, up to `capacity` launches ("unadj" / "adj":
        per-chain step kernels, "grad": the logistic-regression gradient
        kernel); capacity 0 stops."""
        _check(lib().laps_kernel_log(self.ctx, self.KERNELS[which] if capacity else 0, capacity, every), self.ctx)

    def kernel_log_read(self):
        """(launches logged, summed milliseconds) of the kernel log."""
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(lib().laps_kernel_log_read(self.ctx, ctypes.byref(n), ctypes.byref(ms)), self.ctx)
        return n.value, ms.value

    def eval(self, x, grad: bool = True):
        """log p [N] (float64) and gradient [N, d] of the sampler's target at
        positions x ([N, d] or padded [N, ld]) through the context
        (laps_eval): works for every target kind; enqueued on the sampler's
        stream between steps, the sampler's state is left alone."""
        torch = _torch()
        dt = _state_dtype(self.prec)
        if x.shape[0] != self.N:
            raise ValueError(f"x needs {self.N} rows")
        if x.shape[1] != self.ld or x.dtype != dt or not x.is_contiguous():
            xp = torch.zeros((self.N, self.ld), dtype=dt, device=x.device)
            xp[:, :self.d] = x[:, :self.d].to(dt)
        else:
            xp = x
        lp = torch.empty(self.N, dtype=torch.float64, device=x.device)
        g = torch.empty((self.N, self.ld), dtype=dt, device=x.device) if grad else None
        if self.target.kind == CALLBACK:
            self.target.buffers.append(xp)
        try:  # a callback runs inside this call, so x is registered only meanwhile
            _check(lib().laps_eval(self.ctx, ctypes.c_void_p(xp.data_ptr()), ctypes.c_void_p(lp.data_ptr()),
                                   ctypes.c_void_p(g.data_ptr()) if grad else None), self.ctx)
        finally:
            if self.target.kind == CALLBACK:
                self.target.buffers.pop()
        return lp, (g[:, :self.d] if grad else None)

    def time_gradient(self, n_reps: int = 20) -> float:
        """Mean milliseconds of one ensemble gradient evaluation (HIP events on the sampler's stream)."""
        ms = ctypes.c_float(0.0)
        _check(lib().laps_time_gradient(self.ctx, n_reps, ctypes.byref(ms)), self.ctx)
        return ms.value

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None:
            _lib.laps_destroy(ctx)
            self.ctx = None

    def step_unadjusted(self, n: int = 1):
        _check(lib().laps_step_unadjusted(self.ctx, n), self.ctx)

    def step_adjusted(self, n: int = 1):
        _check(lib().laps_step_adjusted(self.ctx, n), self.ctx)

    def stats(self, per_dim: bool = False) -> dict:
        s = Stats()
        st = lib().laps_ensemble_stats(self.ctx, ctypes.byref(s),
                                       ctypes.c_void_p(self.per_dim.data_ptr()) if per_dim else None)
        if st not in (OK, ENONFINITE):
            _check(st, self.ctx)
        out = {f: getattr(s, f) for f, _ in s._fields_}
        out["status"] = st
        return out

    def positions(self):
        return self.x[:, :self.d]

    def buffer(self, name: str):
        """Views of workspace arrays: u, g ([N, d]), logp, delta, acc ([N]), sigma ([d])."""
        torch = _torch()
        if self.ws is None:
            raise LapsError(EUNSUPPORTED, "buffer views need a caller workspace (not static_workspace)")
        idx = {"u": 0, "g": 1, "logp": 2, "delta": 3, "acc": 4, "sigma": 5}[name]
        ptr = lib().laps_buffer(self.ctx, idx)
        off = ptr - self.ws.data_ptr()
        dt = _state_dtype(self.prec)
        es = 8 if dt == torch.float64 else 4
        if name in ("u", "g"):
            n = self.N * self.ld * es
            return self.ws[off:off + n].view(dt).view(self.N, self.ld)[:, :self.d]
        if name == "sigma":
            return self.ws[off:off + self.ld * es].view(dt)[:self.d]
        return self.ws[off:off + self.N * 8].view(torch.float64)


class RunGraph:
    """One executable graph replaying a segment of LAPS runs of several
    samplers concurrently, each on the created (non-default) stream it was
    made on: an optional restart, n_unadj unadjusted steps, n_adj adjusted
    transitions.  Segments are created in run order and launched in the same
    order.

    x0s: per-sampler device tensors [N, ld] in the sampler's state type, the
    starting positions of a restart (None restarts from the positions the
    sampler holds at replay time)."""

    def __init__(self, samplers, n_unadj: int, n_adj: int, restart: bool = False, x0s=None):
        self.samplers = list(samplers)
        self.x0s = None if x0s is None else list(x0s)
        n = len(self.samplers)
        ctxs = (ctypes.c_void_p * n)(*[s.ctx.value for s in self.samplers])
        xp = None
        if self.x0s is not None:
            xp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in self.x0s])
        self.g = ctypes.c_void_p()
        _check(lib().laps_graph_create(ctxs, n, 1 if restart else 0, xp, n_unadj, n_adj, ctypes.byref(self.g)))

    def launch(self, stream=None):
        _check(lib().laps_graph_launch(self.g, _stream_ptr(stream)))

    def __del__(self):
        g = getattr(self, "g", None)
        if g and _lib is not None:
            _lib.laps_graph_destroy(g)
            self.g = None


def philox_words(ctr: np.ndarray, seed: int, device="cuda:0") -> np.ndarray:
    torch = _torch()
    c = torch.as_tensor(np.ascontiguousarray(ctr, dtype=np.uint64).view(np.int64), device=device)
    out = torch.empty_like(c)
    _check(lib().laps_philox_words(ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   c.shape[0], seed, _stream_ptr()))
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64)


def philox_normals(seed: int, n_chains: int, d: int, t: int, tag: int, substep: int, prec="f64", device="cuda:0"):
    torch = _torch()
    p = PRECISIONS[prec]
    out = torch.empty((n_chains, row_stride(d)), dtype=_state_dtype(p), device=device)
    _check(lib().laps_philox_normals(seed, n_chains, d, t, tag, substep, p, ctypes.c_void_p(out.data_ptr()),
                                     _stream_ptr()))
    return out[:, :d]


_LOG_DENSITY_FN = None


def log_density(target, x):
    """log p of the rows of x ([n, d]) as a differentiable torch function: the
    forward pass evaluates log p and its gradient together in the library's
    target kernels, the backward pass scales the saved gradient by the
    incoming one.  target is a Target (standalone evaluation, laps_target_eval:
    diagonal Gaussian, stochastic volatility, phi^4, any n) or a Sampler
    (laps_eval through its context: every target kind, including logistic
    regression and the dense Gaussian, with x of the sampler's chain count)."""
    global _LOG_DENSITY_FN
    torch = _torch()
    if _LOG_DENSITY_FN is None:
        class _LogDensity(torch.autograd.Function):
            @staticmethod
            def forward(ctx, xx, tgt):
                lp, g = tgt.eval(xx, grad=True)
                ctx.save_for_backward(g)
                ctx.xdtype = xx.dtype
                return lp.to(xx.dtype)

            @staticmethod
            def backward(ctx, gout):
                (g,) = ctx.saved_tensors
                return (gout[:, None].to(torch.float64) * g.to(torch.float64)).to(ctx.xdtype), None

        _LOG_DENSITY_FN = _LogDensity
    return _LOG_DENSITY_FN.apply(x, target)


def _shape_candidates(w: dict, prec) -> list:
    """Launch shapes worth timing for a workload: team widths and workgroup
    sizes of the per-chain kernels, or gradient workgroup counts and update
    workgroup sizes for logistic regression (others have one shape)."""
    kind = KINDS[w["kind"]]
    if kind in (GAUSS_DIAG, STOCHVOL, PHI4):
        out = [dict(team_lanes=0, block_threads=0)]
        for T in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512):
            for b in ((0, 64, 128) if T <= 64 else (0,)):
                out.append(dict(team_lanes=T, block_threads=b))
        return out
    if kind == LOGREG:
        return [dict(grad_workgroups=g, block_threads=b) for g in (0, 256, 512, 1024) for b in (0, 64, 128)]
    return [dict()]


def _tune_key(w: dict, prec) -> str:
    n = int(np.asarray(w["X"]).shape[0]) if w["kind"] == "logreg" else 0
    pname = {F64: "f64", F32: "f32", MIXED_BF16: "bf16"}[PRECISIONS[prec]]
    return f"{w['kind']}:d={int(w['d'])}:n={n}:N={int(w['n_chains'])}:prec={pname}"


def autotune(w: dict, prec="f64", cache: str | None = None, n_steps: int = 20, **cfg) -> dict:
    """Times n_steps unadjusted steps of every valid launch shape of the
    workload (after a warm-up) and returns the fastest shape's config fields,
    with its ms per step.  Results are kept in the JSON file `cache` (if
    given) under the key (target kind, d, n, N, precision); a cached key is
    returned without timing.  A fresh search also returns every shape's time
    under "trials".  The shapes change rounding order only: every
    one runs the same method."""
    import json
    torch = _torch()
    key = _tune_key(w, prec)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            return dict(table[key], cached=True)
    best, errors, trials = None, [], []
    base = dict(cfg)
    base.setdefault("switch_policy", 1)
    base.setdefault("max_steps_unadj", 10 * n_steps + 10)
    for cand in _shape_candidates(w, prec):
        try:
            s = Sampler(w, prec, **base, **cand)
        except LapsError as e:
            errors.append(f"{cand}: {e}")
            continue  # not a valid shape for this size
        s.step_unadjusted(2)
        ms = float("inf")
        for _ in range(2):  # the faster of two timings, against clock noise
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step_unadjusted(n_steps)
            e1.record()
            e1.synchronize()
            ms = min(ms, e0.elapsed_time(e1) / n_steps)
        del s
        trials.append(dict(cand, ms_per_step=ms))
        if best is None or ms < best["ms_per_step"]:
            best = dict(cand, ms_per_step=ms)
    if best is None:
        raise LapsError(EUNSUPPORTED, "no valid launch shape: " + "; ".join(errors[:3]))
    if cache:
        table[key] = best
        with open(cache + ".tmp", "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(cache + ".tmp", cache)
    return dict(best, cached=False, trials=trials)
