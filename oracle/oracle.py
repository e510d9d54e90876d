"""ctypes binding of the plain FP64 CPU oracle of LAPS (arXiv 2601.16696).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  The oracle shares no
code with the GPU library; the only thing both sides see is the seeded input
generator module, which holds none of the method's arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "laps_oracle.c")
LIB = os.path.join(HERE, "liblaps_oracle.so")

GAUSS_DIAG, LOGREG, STOCHVOL, PHI4, GAUSS_DENSE = 0, 1, 2, 3, 5
TAG_O_FIRST, TAG_O_SECOND, TAG_FULL_REFRESH, TAG_MH, TAG_INIT_DIR = 1, 2, 3, 4, 5
PH_UNADJ, PH_SWITCH_PENDING, PH_ADJ = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Target(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("d", ctypes.c_int64), ("a", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("n", ctypes.c_int64), ("p0", ctypes.c_double),
                ("p1", ctypes.c_double)]


class _Config(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int64), ("d", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("C", ctypes.c_double), ("alpha", ctypes.c_double), ("eps0_factor", ctypes.c_double),
                ("switch_tol", ctypes.c_double), ("window_frac", ctypes.c_double),
                ("acc_tol", ctypes.c_double), ("acc_target", ctypes.c_double),
                ("L_partial_factor", ctypes.c_double), ("n_steps_traj", ctypes.c_int32),
                ("integrator_adj", ctypes.c_int32), ("eevpd_mode", ctypes.c_int32),
                ("switch_policy", ctypes.c_int32), ("max_steps_unadj", ctypes.c_int64),
                ("max_steps_total", ctypes.c_int64), ("full_rank_probes", ctypes.c_int32),
                ("eps_fixed", ctypes.c_double), ("dynamics", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("grads_per_chain", ctypes.c_int64), ("phase", ctypes.c_int32),
                ("adapt", ctypes.c_int32), ("switch_ready", ctypes.c_int32), ("status_bits", ctypes.c_int32),
                ("eps", ctypes.c_double), ("L", ctypes.c_double), ("eevpd", ctypes.c_double),
                ("eevpd_target", ctypes.c_double), ("dtilde", ctypes.c_double), ("max_delta", ctypes.c_double),
                ("acc_mean", ctypes.c_double), ("n_nonfinite", ctypes.c_int64), ("integrator", ctypes.c_int32),
                ("have_lo", ctypes.c_int32), ("have_hi", ctypes.c_int32), ("ring_full", ctypes.c_int32),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("a_star", ctypes.c_double),
                ("sum_var", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P, D, I64, U64, I32, U32 = (ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                                    ctypes.c_int32, ctypes.c_uint32)
        sig = {
            "orc_philox4x64_10": (None, [P, P, P]),
            "orc_u01": (D, [U64]),
            "orc_normals": (None, [U64, U64, U64, U32, U32, I64, P]),
            "orc_mh_uniform": (D, [U64, U64, U64]),
            "orc_logp_grad": (D, [P, P, P]),
            "orc_map_O": (None, [P, P, I64, D, D]),
            "orc_map_B": (D, [P, P, I64, D]),
            "orc_map_O_lang": (None, [P, P, I64, D, D]),
            "orc_map_B_lang": (D, [P, P, I64, D]),
            "orc_map_A": (None, [P, P, P, I64, D]),
            "orc_integrator_coeffs": (I32, [I32, P, P, P]),
            "orc_create": (P, [P, P]),
            "orc_destroy": (None, [P]),
            "orc_init": (I32, [P, P, P]),
            "orc_unadj_move": (None, [P]),
            "orc_unadj_control": (None, [P]),
            "orc_step_unadjusted": (I32, [P, I64]),
            "orc_do_switch": (None, [P]),
            "orc_mams_move": (None, [P]),
            "orc_adj_control": (None, [P]),
            "orc_step_adjusted": (I32, [P, I64]),
            "orc_run": (I32, [P]),
            "orc_get_stats": (None, [P, P]),
            "orc_ptr": (P, [P, I32]),
            "orc_set_hyper": (None, [P, D, D]),
            "orc_F": (D, [D]),
            "orc_sum": (D, [P, I64]),
            "orc_rademacher": (None, [U64, U64, I64, I64, P]),
            "orc_dtilde_full": (D, [P, P, I64, I64, P, I64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------- RNG
def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def u01(w: int) -> float:
    return lib().orc_u01(int(w))


def normals(seed, chain, t, tag, substep, d) -> np.ndarray:
    z = np.zeros(d + 8)
    lib().orc_normals(seed, chain, t, tag, substep, d, _p(z))
    return z[:d].copy()


def mh_uniform(seed, chain, t) -> float:
    return lib().orc_mh_uniform(seed, chain, t)


def rademacher(seed, t, p, d) -> np.ndarray:
    """Probe p of step t: entries +-1 from the bits of Philox blocks (p, i // 256, t, 6)."""
    z = np.zeros(d)
    lib().orc_rademacher(seed, t, p, d, _p(z))
    return z


def dtilde_full(x, g, z) -> float:
    """Hutchinson estimate of the full-rank equipartition loss for positions x,
    gradients g ([N, d]) and probes z ([P, d])."""
    x, g, z = _f64(x), _f64(g), _f64(z)
    N, d = x.shape
    return lib().orc_dtilde_full(_p(x), _p(g), N, d, _p(z), z.shape[0])


# ----------------------------------------------------------------------------- targets
class Target:
    """Keeps the numpy buffers alive for the C struct that points at them."""

    def __init__(self, kind: int, d: int, a=None, b=None, n: int = 0, p0: float = 0.0, p1: float = 0.0):
        self.a = None if a is None else _f64(a).ravel()
        self.b = None if b is None else _f64(b).ravel()
        self.s = _Target(kind, d, None if self.a is None else self.a.ctypes.data,
                         None if self.b is None else self.b.ctypes.data, n, p0, p1)
        self.kind, self.d = kind, d

    @staticmethod
    def from_workload(w: dict) -> "Target":
        k = w["kind"]
        if k == "gauss":
            return Target(GAUSS_DIAG, w["d"], a=w["sigma2"])
        if k == "logreg":
            return Target(LOGREG, w["d"], a=w["X"], b=w["y"], n=w["X"].shape[0])
        if k == "stochvol":
            return Target(STOCHVOL, w["d"], a=w["y"], n=w["y"].shape[0])
        if k == "phi4":
            return Target(PHI4, w["d"], n=w["side"], p0=w["m2"], p1=w["lam"])
        if k == "gauss_dense":
            return Target(GAUSS_DENSE, w["d"], a=w["prec"])
        raise ValueError(k)

    def logp_grad(self, x) -> tuple[float, np.ndarray]:
        x = _f64(x)
        g = np.zeros(self.d)
        l = lib().orc_logp_grad(ctypes.byref(self.s), _p(x), _p(g))
        return l, g

    def logp(self, x) -> float:
        x = _f64(x)
        return lib().orc_logp_grad(ctypes.byref(self.s), _p(x), None)


# ----------------------------------------------------------------------------- maps
def map_O(u, xi, h, L) -> np.ndarray:
    u = _f64(u).copy()
    xi = _f64(xi)
    lib().orc_map_O(_p(u), _p(xi), u.size, h, L)
    return u


def map_B(u, gt, h) -> tuple[np.ndarray, float]:
    u = _f64(u).copy()
    gt = _f64(gt)
    dk = lib().orc_map_B(_p(u), _p(gt), u.size, h)
    return u, dk


def map_O_lang(u, xi, h, L) -> np.ndarray:
    u = _f64(u).copy()
    xi = _f64(xi)
    lib().orc_map_O_lang(_p(u), _p(xi), u.size, h, L)
    return u


def map_B_lang(u, gt, h) -> tuple[np.ndarray, float]:
    u = _f64(u).copy()
    gt = _f64(gt)
    dk = lib().orc_map_B_lang(_p(u), _p(gt), u.size, h)
    return u, dk


def map_A(x, u, h, sigma=None) -> np.ndarray:
    x = _f64(x).copy()
    u = _f64(u)
    s = None if sigma is None else _p(_f64(sigma))
    lib().orc_map_A(_p(x), _p(u), s, x.size, h)
    return x


def integrator_coeffs(which: int) -> tuple[np.ndarray, np.ndarray]:
    b = np.zeros(8)
    a = np.zeros(8)
    K = ctypes.c_int(0)
    rc = lib().orc_integrator_coeffs(which, _p(b), _p(a), ctypes.byref(K))
    if rc != 0:
        raise ValueError(which)
    return b[:K.value].copy(), a[:K.value - 1].copy()


def F(D: float) -> float:
    return lib().orc_F(D)


def fsum(v) -> float:
    v = _f64(v)
    return lib().orc_sum(_p(v), v.size)


# ----------------------------------------------------------------------------- ensemble
DEFAULTS = dict(C=0.025, alpha=2.0, eps0_factor=0.01, switch_tol=0.01, window_frac=0.2, acc_tol=0.03,
                acc_target=0.0, L_partial_factor=1.25, n_steps_traj=15, integrator_adj=0, eevpd_mode=1,
                switch_policy=0, max_steps_unadj=1000, max_steps_total=2000, full_rank_probes=0,
                eps_fixed=0.0, dynamics=0)

_ARR = dict(x=0, u=1, g=2, logp=3, delta=4, acc=5, mean=6, var=7, m2=8, Vii=9, sigma=10, ring=11, wdelta=12)


class Ensemble:
    def __init__(self, target: Target, n_chains: int, seed: int, **cfg):
        c = dict(DEFAULTS)
        c.update(cfg)
        self.cfg = c
        self.target = target
        self.N, self.d = n_chains, target.d
        self._c = _Config(n_chains, target.d, seed, c["C"], c["alpha"], c["eps0_factor"], c["switch_tol"],
                          c["window_frac"], c["acc_tol"], c["acc_target"], c["L_partial_factor"],
                          c["n_steps_traj"], c["integrator_adj"], c["eevpd_mode"], c["switch_policy"],
                          c["max_steps_unadj"], c["max_steps_total"], c["full_rank_probes"], c["eps_fixed"], c["dynamics"])
        self.h = lib().orc_create(ctypes.byref(self._c), ctypes.byref(target.s))
        if not self.h:
            raise ValueError("orc_create rejected the configuration")
        self.Tw = max(2, int(round(c["window_frac"] * c["max_steps_total"])))

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self.h = None

    def init(self, x0, u0=None):
        x0 = _f64(x0).reshape(self.N, self.d)
        u0p = None if u0 is None else _p(_f64(u0).reshape(self.N, self.d))
        lib().orc_init(self.h, _p(x0), u0p)

    def unadj_move(self):
        lib().orc_unadj_move(self.h)

    def unadj_control(self):
        lib().orc_unadj_control(self.h)

    def step_unadjusted(self, n: int) -> int:
        return lib().orc_step_unadjusted(self.h, n)

    def do_switch(self):
        lib().orc_do_switch(self.h)

    def mams_move(self):
        lib().orc_mams_move(self.h)

    def adj_control(self):
        lib().orc_adj_control(self.h)

    def step_adjusted(self, n: int) -> int:
        return lib().orc_step_adjusted(self.h, n)

    def run(self):
        lib().orc_run(self.h)

    def set_hyper(self, eps: float, L: float):
        lib().orc_set_hyper(self.h, eps, L)

    def stats(self) -> dict:
        s = _Stats()
        lib().orc_get_stats(self.h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def array(self, name: str) -> np.ndarray:
        n = {"x": self.N * self.d, "u": self.N * self.d, "g": self.N * self.d, "logp": self.N,
             "delta": self.N, "acc": self.N, "ring": self.Tw * self.d}.get(name, self.d)
        ptr = lib().orc_ptr(self.h, _ARR[name])
        buf = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctypes.c_double)), shape=(n,)).copy()
        if name in ("x", "u", "g"):
            return buf.reshape(self.N, self.d)
        if name == "ring":
            return buf.reshape(self.Tw, self.d)
        return buf

    def set_array(self, name: str, v):
        n = {"x": self.N * self.d, "u": self.N * self.d, "g": self.N * self.d, "logp": self.N,
             "delta": self.N, "acc": self.N, "ring": self.Tw * self.d}.get(name, self.d)
        ptr = lib().orc_ptr(self.h, _ARR[name])
        dst = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctypes.c_double)), shape=(n,))
        dst[:] = _f64(v).ravel()
