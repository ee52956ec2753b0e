"""ctypes wrapper of the FP64 CPU oracle (oracle/kds_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py, never by the product path.  It shares no code with
the GPU library.  Problem descriptions are the plain dicts of
paper_2212_11010_amd/workloads.py.

Kinetic layout on this side: F[k, c, cell, node] (FP64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kds_oracle.cpp")
# KDS_ORACLE_LIB: another build of the same source (the sanitizer test's)
LIB = os.environ.get("KDS_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ -O2 (no fast-math), OpenMP for (k, c) tasks."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n_cells", C.c_int32 * 3), ("sub_cells", C.c_int32 * 3),
        ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("degree", C.c_int32), ("m", C.c_int32), ("law", C.c_int32),
        ("law_params", C.POINTER(C.c_double)), ("n_law_params", C.c_int32),
        ("n_vel", C.c_int32), ("vel", C.POINTER(C.c_double)),
        ("eq_a", C.POINTER(C.c_double)), ("eq_b", C.POINTER(C.c_double)),
        ("omega", C.c_double), ("dt", C.c_double), ("theta", C.c_double),
        ("n_iter", C.c_int32), ("source_sigma", C.POINTER(C.c_double)),
        ("periodic", C.POINTER(C.c_int32)), ("bnd_W_old", C.POINTER(C.c_double)),
        ("bnd_W_new", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        cp = C.POINTER(_Cfg)
        _lib.orc_gl.argtypes = [C.c_int, dp, dp]
        _lib.orc_deriv.argtypes = [C.c_int, dp]
        _lib.orc_flux.argtypes = [cp, dp, dp]
        _lib.orc_eq_weights.argtypes = [cp, dp, dp]
        _lib.orc_equilibrium.argtypes = [cp, dp, dp]
        _lib.orc_cell_residual.argtypes = [cp, dp, dp, dp, dp]
        _lib.orc_transport.argtypes = [cp, C.c_int, dp, dp, dp, dp]
        _lib.orc_transport_lines.argtypes = [cp, C.c_int, dp, dp, dp, C.c_int]
        _lib.orc_n_boundary_nodes.argtypes = [cp]
        _lib.orc_n_boundary_nodes.restype = C.c_long
        _lib.orc_init.argtypes = [cp, dp, dp]
        _lib.orc_moments.argtypes = [cp, dp, dp]
        _lib.orc_relax.argtypes = [cp, dp]
        _lib.orc_step.argtypes = [cp, dp, C.c_int, C.c_int]
        _lib.orc_max_threads.argtypes = []
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Config:
    """Holds a ctypes config plus the arrays it points to."""

    def __init__(self, spec: dict):
        self.spec = spec
        d = spec["dim"]
        self.dim = d
        self.P = spec["degree"] + 1
        self.nn = self.P ** d
        self.ncell = int(np.prod(spec["n_cells"][:d]))
        self.m = spec["m"]
        self.n_vel = spec["n_vel"]
        self._params = np.ascontiguousarray(spec["law_params"], dtype=np.float64)
        self._vel = np.ascontiguousarray(spec["vel"], dtype=np.float64)
        self._eqa = None if spec.get("eq_a") is None else np.ascontiguousarray(spec["eq_a"], dtype=np.float64)
        self._eqb = None if spec.get("eq_b") is None else np.ascontiguousarray(spec["eq_b"], dtype=np.float64)
        self._src = None if spec.get("source_sigma") is None else np.ascontiguousarray(
            spec["source_sigma"], dtype=np.float64)
        c = _Cfg()
        c.dim = d
        for a in range(3):
            c.n_cells[a] = int(spec["n_cells"][a])
            c.sub_cells[a] = int(spec["sub_cells"][a])
            c.box_lo[a] = float(spec["box_lo"][a])
            c.box_hi[a] = float(spec["box_hi"][a])
        c.degree = spec["degree"]
        c.m = spec["m"]
        c.law = spec["law"]
        c.law_params = _dp(self._params)
        c.n_law_params = len(self._params)
        c.n_vel = spec["n_vel"]
        c.vel = _dp(self._vel)
        c.eq_a = _dp(self._eqa) if self._eqa is not None else C.POINTER(C.c_double)()
        c.eq_b = _dp(self._eqb) if self._eqb is not None else C.POINTER(C.c_double)()
        c.omega = spec["omega"]
        c.dt = spec["dt"]
        c.theta = spec.get("theta", 0.5)
        c.n_iter = spec.get("n_iter", 3)
        c.source_sigma = _dp(self._src) if self._src is not None else C.POINTER(C.c_double)()
        self._per = np.ascontiguousarray(spec.get("periodic", [1, 1, 1]), dtype=np.int32)
        c.periodic = self._per.ctypes.data_as(C.POINTER(C.c_int32))
        c.bnd_W_old = C.POINTER(C.c_double)()
        c.bnd_W_new = C.POINTER(C.c_double)()
        self.c = c

    @property
    def ref(self):
        return C.byref(self.c)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed (%d)" % (what, rc))


def gl(p: int):
    xi = np.zeros(p + 1)
    w = np.zeros(p + 1)
    _check(lib().orc_gl(p, _dp(xi), _dp(w)), "gl")
    return xi, w


def deriv(p: int):
    D = np.zeros((p + 1, p + 1))
    _check(lib().orc_deriv(p, _dp(D)), "deriv")
    return D


def flux(cfg: Config, W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    Q = np.zeros((cfg.dim, cfg.m))
    _check(lib().orc_flux(cfg.ref, _dp(W), _dp(Q)), "flux")
    return Q


def eq_weights(cfg: Config):
    a = np.zeros(cfg.n_vel)
    b = np.zeros((cfg.n_vel, cfg.dim))
    _check(lib().orc_eq_weights(cfg.ref, _dp(a), _dp(b)), "eq_weights")
    return a, b


def equilibrium(cfg: Config, W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    M = np.zeros((cfg.n_vel, cfg.m))
    _check(lib().orc_equilibrium(cfg.ref, _dp(W), _dp(M)), "equilibrium")
    return M


def cell_residual(cfg: Config, V, f, tr):
    V = np.ascontiguousarray(V, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    tr = np.ascontiguousarray(tr, dtype=np.float64)
    r = np.zeros(cfg.nn)
    _check(lib().orc_cell_residual(cfg.ref, _dp(V), _dp(f), _dp(tr), _dp(r)), "cell_residual")
    return r


def _opt(a):
    if a is None:
        return None, C.POINTER(C.c_double)()
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, _dp(a)


def transport(cfg: Config, k: int, f_old, fb_old=None, fb_new=None):
    """One transport step of a scalar field f[cell, node] for velocity k;
    fb_old / fb_new: its values at the boundary nodes (Dirichlet axes)."""
    f_old = np.ascontiguousarray(f_old, dtype=np.float64)
    out = np.zeros_like(f_old)
    bo, po = _opt(fb_old)
    bn, pn = _opt(fb_new)
    _check(lib().orc_transport(cfg.ref, k, _dp(f_old), _dp(out), po, pn), "transport")
    return out


def transport_lines(cfg: Config, v, f_old, threads: int = 0):
    """Transport of many independent fields f[line, cell, node] of the 1-D
    periodic problem cfg (dim = 1), line l at velocity v[l]."""
    f_old = np.ascontiguousarray(f_old, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert cfg.dim == 1 and f_old.ndim == 3 and f_old.shape[0] == v.shape[0]
    out = np.zeros_like(f_old)
    _check(lib().orc_transport_lines(cfg.ref, int(v.shape[0]), _dp(v), _dp(f_old), _dp(out),
                                     int(threads)), "transport_lines")
    return out


def n_boundary_nodes(cfg: Config) -> int:
    return int(lib().orc_n_boundary_nodes(cfg.ref))


def init(cfg: Config, W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    F = np.zeros((cfg.n_vel, cfg.m, cfg.ncell, cfg.nn))
    _check(lib().orc_init(cfg.ref, _dp(W), _dp(F)), "init")
    return F


def moments(cfg: Config, F):
    F = np.ascontiguousarray(F, dtype=np.float64)
    W = np.zeros((cfg.ncell, cfg.nn, cfg.m))
    _check(lib().orc_moments(cfg.ref, _dp(F), _dp(W)), "moments")
    return W


def relax(cfg: Config, F):
    F = np.array(F, dtype=np.float64, order="C", copy=True)
    _check(lib().orc_relax(cfg.ref, _dp(F)), "relax")
    return F


def step(cfg: Config, F, n_steps: int = 1, threads: int = 0, Wb_old=None, Wb_new=None):
    """n_steps steps; Wb_old / Wb_new [boundary node, c]: boundary state at the
    start and the end of the first step (later steps hold Wb_new)."""
    F = np.array(F, dtype=np.float64, order="C", copy=True)
    bo, po = _opt(Wb_old)
    bn, pn = _opt(Wb_new)
    cfg.c.bnd_W_old, cfg.c.bnd_W_new = po, pn
    try:
        _check(lib().orc_step(cfg.ref, _dp(F), n_steps, threads), "step")
    finally:
        cfg.c.bnd_W_old = C.POINTER(C.c_double)()
        cfg.c.bnd_W_new = C.POINTER(C.c_double)()
    return F


def max_threads() -> int:
    return int(lib().orc_max_threads())


def run(spec: dict, W0, n_steps: int, threads: int = 0):
    """Initial equilibrium then n_steps steps; returns (F, W)."""
    cfg = Config(spec)
    F = init(cfg, W0)
    F = step(cfg, F, n_steps, threads)
    return F, moments(cfg, F)
