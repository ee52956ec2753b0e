"""Python binding of libkds (include/kds.h): argument marshalling only.

Every step of the kinetic DG time step runs in the HIP kernels of libkds.so;
this module converts problem descriptions and arrays into the C ABI calls of
the same names.  Host arrays are numpy FP64; device arrays are torch CUDA
(HIP) FP64 tensors, passed by pointer with on_device = 1.  The library is built
in-tree by paper_2212_11010_amd.build; importing the binding without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkds.so")

KDS_OK, KDS_E_INVALID, KDS_E_NOMEM, KDS_E_DEVICE, KDS_E_STATE, KDS_E_NONFINITE, KDS_E_UNSUPPORTED = range(7)
STATUS_NAMES = {0: "KDS_OK", 1: "KDS_E_INVALID", 2: "KDS_E_NOMEM", 3: "KDS_E_DEVICE",
                4: "KDS_E_STATE", 5: "KDS_E_NONFINITE", 6: "KDS_E_UNSUPPORTED"}
KDS_FP64, KDS_FP32, KDS_FP32_SPLIT_F16, KDS_FP32_SPLIT_BF16 = range(4)
KDS_SCHED_AUTO, KDS_SCHED_PLAIN, KDS_SCHED_LINE, KDS_SCHED_FRONT = range(4)
PRECISIONS = {"fp64": KDS_FP64, "fp32": KDS_FP32, "fp32_split_f16": KDS_FP32_SPLIT_F16,
              "fp32_split_bf16": KDS_FP32_SPLIT_BF16}
SCHEDULES = {"auto": KDS_SCHED_AUTO, "plain": KDS_SCHED_PLAIN, "line": KDS_SCHED_LINE,
             "front": KDS_SCHED_FRONT}
N_KERNEL_KINDS = 2
EXPORTED = ["kds_create", "kds_set_state", "kds_set_boundary", "kds_step", "kds_step_timed",
            "kds_tune", "kds_tune_cached", "kds_tune_subdomains", "kds_set_launch",
            "kds_get_plan", "kds_set_plan",
            "kds_time_kernels", "kds_moments", "kds_moments_static",
            "kds_get_kinetic", "kds_set_kinetic", "kds_check_finite", "kds_trace_residual",
            "kds_synchronize",
            "kds_info", "kds_destroy", "kds_last_error",
            "kds_batch_create", "kds_batch_step", "kds_batch_step_timed",
            "kds_batch_time_kernels", "kds_batch_tune", "kds_batch_synchronize",
            "kds_batch_destroy",
            "kds_batch_last_error"]
_NO_STATUS = ("kds_destroy", "kds_last_error", "kds_batch_destroy", "kds_batch_last_error")


class kds_config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n_cells", C.c_int32 * 3), ("sub_cells", C.c_int32 * 3),
        ("periodic", C.c_int32 * 3), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
        ("degree", C.c_int32), ("m", C.c_int32), ("law", C.c_int32),
        ("law_params", C.POINTER(C.c_double)), ("n_law_params", C.c_int32),
        ("n_vel", C.c_int32), ("vel", C.POINTER(C.c_double)),
        ("eq_a", C.POINTER(C.c_double)), ("eq_b", C.POINTER(C.c_double)),
        ("omega", C.c_double), ("dt", C.c_double), ("theta", C.c_double),
        ("n_iter", C.c_int32), ("precision", C.c_int32), ("schedule", C.c_int32),
        ("source_sigma", C.POINTER(C.c_double)),
    ]


class kds_info_t(C.Structure):
    _fields_ = [
        ("n_unknowns", C.c_int64), ("state_bytes", C.c_int64), ("schedule", C.c_int32),
        ("precision", C.c_int32), ("steps_done", C.c_int32),
        ("max_kinetic_courant", C.c_double), ("min_subdomain_width", C.c_double),
        ("proposition_ok", C.c_int32), ("line_Q", C.c_int32 * 3), ("line_bw", C.c_int32 * 3),
        ("tuned", C.c_int32), ("line_xdirect", C.c_int32), ("line_lds_bytes", C.c_int32),
        ("step_eager", C.c_int32), ("relax_vec", C.c_int32), ("line_qmax", C.c_int32),
        ("eq_monotone", C.c_int32), ("eq_min_eig", C.c_double), ("max_wave_speed", C.c_double),
        ("subchar_ok", C.c_int32),
    ]


class kds_plan_t(C.Structure):
    _fields_ = [
        ("Q", C.c_int32 * 3), ("bw", C.c_int32 * 3), ("xdirect", C.c_int32),
        ("lds_bytes", C.c_int32), ("step_eager", C.c_int32), ("relax_vec", C.c_int32),
        ("front_kernel", C.c_int32),
    ]


_lib = None


def lib():
    """Load libkds.so (torch first, so that one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libkds.so is not built: run paper_2212_11010_amd.build.build() "
                              "(or __graft_entry__.build()) first")
        try:
            import torch  # noqa: F401  (loads the HIP runtime torch uses)
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.kds_create.argtypes = [C.POINTER(kds_config), vp, C.POINTER(vp)]
        L.kds_set_state.argtypes = [vp, vp, C.c_int32]
        L.kds_set_boundary.argtypes = [vp, vp, C.c_int32]
        L.kds_step.argtypes = [vp, C.c_int32]
        L.kds_step_timed.argtypes = [vp, C.c_int32, dp]
        L.kds_tune.argtypes = [vp, C.c_int32, dp]
        L.kds_tune_cached.argtypes = [vp, C.c_int32, C.c_char_p, C.POINTER(C.c_int32)]
        L.kds_tune_subdomains.argtypes = [C.POINTER(kds_config), dp, C.c_int32, C.POINTER(C.c_int32), dp]
        L.kds_set_launch.argtypes = [vp, C.c_int32, C.c_int32]
        L.kds_get_plan.argtypes = [vp, C.POINTER(kds_plan_t)]
        L.kds_set_plan.argtypes = [vp, C.POINTER(kds_plan_t)]
        L.kds_time_kernels.argtypes = [vp, C.c_int32, dp]
        L.kds_moments.argtypes = [vp, vp, C.c_int32]
        L.kds_moments_static.argtypes = [vp, C.c_int64, C.c_int64, vp]
        L.kds_get_kinetic.argtypes = [vp, vp, C.c_int32]
        L.kds_set_kinetic.argtypes = [vp, vp, C.c_int32]
        L.kds_check_finite.argtypes = [vp]
        L.kds_trace_residual.argtypes = [vp, dp]
        L.kds_synchronize.argtypes = [vp]
        L.kds_info.argtypes = [vp, C.POINTER(kds_info_t)]
        L.kds_destroy.argtypes = [vp]
        L.kds_destroy.restype = None
        L.kds_last_error.argtypes = [vp]
        L.kds_last_error.restype = C.c_char_p
        L.kds_batch_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(vp)]
        L.kds_batch_step.argtypes = [vp, C.c_int32]
        L.kds_batch_step_timed.argtypes = [vp, C.c_int32, dp]
        L.kds_batch_time_kernels.argtypes = [vp, C.c_int32, dp]
        L.kds_batch_tune.argtypes = [vp, C.c_int32, dp]
        L.kds_batch_synchronize.argtypes = [vp]
        L.kds_batch_destroy.argtypes = [vp]
        L.kds_batch_destroy.restype = None
        L.kds_batch_last_error.argtypes = [vp]
        L.kds_batch_last_error.restype = C.c_char_p
        for name in EXPORTED:
            if name not in _NO_STATUS:
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class KdsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status
        self.message = message


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(spec: dict, precision="fp32", schedule="auto"):
    """kds_config from a problem description dict; returns (config, keepalive)."""
    d = spec["dim"]
    keep = {
        "law_params": np.ascontiguousarray(spec["law_params"], dtype=np.float64),
        "vel": np.ascontiguousarray(spec["vel"], dtype=np.float64),
        "eq_a": None if spec.get("eq_a") is None else np.ascontiguousarray(spec["eq_a"], dtype=np.float64),
        "eq_b": None if spec.get("eq_b") is None else np.ascontiguousarray(spec["eq_b"], dtype=np.float64),
        "source_sigma": None if spec.get("source_sigma") is None else np.ascontiguousarray(
            spec["source_sigma"], dtype=np.float64),
    }
    c = kds_config()
    c.dim = d
    for a in range(3):
        c.n_cells[a] = int(spec["n_cells"][a])
        c.sub_cells[a] = int(spec["sub_cells"][a])
        c.periodic[a] = int(spec.get("periodic", [1, 1, 1])[a])
        c.box_lo[a] = float(spec["box_lo"][a])
        c.box_hi[a] = float(spec["box_hi"][a])
    c.degree = int(spec["degree"])
    c.m = int(spec["m"])
    c.law = int(spec["law"])
    c.law_params = _dptr(keep["law_params"])
    c.n_law_params = len(keep["law_params"])
    c.n_vel = int(spec["n_vel"])
    c.vel = _dptr(keep["vel"])
    c.eq_a = _dptr(keep["eq_a"]) if keep["eq_a"] is not None else C.POINTER(C.c_double)()
    c.eq_b = _dptr(keep["eq_b"]) if keep["eq_b"] is not None else C.POINTER(C.c_double)()
    c.omega = float(spec["omega"])
    c.dt = float(spec["dt"])
    c.theta = float(spec.get("theta", 0.5))
    c.n_iter = int(spec.get("n_iter", 3))
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    c.source_sigma = (_dptr(keep["source_sigma"]) if keep["source_sigma"] is not None
                      else C.POINTER(C.c_double)())
    return c, keep


def _check(status, handle=None):
    if status != KDS_OK:
        msg = lib().kds_last_error(handle)
        raise KdsError(status, msg.decode() if msg else "")


def _buf(x, nbytes_expected):
    """(pointer, on_device) for a numpy array or a torch tensor."""
    if isinstance(x, np.ndarray):
        if x.dtype != np.float64 or not x.flags.c_contiguous:
            raise ValueError("host arrays must be C-contiguous float64")
        if x.nbytes != nbytes_expected:
            raise ValueError("array has %d bytes, expected %d" % (x.nbytes, nbytes_expected))
        return C.c_void_p(x.ctypes.data), 0
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected numpy.ndarray or torch.Tensor")
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise ValueError("tensors must be contiguous float64")
    if x.numel() * 8 != nbytes_expected:
        raise ValueError("tensor has %d bytes, expected %d" % (x.numel() * 8, nbytes_expected))
    if x.is_cuda:
        # the library works on its own stream: finish torch's pending work first
        torch.cuda.current_stream(x.device).synchronize()
        return C.c_void_p(x.data_ptr()), 1
    return C.c_void_p(x.data_ptr()), 0


# --------------------------------------------------------- C ABI, same names

def kds_create(spec, precision="fp32", schedule="auto", stream=None):
    cfg, keep = make_config(spec, precision, schedule)
    h = C.c_void_p()
    _check(lib().kds_create(C.byref(cfg), stream, C.byref(h)))
    return h


def kds_tune_subdomains(spec, W, precision="fp32", schedule="auto", reps=3):
    """kds_tune_subdomains: (sub_cells [3], ms per step) for the problem
    `spec` started from W (FP64 host [cell][node][c])."""
    cfg, keep = make_config(spec, precision, schedule)
    W = np.ascontiguousarray(W, dtype=np.float64)
    out = (C.c_int32 * 3)()
    ms = C.c_double(0.0)
    _check(lib().kds_tune_subdomains(C.byref(cfg), W.ctypes.data_as(C.POINTER(C.c_double)),
                                     int(reps), out, C.byref(ms)))
    return list(out), ms.value


def kds_set_state(h, W, nbytes):
    ptr, dev = _buf(W, nbytes)
    _check(lib().kds_set_state(h, ptr, dev), h)


def kds_set_boundary(h, Wb, nbytes):
    ptr, dev = _buf(Wb, nbytes)
    _check(lib().kds_set_boundary(h, ptr, dev), h)


def kds_step(h, n_steps=1):
    _check(lib().kds_step(h, int(n_steps)), h)


def kds_step_timed(h, n_steps=1):
    out = (C.c_double * N_KERNEL_KINDS)()
    _check(lib().kds_step_timed(h, int(n_steps), out), h)
    return list(out)


def kds_tune(h, reps=3):
    best = C.c_double(0.0)
    _check(lib().kds_tune(h, int(reps), C.byref(best)), h)
    return best.value


def kds_tune_cached(h, path, reps=3):
    """kds_tune through the plan cache file `path`; True if the plan came from it."""
    hit = C.c_int32(0)
    _check(lib().kds_tune_cached(h, int(reps), os.fsencode(path), C.byref(hit)), h)
    return bool(hit.value)


def kds_set_launch(h, step_eager, relax_vec):
    _check(lib().kds_set_launch(h, int(step_eager), int(relax_vec)), h)


def _struct_dict(st):
    out = {}
    for name, _ in st._fields_:
        v = getattr(st, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


def kds_get_plan(h):
    pl = kds_plan_t()
    _check(lib().kds_get_plan(h, C.byref(pl)), h)
    return _struct_dict(pl)


def kds_set_plan(h, plan):
    """plan: a dict with the fields of kds_plan_t (missing fields: 0)."""
    pl = kds_plan_t()
    for name, _ in kds_plan_t._fields_:
        v = plan.get(name, 0)
        if isinstance(v, (list, tuple)):
            for i, x in enumerate(v):
                getattr(pl, name)[i] = int(x)
        else:
            setattr(pl, name, int(v))
    _check(lib().kds_set_plan(h, C.byref(pl)), h)


def kds_time_kernels(h, reps=10):
    out = (C.c_double * N_KERNEL_KINDS)()
    _check(lib().kds_time_kernels(h, int(reps), out), h)
    return list(out)


def kds_moments(h, out, nbytes):
    ptr, dev = _buf(out, nbytes)
    _check(lib().kds_moments(h, ptr, dev), h)
    return out


def kds_moments_static(h, node_begin, node_count, out):
    """out: host float64 array of node_count * m values (C-contiguous)."""
    if not isinstance(out, np.ndarray) or out.dtype != np.float64 or not out.flags.c_contiguous:
        raise ValueError("kds_moments_static writes a C-contiguous float64 host array")
    _check(lib().kds_moments_static(h, int(node_begin), int(node_count),
                                    C.c_void_p(out.ctypes.data)), h)
    return out


def kds_get_kinetic(h, out, nbytes):
    ptr, dev = _buf(out, nbytes)
    _check(lib().kds_get_kinetic(h, ptr, dev), h)
    return out


def kds_set_kinetic(h, F, nbytes):
    ptr, dev = _buf(F, nbytes)
    _check(lib().kds_set_kinetic(h, ptr, dev), h)


def kds_check_finite(h):
    st = lib().kds_check_finite(h)
    if st == KDS_E_NONFINITE:
        return False
    _check(st, h)
    return True


def kds_trace_residual(h):
    out = (C.c_double * 2)()
    _check(lib().kds_trace_residual(h, out), h)
    return out[0], out[1]


def kds_synchronize(h):
    _check(lib().kds_synchronize(h), h)


def kds_info(h):
    info = kds_info_t()
    _check(lib().kds_info(h, C.byref(info)), h)
    return _struct_dict(info)


def kds_destroy(h):
    lib().kds_destroy(h)


def kds_last_error(h=None):
    msg = lib().kds_last_error(h)
    return msg.decode() if msg else ""


def _bcheck(status, handle=None):
    if status != KDS_OK:
        msg = lib().kds_batch_last_error(handle)
        raise KdsError(status, msg.decode() if msg else "")


def kds_batch_create(handles):
    arr = (C.c_void_p * len(handles))(*[h.value for h in handles])
    b = C.c_void_p()
    _bcheck(lib().kds_batch_create(arr, len(handles), C.byref(b)))
    return b


def kds_batch_step(b, n_steps=1):
    _bcheck(lib().kds_batch_step(b, int(n_steps)), b)


def kds_batch_step_timed(b, n_steps=1):
    ms = C.c_double(0.0)
    _bcheck(lib().kds_batch_step_timed(b, int(n_steps), C.byref(ms)), b)
    return ms.value


def kds_batch_time_kernels(b, reps=10):
    out = (C.c_double * N_KERNEL_KINDS)()
    _bcheck(lib().kds_batch_time_kernels(b, int(reps), out), b)
    return list(out)


def kds_batch_tune(b, reps=3):
    ms = C.c_double(0.0)
    _bcheck(lib().kds_batch_tune(b, int(reps), C.byref(ms)), b)
    return ms.value


def kds_batch_synchronize(b):
    _bcheck(lib().kds_batch_synchronize(b), b)


def kds_batch_destroy(b):
    lib().kds_batch_destroy(b)


def kds_batch_last_error(b=None):
    msg = lib().kds_batch_last_error(b)
    return msg.decode() if msg else ""


# ------------------------------------------------------------ convenience

class Problem:
    """Owns one kds_problem.  stream: a HIP stream handle (int) or None; with
    torch available the current torch stream is used by default."""

    def __init__(self, spec, precision="fp32", schedule="auto", stream="torch"):
        self.spec = spec
        d = spec["dim"]
        self.ncell = int(np.prod(spec["n_cells"][:d]))
        self.nn = (spec["degree"] + 1) ** d
        self.m = spec["m"]
        self.n_vel = spec["n_vel"]
        per = list(spec.get("periodic", [1, 1, 1]))
        P = spec["degree"] + 1
        self.n_boundary = sum(2 * (self.ncell // spec["n_cells"][a]) * (self.nn // P)
                              for a in range(d) if not per[a])
        if stream == "torch":
            stream = None
            try:
                import torch
                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream().cuda_stream
            except ImportError:
                pass
        self.stream = stream
        self.h = kds_create(spec, precision, schedule, C.c_void_p(stream) if stream else None)

    @property
    def w_shape(self):
        return (self.ncell, self.nn, self.m)

    @property
    def f_shape(self):
        return (self.n_vel, self.ncell, self.nn, self.m)

    def set_state(self, W):
        kds_set_state(self.h, W, self.ncell * self.nn * self.m * 8)

    def set_boundary(self, Wb):
        """Dirichlet data W_b [boundary node, m] for the end of the next step."""
        kds_set_boundary(self.h, Wb, self.n_boundary * self.m * 8)

    def step(self, n=1):
        kds_step(self.h, n)

    def step_timed(self, n=1):
        return kds_step_timed(self.h, n)

    def tune(self, reps=3):
        return kds_tune(self.h, reps)

    def tune_cached(self, path, reps=3):
        return kds_tune_cached(self.h, path, reps)

    def time_kernels(self, reps=10):
        return kds_time_kernels(self.h, reps)

    def set_launch(self, step_eager, relax_vec):
        kds_set_launch(self.h, step_eager, relax_vec)

    def get_plan(self):
        return kds_get_plan(self.h)

    def set_plan(self, plan):
        kds_set_plan(self.h, plan)

    def moments(self, out=None):
        if out is None:
            out = np.empty(self.w_shape)
        return kds_moments(self.h, out, self.ncell * self.nn * self.m * 8)

    def get_kinetic(self, out=None):
        if out is None:
            out = np.empty(self.f_shape)
        return kds_get_kinetic(self.h, out, self.n_vel * self.ncell * self.nn * self.m * 8)

    def set_kinetic(self, F):
        kds_set_kinetic(self.h, F, self.n_vel * self.ncell * self.nn * self.m * 8)

    def check_finite(self):
        return kds_check_finite(self.h)

    def trace_residual(self):
        """(max |tr^(K) - tr^(K-1)|, max |tr^(K)|) of the step that would
        start from the current state."""
        return kds_trace_residual(self.h)

    def synchronize(self):
        kds_synchronize(self.h)

    def info(self):
        return kds_info(self.h)

    def close(self):
        if self.h is not None:
            kds_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Owns one kds_batch over Problem objects (kept alive by the batch)."""

    def __init__(self, problems):
        self.problems = list(problems)
        self.h = kds_batch_create([p.h for p in self.problems])

    def step(self, n=1):
        kds_batch_step(self.h, n)

    def step_timed(self, n=1):
        return kds_batch_step_timed(self.h, n)

    def time_kernels(self, reps=10):
        return kds_batch_time_kernels(self.h, reps)

    def tune(self, reps=3):
        return kds_batch_tune(self.h, reps)

    def synchronize(self):
        kds_batch_synchronize(self.h)

    def close(self):
        if self.h is not None:
            kds_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
