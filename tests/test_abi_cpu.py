"""C ABI checks that need no GPU: the library loads, exports every symbol its
header declares, and rejects bad configurations before touching a device."""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2212_11010_amd import kds
from paper_2212_11010_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "kds.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kds_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = kds.lib()
    names = _header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(kds.EXPORTED)


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors have the size and field offsets the C compiler gives
    the header's structs."""
    import subprocess
    src = tmp_path / "sz.c"
    fields = [n for n, _ in kds.kds_config._fields_]
    ifields = [n for n, _ in kds.kds_info_t._fields_]
    pfields = [n for n, _ in kds.kds_plan_t._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kds.h"', "int main(void) {",
             'printf("%zu %zu %zu\\n", sizeof(kds_config), sizeof(kds_info_t), sizeof(kds_plan_t));']
    lines += ['printf("%%zu\\n", offsetof(kds_config, %s));' % f for f in fields]
    lines += ['printf("%%zu\\n", offsetof(kds_info_t, %s));' % f for f in ifields]
    lines += ['printf("%%zu\\n", offsetof(kds_plan_t, %s));' % f for f in pfields]
    lines += ["return 0; }"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert int(out[0]) == C.sizeof(kds.kds_config)
    assert int(out[1]) == C.sizeof(kds.kds_info_t)
    assert int(out[2]) == C.sizeof(kds.kds_plan_t)
    offs = [int(v) for v in out[3:]]
    nf, ni = len(fields), len(ifields)
    assert offs[:nf] == [getattr(kds.kds_config, f).offset for f in fields]
    assert offs[nf:nf + ni] == [getattr(kds.kds_info_t, f).offset for f in ifields]
    assert offs[nf + ni:] == [getattr(kds.kds_plan_t, f).offset for f in pfields]


def _create_status(spec, **kw):
    cfg, keep = kds.make_config(spec, kw.pop("precision", "fp32"), kw.pop("schedule", "auto"))
    for k, v in kw.items():
        setattr(cfg, k, v)
    h = C.c_void_p()
    st = kds.lib().kds_create(C.byref(cfg), None, C.byref(h))
    return st, kds.kds_last_error(None)


@pytest.fixture
def spec():
    s, _ = wl.make_workload(2, n_cells=[8, 8], sub_cells=[4, 4])
    return s


@pytest.mark.parametrize("field,value,status", [
    ("dim", 0, kds.KDS_E_INVALID),
    ("dim", 4, kds.KDS_E_INVALID),
    ("degree", 4, kds.KDS_E_INVALID),
    ("degree", -1, kds.KDS_E_INVALID),
    ("m", 0, kds.KDS_E_INVALID),
    ("n_vel", 0, kds.KDS_E_INVALID),
    ("n_vel", 9, kds.KDS_E_INVALID),
    ("omega", 2.5, kds.KDS_E_INVALID),
    ("omega", -0.1, kds.KDS_E_INVALID),
    ("dt", 0.0, kds.KDS_E_INVALID),
    ("dt", float("nan"), kds.KDS_E_INVALID),
    ("theta", 0.3, kds.KDS_E_INVALID),
    ("n_iter", -1, kds.KDS_E_INVALID),
    ("n_iter", -5, kds.KDS_E_INVALID),
    ("law", 7, kds.KDS_E_INVALID),
    ("schedule", kds.KDS_SCHED_LINE + 10, kds.KDS_E_INVALID),
    ("precision", 9, kds.KDS_E_INVALID),
    ("schedule", 5, kds.KDS_E_INVALID),
])
def test_create_rejects_bad_scalar_fields(spec, field, value, status):
    st, msg = _create_status(spec, **{field: value})
    assert st == status, (st, msg)
    assert msg


def test_create_rejects_subdomains_not_dividing(spec):
    s = dict(spec, sub_cells=[3, 4, 1])
    st, msg = _create_status(s)
    assert st == kds.KDS_E_INVALID and "divide" in msg


def test_create_rejects_bad_periodic_flag(spec):
    s = dict(spec, periodic=[1, 2, 1])
    st, msg = _create_status(s)
    assert st == kds.KDS_E_INVALID and "periodic" in msg


def test_set_boundary_rejects_null_problem():
    assert kds.lib().kds_set_boundary(None, None, 0) == kds.KDS_E_INVALID


@pytest.mark.parametrize("sched", ["line", "plain"])
def test_create_rejects_oblique_velocity_outside_front_schedule(spec, sched):
    s = dict(spec, vel=[1.0, 1.0, -1.0, 0.0, 0.0, 1.0, 0.0, -1.0])
    st, msg = _create_status(s, schedule=sched)
    assert st == kds.KDS_E_UNSUPPORTED and "front" in msg


def test_create_rejects_split_precision_outside_front_schedule(spec):
    st, msg = _create_status(spec, precision="fp32_split_f16", schedule="line")
    assert st == kds.KDS_E_UNSUPPORTED


def test_create_rejects_zero_velocity(spec):
    s = dict(spec, vel=[1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, -1.0])
    st, msg = _create_status(s)
    assert st == kds.KDS_E_INVALID


def test_create_rejects_missing_law_params(spec):
    s = dict(spec, law_params=[0.0] * 5)
    st, msg = _create_status(s)
    assert st == kds.KDS_E_INVALID


def test_create_rejects_euler_with_wrong_m():
    s, _ = wl.make_workload(3, n_cells=[4, 4, 4], sub_cells=[2, 2, 2])
    st, msg = _create_status(dict(s, m=4))
    assert st == kds.KDS_E_INVALID


def test_create_rejects_velocity_set_without_equilibrium(spec):
    # all velocities along x: the moment conditions in y cannot be met
    s = dict(spec, vel=[1.0, 0.0, -1.0, 0.0, 2.0, 0.0, -2.0, 0.0])
    st, msg = _create_status(s)
    assert st == kds.KDS_E_INVALID and "moment" in msg


def test_null_arguments_are_rejected():
    L = kds.lib()
    assert L.kds_create(None, None, None) == kds.KDS_E_INVALID
    assert L.kds_step(None, 1) == kds.KDS_E_INVALID
    assert L.kds_set_state(None, None, 0) == kds.KDS_E_INVALID
    assert L.kds_moments(None, None, 0) == kds.KDS_E_INVALID
    assert L.kds_synchronize(None) == kds.KDS_E_INVALID
    assert L.kds_set_launch(None, 0, 0) == kds.KDS_E_INVALID
    assert L.kds_get_plan(None, None) == kds.KDS_E_INVALID
    assert L.kds_set_plan(None, None) == kds.KDS_E_INVALID
    assert L.kds_tune_cached(None, 1, b"plans.txt", None) == kds.KDS_E_INVALID
    assert L.kds_trace_residual(None, None) == kds.KDS_E_INVALID
    L.kds_destroy(None)


def test_binding_rejects_wrong_arrays():
    with pytest.raises(ValueError):
        kds._buf(np.zeros(4, dtype=np.float32), 16)
    with pytest.raises(ValueError):
        kds._buf(np.zeros(3), 32)


def test_batch_calls_reject_null_and_empty():
    L = kds.lib()
    out = C.c_void_p()
    assert L.kds_batch_create(None, 0, C.byref(out)) == kds.KDS_E_INVALID
    assert "at least one" in kds.kds_batch_last_error(None)
    assert L.kds_batch_create(None, 1, None) == kds.KDS_E_INVALID
    arr = (C.c_void_p * 2)(None, None)
    assert L.kds_batch_create(arr, 2, C.byref(out)) == kds.KDS_E_INVALID
    assert not out.value
    assert L.kds_batch_step(None, 1) == kds.KDS_E_INVALID
    assert L.kds_batch_tune(None, 3, None) == kds.KDS_E_INVALID
    assert L.kds_batch_synchronize(None) == kds.KDS_E_INVALID
    L.kds_batch_destroy(None)
