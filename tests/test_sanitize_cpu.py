"""AddressSanitizer / UndefinedBehaviorSanitizer runs of the host code
(CPU only): the FP64 CPU oracle, built with -fsanitize=address,undefined and
run through one step of every workload family (linear and Euler laws, 1-D to
3-D, axis-aligned and D3Q4 velocities, Dirichlet boundaries, the source
term), and the library's FP64 setup routines (tests/sanitize_setup_driver.cpp).
A sanitizer report makes the run fail (halt_on_error)."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _gcc_runtime(name):
    path = subprocess.run(["g++", "-print-file-name=" + name], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def tmp():
    d = tempfile.mkdtemp(prefix="kds_san_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _report(res):
    return "runtime error" in res.stderr or "AddressSanitizer" in res.stderr


def test_setup_routines_under_sanitizers(tmp):
    if not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("HIP headers not installed")
    exe = os.path.join(tmp, "setup_driver")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
                           "-I" + os.path.join(ROOT, "paper_2212_11010_amd", "csrc"),
                           os.path.join(ROOT, "paper_2212_11010_amd", "csrc", "kds_setup.cpp"),
                           os.path.join(ROOT, "tests", "sanitize_setup_driver.cpp"), "-o", exe])
    res = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    print(res.stdout[-2000:], res.stderr[-4000:])
    assert res.returncode == 0 and not _report(res)


ORACLE_RUN = r"""
import sys
sys.path.insert(0, %r)
import numpy as np
from oracle import oracle
from paper_2212_11010_amd import workloads as wl
cases = [
    (1, dict(n_cells=[12], sub_cells=[4], steps=2)),
    (2, dict(n_cells=[6, 4], sub_cells=[3, 2], steps=2)),
    (2, dict(n_cells=[6, 4], sub_cells=[3, 4], steps=2, source_sigma=[0.5, 0.0, 0.0])),
    (3, dict(n_cells=[4, 3, 2], sub_cells=[2, 3, 1], steps=1)),
    (4, dict(n_cells=[3, 2, 2], sub_cells=[3, 1, 2], steps=1)),
    (6, dict(n_cells=[4, 2, 2], sub_cells=[2, 2, 1], steps=1, degree=1)),
    (2, dict(n_cells=[6, 4], sub_cells=[3, 2], steps=1, periodic=[0, 1, 1])),
]
for cfg, ov in cases:
    spec, W0 = wl.make_workload(cfg, **ov)
    c = oracle.Config(spec)
    B = None
    if not all(spec["periodic"][:spec["dim"]]):
        nb = oracle.n_boundary_nodes(c)
        B = [np.full((nb, spec["m"]), 0.1 * (s + 1)) for s in range(2)]
    F = oracle.init(c, W0)
    if B is None:
        F = oracle.step(c, F, spec["steps"], threads=2)
    else:
        F = oracle.step(c, F, 1, threads=2, Wb_old=B[0], Wb_new=B[1])
    W = oracle.moments(c, F)
    assert np.isfinite(F).all() and np.isfinite(W).all()
    print("case", cfg, "ok", flush=True)
print("all ok")
"""


def test_oracle_under_sanitizers(tmp):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("no sanitizer runtime for g++")
    lib = os.path.join(tmp, "liboracle_san.so")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-fPIC", "-shared", "-fopenmp",
                           "-o", lib, os.path.join(ROOT, "oracle", "kds_oracle.cpp")])
    # the interpreter is not instrumented: the runtime comes first by preload,
    # and leaks of the interpreter itself are not counted
    env = dict(ENV, KDS_ORACLE_LIB=lib, LD_PRELOAD=asan + ":" + ubsan,
               ASAN_OPTIONS="halt_on_error=1:detect_leaks=0")
    res = subprocess.run([sys.executable, "-c", ORACLE_RUN % ROOT], capture_output=True,
                         text=True, env=env, timeout=600)
    print(res.stdout[-2000:], res.stderr[-4000:])
    assert res.returncode == 0 and "all ok" in res.stdout and not _report(res)
