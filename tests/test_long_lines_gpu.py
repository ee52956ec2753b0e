"""Line schedule for grid lines longer than 64 lanes x the cells a lane holds
in registers (kds_info_t.line_qmax): the lanes own more cells and stream
them through the LDS tile in rounds (-m gpu).  Every case is checked against
the FP64 oracle (W and F, global and per plane), in FP64 and FP32, with the
automatic schedule (which must be the line schedule with rounds); one case
forces plans with and without rounds on the same problem."""
import functools

import numpy as np
import pytest

from tests import parity as pt

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}

# (workload, overrides): lines of 2 to 8 rounds along each axis
CASES = {
    # acoustics 2-D, p = 2 (9 nodes, 4 cells per lane in registers): x lines of 512
    "acoustics_p2_x512": (2, dict(n_cells=[512, 4], sub_cells=[64, 4], steps=2)),
    # ... along y, two subdomains per line
    "acoustics_p2_y512": (2, dict(n_cells=[4, 512], sub_cells=[4, 256], steps=2)),
    # p = 3 in 2-D (16 nodes): x lines of 512, and the converged limit (n_iter = 0)
    "acoustics_p3_x512": (2, dict(n_cells=[512, 2], sub_cells=[128, 2], steps=2, degree=3)),
    "acoustics_p2_x512_converged": (2, dict(n_cells=[512, 2], sub_cells=[64, 2], steps=2,
                                            n_iter=0)),
    # Dirichlet ends on x (boundary data change every step)
    "acoustics_p2_x512_dir": (2, dict(n_cells=[512, 2], sub_cells=[128, 2], steps=2,
                                      periodic=[0, 1, 1])),
    # Euler 3-D, p = 2 (27 nodes, 2 cells per lane in registers): x and z lines of 256
    "euler_p2_x256": (3, dict(n_cells=[256, 2, 2], sub_cells=[32, 2, 2], steps=2)),
    "euler_p2_z256": (3, dict(n_cells=[2, 2, 256], sub_cells=[2, 2, 64], steps=2)),
    # advection 1-D, p = 1 (8 cells per lane in registers): lines of 1024
    "advection_p1_1024": (1, dict(n_cells=[1024], sub_cells=[256], steps=3)),
}


@functools.lru_cache(maxsize=None)
def case(name):
    from oracle import oracle
    from paper_2212_11010_amd import workloads as wl
    cfg, ov = CASES[name]
    spec, W0 = wl.make_workload(cfg, **ov)
    B = None
    if not all(spec["periodic"][:spec["dim"]]):
        c = oracle.Config(spec)
        nb = oracle.n_boundary_nodes(c)
        rng = np.random.default_rng(7)
        B = [W0.reshape(-1, spec["m"])[:nb].copy() * (1.0 + 0.01 * rng.standard_normal((nb, 1)))
             for _ in range(spec["steps"] + 1)]
        F = oracle.init(c, W0)
        for s in range(spec["steps"]):
            F = oracle.step(c, F, 1, threads=0, Wb_old=B[s], Wb_new=B[s + 1])
        W = oracle.moments(c, F)
    else:
        F, W = oracle.run(spec, W0, spec["steps"], threads=0)
    return spec, W0, B, np.ascontiguousarray(F.transpose(0, 2, 3, 1)), W


def run_gpu(spec, W0, B, prec, plan=None):
    import torch
    from paper_2212_11010_amd import kds
    with kds.Problem(spec, precision=prec) as pb:
        if plan is not None:
            pb.set_plan(plan)
        info, got = pb.info(), pb.get_plan()
        pb.set_state(torch.from_numpy(W0).cuda())
        if B is not None:
            pb.set_boundary(B[0])
        for s in range(spec["steps"]):
            if B is not None:
                pb.set_boundary(B[s + 1])
            pb.step(1)
        return pb.moments(), pb.get_kinetic(), info, got


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", list(TOL))
def test_long_lines_parity(name, prec):
    from paper_2212_11010_amd import kds
    spec, W0, B, Fref, Wref = case(name)
    print("long-line case", name, prec, flush=True)
    W, F, info, plan = run_gpu(spec, W0, B, prec)
    assert info["schedule"] == kds.KDS_SCHED_LINE
    long_axes = [a for a in range(spec["dim"]) if plan["Q"][a] > info["line_qmax"]]
    assert long_axes, (plan, info["line_qmax"])
    print("  Q", plan["Q"], "line_qmax", info["line_qmax"], flush=True)
    pt.check(W, Wref, F, Fref, TOL[prec], label=name)


@pytest.mark.parametrize("prec", list(TOL))
def test_rounds_against_register_plans(prec):
    """128 x 4 cells, p = 2: x lines fit one wavefront with Q = 2 or 4 in
    registers (line_qmax 4) and also with Q = 8 or 16 in rounds; every plan
    matches the oracle."""
    import copy
    from paper_2212_11010_amd import workloads as wl
    from oracle import oracle
    spec, W0 = wl.make_workload(2, n_cells=[128, 4], sub_cells=[16, 4], steps=2)
    F, Wref = oracle.run(spec, W0, spec["steps"], threads=0)
    Fref = np.ascontiguousarray(F.transpose(0, 2, 3, 1))
    _, _, info, base = run_gpu(spec, W0, None, prec)
    for Q in (2, 4, 8, 16):
        plan = copy.deepcopy(base)
        plan["Q"][0] = Q
        plan["bw"][0] = 1
        plan["xdirect"] = 0
        W, Fg, _, got = run_gpu(spec, W0, None, prec, plan)
        assert got["Q"][0] == Q
        pt.check(W, Wref, Fg, Fref, TOL[prec], label="Q%d" % Q)
