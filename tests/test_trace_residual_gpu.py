"""kds_trace_residual (-m gpu): the change of the subdomain outflow traces
between the last two Jacobi iterates of Sec. 5.1 (eq:ibvp), for the step
that would start from the current state.  The expected values come from the
FP64 oracle: its transport run with n_iter = K and with n_iter = K - 1 (or,
for K = 1, the state itself: iterate 0), read at every node on the
subdomains' outflow faces (for each axis along which the velocity has a
component, the downwind face of the subdomain's last cell on that axis):
axis-aligned sets (plain, line and front schedules) and the D3Q4 set of
the paper (front schedule)."""
import numpy as np
import pytest

from tests.parity import outflow_nodes

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}

# (workload, overrides, steps taken before the residual is read)
CASES = {
    "acoustics2d_K3": (2, dict(n_cells=[16, 8], sub_cells=[4, 4], n_iter=3), 1),
    "acoustics2d_K1": (2, dict(n_cells=[16, 8], sub_cells=[4, 2], n_iter=1), 0),
    "advection2d_K4": (1, dict(n_cells=[32, 16], sub_cells=[8, 4], n_iter=4), 2),
    "euler3d_K2": (3, dict(n_cells=[6, 4, 4], sub_cells=[3, 2, 2], n_iter=2), 1),
}
# D3Q4 Maxwell (oblique velocities: front schedule only)
OBLIQUE = {
    "maxwell_q2_K3": (6, dict(n_cells=[8, 8, 4], sub_cells=[4, 4, 2], n_iter=3), 1),
    "maxwell_q1_K1": (6, dict(n_cells=[6, 4, 4], sub_cells=[3, 2, 4], n_iter=1, degree=1), 0),
}


def oracle_residual(wcfg, ov, steps):
    from oracle import oracle
    from paper_2212_11010_amd import workloads as wl
    spec, W0 = wl.make_workload(wcfg, steps=max(steps, 1), **ov)
    K = spec["n_iter"]
    c = oracle.Config(spec)
    F = oracle.init(c, W0)
    if steps:
        F = oracle.step(c, F, steps, threads=0)
    cK = oracle.Config(spec)
    cP = oracle.Config(dict(spec, n_iter=K - 1)) if K > 1 else None
    dmax, vmax = 0.0, 0.0
    for k in range(c.n_vel):
        for comp in range(c.m):
            TK = oracle.transport(cK, k, F[k, comp])
            TP = oracle.transport(cP, k, F[k, comp]) if cP is not None else F[k, comp]
            a, b = outflow_nodes(c, k, TK), outflow_nodes(c, k, TP)
            dmax = max(dmax, float(np.max(np.abs(a - b))))
            vmax = max(vmax, float(np.max(np.abs(a))))
    return spec, W0, dmax, vmax


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,sched", [("fp64", "auto"), ("fp64", "plain"), ("fp32", "auto"),
                                        ("fp32", "front")])
def test_trace_residual_against_oracle(name, prec, sched):
    import torch
    from paper_2212_11010_amd import kds
    wcfg, ov, steps = CASES[name]
    spec, W0, dref, vref = oracle_residual(wcfg, ov, steps)
    print("trace residual", name, prec, sched, flush=True)
    with kds.Problem(spec, precision=prec, schedule=sched) as pb:
        pb.set_state(torch.from_numpy(W0).cuda())
        if steps:
            pb.step(steps)
        d, v = pb.trace_residual()
        # reading the residual leaves the state as it was
        W1 = pb.moments()
        pb.step(1)
        pb.set_state(torch.from_numpy(W0).cuda())
        if steps:
            pb.step(steps)
        W2 = pb.moments()
    print("  residual %.6e (oracle %.6e), max trace %.6e (oracle %.6e)" % (d, dref, v, vref),
          flush=True)
    assert dref > 0.0
    assert abs(v - vref) <= TOL[prec] * vref
    assert abs(d - dref) <= TOL[prec] * vref
    assert np.array_equal(W1, W2)


@pytest.mark.parametrize("name", list(OBLIQUE))
@pytest.mark.parametrize("prec,kernel", [("fp64", 2), ("fp64", 1), ("fp32", 2),
                                         ("fp32_split_f16", 2)])
def test_trace_residual_oblique_against_oracle(name, prec, kernel):
    import torch
    from paper_2212_11010_amd import kds
    wcfg, ov, steps = OBLIQUE[name]
    spec, W0, dref, vref = oracle_residual(wcfg, ov, steps)
    print("trace residual", name, prec, "front kernel", kernel, flush=True)
    tol = {"fp64": 1e-12, "fp32": 2e-5, "fp32_split_f16": 2e-5}[prec]
    with kds.Problem(spec, precision=prec, schedule="front") as pb:
        plan = pb.get_plan()
        plan["front_kernel"] = kernel
        pb.set_plan(plan)
        pb.set_state(torch.from_numpy(W0).cuda())
        if steps:
            pb.step(steps)
        W1 = pb.moments()
        d, v = pb.trace_residual()
        assert np.array_equal(W1, pb.moments())
    print("  residual %.6e (oracle %.6e), max trace %.6e (oracle %.6e)" % (d, dref, v, vref),
          flush=True)
    assert dref > 0.0
    assert abs(v - vref) <= tol * vref
    assert abs(d - dref) <= tol * vref


def test_trace_residual_converged_and_no_state():
    import torch
    from paper_2212_11010_amd import kds, workloads as wl
    spec, W0 = wl.make_workload(2, n_cells=[16, 8], sub_cells=[4, 4], n_iter=0, steps=1)
    with kds.Problem(spec, precision="fp64") as pb:
        with pytest.raises(kds.KdsError) as ei:
            pb.trace_residual()
        assert ei.value.status == kds.KDS_E_STATE
        pb.set_state(torch.from_numpy(W0).cuda())
        assert pb.trace_residual() == (0.0, -1.0)
