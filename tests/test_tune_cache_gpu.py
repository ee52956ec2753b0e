"""The plan cache (kds_tune_cached, -m gpu): a plan tuned once is taken from
the file by later problems of the same shape, which then reproduce the FP32
results of the first bit for bit; other shapes miss and are tuned."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _problem(spec, W0, prec="fp32"):
    import torch
    from paper_2212_11010_amd import kds
    pb = kds.Problem(spec, precision=prec)
    pb.set_state(torch.from_numpy(W0).cuda())
    return pb


def test_cached_plan_reproduces_bitwise(tmp_path):
    from paper_2212_11010_amd import workloads as wl
    path = str(tmp_path / "plans.txt")
    spec, W0 = wl.make_workload(2, n_cells=[64, 48], sub_cells=[16, 12], steps=4)
    with _problem(spec, W0) as pb:
        assert pb.tune_cached(path) is False            # empty cache: tuned and stored
        plan1 = pb.get_plan()
        pb.step(4)
        F1 = pb.get_kinetic()
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and "arch=gfx" in lines[0] and "N=64x48x1" in lines[0], lines
    with _problem(spec, W0) as pb:
        assert pb.tune_cached(path) is True             # same shape: from the file
        assert pb.get_plan() == plan1
        pb.step(4)
        assert np.array_equal(pb.get_kinetic(), F1)
    # another grid misses
    spec2, W2 = wl.make_workload(2, n_cells=[32, 48], sub_cells=[16, 12], steps=1)
    with _problem(spec2, W2) as pb:
        assert pb.tune_cached(path) is False
    assert len(open(path).read().splitlines()) == 2


def test_cached_front_kernel_choice(tmp_path):
    from paper_2212_11010_amd import workloads as wl
    path = str(tmp_path / "plans.txt")
    spec, W0 = wl.make_workload(6, n_cells=[16, 16, 16], sub_cells=[8, 8, 8], steps=2)
    with _problem(spec, W0) as pb:
        assert pb.tune_cached(path) is False
        plan = pb.get_plan()
        assert plan["front_kernel"] in (1, 2)
        pb.step(2)
        F1 = pb.get_kinetic()
    with _problem(spec, W0) as pb:
        assert pb.tune_cached(path) is True
        assert pb.get_plan() == plan
        pb.step(2)
        assert np.array_equal(pb.get_kinetic(), F1)


def test_subdomain_tuner_keeps_the_proposition_and_parity():
    """kds_tune_subdomains returns widths that divide the grid and satisfy
    the Proposition of Sec. 5.1 (|V| dt <= S h); the widths change the answer,
    so the problem built with them is checked against the oracle run with
    the same widths (FP64, 1e-12)."""
    import torch
    from oracle import oracle
    from paper_2212_11010_amd import kds, workloads as wl
    from tests import parity as pt
    spec, W0 = wl.make_workload(2, n_cells=[64, 32], sub_cells=[16, 16], steps=2)
    # the Proposition per axis: max_k |V_k^a| dt <= S_a h_a (cells are not
    # square here: h_y = 2 h_x, so the y widths may be half the x ones)
    d = spec["dim"]
    vel = np.asarray(spec["vel"], dtype=float).reshape(spec["n_vel"], d)
    nu = [np.abs(vel[:, a]).max() * spec["dt"] * spec["n_cells"][a] /
          (spec["box_hi"][a] - spec["box_lo"][a]) for a in range(d)]
    S, ms = kds.kds_tune_subdomains(spec, W0, precision="fp32", reps=2)
    print("  chosen sub_cells", S, "%.4f ms/step (nu per axis %s)" % (ms, nu), flush=True)
    assert ms > 0
    for a in range(d):
        assert spec["n_cells"][a] % S[a] == 0 and S[a] >= nu[a] * (1 - 1e-12), (S, nu)
    spec2 = dict(spec, sub_cells=list(S))
    F, Wref = oracle.run(spec2, W0, spec2["steps"], threads=0)
    Fref = np.ascontiguousarray(F.transpose(0, 2, 3, 1))
    with kds.Problem(spec2, precision="fp64") as pb:
        pb.set_state(torch.from_numpy(W0).cuda())
        pb.step(spec2["steps"])
        pt.check(pb.moments(), Wref, pb.get_kinetic(), Fref, 1e-12, label="tuned S")
    # Dirichlet problems need their boundary data: refused
    specd, Wd = wl.make_workload(2, n_cells=[32, 16], sub_cells=[8, 8], steps=1, periodic=[0, 1, 1])
    with pytest.raises(kds.KdsError) as e:
        kds.kds_tune_subdomains(specd, Wd)
    assert e.value.status == kds.KDS_E_UNSUPPORTED
