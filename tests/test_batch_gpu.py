"""Batched launches (kds_batch_*): many uneven problems advanced together.

A batch step runs the same arithmetic as kds_step on every member, only
grouped into fewer launches, so every member's state after batched steps must
equal, bit for bit, the state of an identical problem stepped on its own; the
small members are also checked against the FP64 oracle to the usual
tolerances (1e-12 FP64 storage, 1e-5 FP32 storage).
"""
from __future__ import annotations

import functools

import numpy as np
import pytest

from tests import parity as pt

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def small_batch(seed=7, n=10):
    from paper_2212_11010_amd import workloads as wl
    return wl.make_batch_workload(n_problems=n, max_unknowns=4e6, acoustics_n=(16, 24, 32),
                                  euler_n=(8, 12), seed=seed, steps=3)


@functools.lru_cache(maxsize=None)
def member_oracle(seed, i):
    from oracle import oracle
    from paper_2212_11010_amd import workloads as wl
    spec = small_batch(seed)[i]
    W0 = wl.batch_member_state(spec)
    F, W = oracle.run(spec, W0, spec["steps"], threads=0)
    return np.ascontiguousarray(F.transpose(0, 2, 3, 1)), W


relerr = pt.relerr


def make_members(specs, prec, scheds):
    import torch
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    out = []
    for spec, sched in zip(specs, scheds):
        pb = kds.Problem(spec, precision=prec, schedule=sched)
        pb.set_state(torch.from_numpy(wl.batch_member_state(spec)).cuda())
        out.append(pb)
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_equals_single_problems_and_oracle(prec):
    from paper_2212_11010_amd import kds
    specs = small_batch()
    # mostly automatic (line) members, two plain ones for the mixed path
    scheds = ["auto"] * len(specs)
    scheds[1] = "plain"
    scheds[4] = "plain"
    steps = specs[0]["steps"]
    print("batch of", len(specs), prec, [s["name"] for s in specs], flush=True)
    members = make_members(specs, prec, scheds)
    singles = make_members(specs, prec, scheds)
    with kds.Batch(members) as b:
        b.step(steps)
        b.synchronize()
    for pb in singles:
        pb.step(steps)
    for i, (pm, ps) in enumerate(zip(members, singles)):
        Fm, Fs = pm.get_kinetic(), ps.get_kinetic()
        assert pm.info()["steps_done"] == steps
        assert np.array_equal(Fm, Fs), (i, specs[i]["name"], relerr(Fm, Fs))
        Fref, Wref = member_oracle(7, i)
        pt.check(pm.moments(), Wref, Fm, Fref, TOL[prec], label="%s %s" % (specs[i]["name"], scheds[i]))
    for pb in members + singles:
        pb.close()


def test_batch_with_front_member_and_retune():
    """A front-schedule member (D3Q4 Maxwell) in the batch, and a member
    re-tuned after the batch was made (the batch rebuilds its task tables)."""
    import torch
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    specs = small_batch(seed=11, n=5)
    mspec, mW0 = wl.make_workload(6, n_cells=[8, 8, 8], sub_cells=[4, 4, 4], steps=3)
    members = make_members(specs, "fp32", ["auto"] * len(specs))
    singles = make_members(specs, "fp32", ["auto"] * len(specs))
    fm = kds.Problem(mspec, precision="fp32", schedule="front")
    fs = kds.Problem(mspec, precision="fp32", schedule="front")
    for pb in (fm, fs):
        pb.set_state(torch.from_numpy(mW0).cuda())
    with kds.Batch(members + [fm]) as b:
        b.step(1)
        for pb in singles + [fs]:
            pb.step(1)
        members[0].tune(reps=2)
        # the tuned plan, given to the single problem too: bitwise equal results
        singles[0].set_plan(members[0].get_plan())
        b.step(2)
        ms = b.step_timed(1)
        assert ms > 0
        kms = b.time_kernels(reps=2)
        assert kms[0] > 0 and kms[1] > 0
        b.synchronize()
    for pb in singles + [fs]:
        pb.step(3)
    for i, (pm, ps) in enumerate(zip(members + [fm], singles + [fs])):
        assert pm.info()["steps_done"] == 4
        Fm, Fs = pm.get_kinetic(), ps.get_kinetic()
        assert np.array_equal(Fm, Fs), (i, relerr(Fm, Fs))
    for pb in members + singles + [fm, fs]:
        pb.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_front_members_grouped(prec):
    """Front-schedule members on the wave kernel share one launch per
    subdomain iteration and one relaxation launch (two D3Q4 members of
    different sizes, one with Dirichlet faces and data changing between the
    steps), in FP32 and in FP64 (FP64 matrix cores); a member forced to the
    workgroup kernel keeps its own sequence.  All end bitwise equal to the
    same problems stepped on their own."""
    import torch
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    cases = [dict(n_cells=[8, 8, 8], sub_cells=[4, 4, 4], steps=3),
             dict(n_cells=[12, 8, 4], sub_cells=[4, 4, 4], steps=3),
             dict(n_cells=[8, 8, 8], sub_cells=[4, 4, 4], steps=3, periodic=[0, 1, 1]),
             dict(n_cells=[8, 4, 4], sub_cells=[4, 4, 4], steps=3)]
    kernels = [2, 2, 2, 1]        # wave, wave, wave (Dirichlet), workgroup
    specs = [wl.make_workload(6, **c) for c in cases]
    bm, bs = [], []
    for (spec, W0), kern in zip(specs, kernels):
        for lst in (bm, bs):
            pb = kds.Problem(spec, precision=prec, schedule="front")
            pb.set_state(torch.from_numpy(W0).cuda())
            plan = pb.get_plan()
            plan["front_kernel"] = kern
            pb.set_plan(plan)
            assert pb.get_plan()["front_kernel"] == kern
            lst.append(pb)
    dspec = specs[2][0]
    data = [wl.boundary_state(dspec, t=0.1 * s) for s in range(4)]
    for lst in (bm, bs):
        lst[2].set_boundary(data[0])
    with kds.Batch(bm) as b:
        for s in range(3):
            bm[2].set_boundary(data[s + 1])
            b.step(1)
        kms = b.time_kernels(reps=2)
        assert kms[0] > 0 and kms[1] > 0
        b.synchronize()
    for s in range(3):
        bs[2].set_boundary(data[s + 1])
        for pb in bs:
            pb.step(1)
    for i, (pm, ps) in enumerate(zip(bm, bs)):
        assert pm.info()["steps_done"] == 3
        Fm, Fs = pm.get_kinetic(), ps.get_kinetic()
        assert np.array_equal(Fm, Fs), (i, relerr(Fm, Fs))
    for pb in bm + bs:
        pb.close()


def test_batch_tune_keeps_results_and_state():
    """kds_batch_tune times widened bundles for the line members; the states,
    boundary data and step counts are restored, and the batch with the kept
    choice still gives the single-problem results bitwise (a Dirichlet
    member included)."""
    import torch
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    specs = small_batch(seed=17, n=6)
    members = make_members(specs, "fp32", ["auto"] * len(specs))
    singles = make_members(specs, "fp32", ["auto"] * len(specs))
    dspec, dW0 = wl.make_workload(2, n_cells=[24, 16], sub_cells=[8, 8], periodic=[0, 1], steps=2)
    Wb = wl.boundary_state(dspec, dW0)
    dm, ds = [], []
    for lst in (dm, ds):
        pb = kds.Problem(dspec, precision="fp32")
        pb.set_state(torch.from_numpy(dW0).cuda())
        pb.set_boundary(0.99 * Wb)
        pb.set_boundary(Wb)
        lst.append(pb)
    before = [pb.get_kinetic() for pb in members + dm]
    with kds.Batch(members + dm) as b:
        ms = b.tune(reps=2)
        assert ms > 0
        for pb, F in zip(members + dm, before):
            assert pb.info()["steps_done"] == 0
            assert np.array_equal(pb.get_kinetic(), F)
        b.step(2)
        b.synchronize()
    for pb in singles + ds:
        pb.step(2)
    for i, (pm, ps) in enumerate(zip(members + dm, singles + ds)):
        Fm, Fs = pm.get_kinetic(), ps.get_kinetic()
        assert np.array_equal(Fm, Fs), (i, relerr(Fm, Fs))
    for pb in members + singles + dm + ds:
        pb.close()


def test_batch_member_without_state_rejected():
    import torch
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    specs = small_batch(n=2)
    a = kds.Problem(specs[0], precision="fp32")
    c = kds.Problem(specs[1], precision="fp32")
    a.set_state(torch.from_numpy(wl.batch_member_state(specs[0])).cuda())
    with kds.Batch([a, c]) as b:
        with pytest.raises(kds.KdsError) as e:
            b.step(1)
        assert e.value.status == kds.KDS_E_STATE
    a.close()
    c.close()


def test_batch_with_dirichlet_member():
    """Members with Dirichlet axes (2-D along x and along y, 3-D along z) join
    the grouped line launch of their kind; with boundary data that change
    between the batched steps, and over two batched steps in one call, they
    end bitwise equal to the same problems stepped on their own with the same
    data."""
    import torch
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    specs = small_batch(seed=13, n=3)
    dspecs = [wl.make_workload(2, n_cells=[24, 16], sub_cells=[8, 8], periodic=[0, 1], steps=3),
              wl.make_workload(2, n_cells=[16, 32], sub_cells=[8, 16], periodic=[1, 0], steps=3),
              wl.make_workload(3, n_cells=[8, 6, 4], sub_cells=[4, 6, 4], periodic=[1, 1, 0],
                               steps=3)]
    rng = np.random.default_rng(3)
    data = []
    for dspec, dW0 in dspecs:
        Wb = wl.boundary_state(dspec, dW0)
        data.append([Wb * (1.0 + 0.01 * rng.standard_normal((Wb.shape[0], 1))) for _ in range(4)])
    members = make_members(specs, "fp32", ["auto"] * len(specs))
    singles = make_members(specs, "fp32", ["auto"] * len(specs))
    dm, ds = [], []
    for (dspec, dW0), B in zip(dspecs, data):
        for lst in (dm, ds):
            pb = kds.Problem(dspec, precision="fp32")
            pb.set_state(torch.from_numpy(dW0).cuda())
            pb.set_boundary(B[0])
            assert pb.info()["schedule"] == kds.KDS_SCHED_LINE
            lst.append(pb)
    with kds.Batch(members + dm) as b:
        for s in range(3):
            for pb, B in zip(dm, data):
                pb.set_boundary(B[s + 1])
            b.step(1)
        # two batched steps in one call: the second starts from the data at
        # the end of the first
        for pb, B in zip(dm, data):
            pb.set_boundary(B[0])
            pb.set_boundary(B[2])
        b.step(2)
        b.synchronize()
    for pb in singles:
        pb.step(5)
    for s in range(3):
        for pb, B in zip(ds, data):
            pb.set_boundary(B[s + 1])
            pb.step(1)
    for pb, B in zip(ds, data):
        pb.set_boundary(B[0])
        pb.set_boundary(B[2])
        pb.step(2)
    for pm, ps in zip(members + dm, singles + ds):
        assert pm.info()["steps_done"] == 5
        assert np.array_equal(pm.get_kinetic(), ps.get_kinetic())
    for pb in members + singles + dm + ds:
        pb.close()


def test_batch_with_degree3_members():
    """Degree-3 3-D members (64-node cells: node-line groups streamed through
    LDS) share the batched line launch of their (precision, degree,
    dimension); they end bitwise equal to the same problems stepped on their
    own, and the first matches the FP64 oracle."""
    import torch
    from oracle import oracle
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    cases = [wl.make_workload(4, n_cells=[8, 6, 4], sub_cells=[4, 3, 2], steps=2, seed=41),
             wl.make_workload(4, n_cells=[12, 8, 6], sub_cells=[6, 4, 3], steps=2, seed=42)]
    members, singles = [], []
    for spec, W0 in cases:
        for lst in (members, singles):
            pb = kds.Problem(spec, precision="fp32")
            pb.set_state(torch.from_numpy(W0).cuda())
            lst.append(pb)
    with kds.Batch(members) as b:
        b.step(2)
        b.synchronize()
    for pb in singles:
        pb.step(2)
    for pm, ps in zip(members, singles):
        assert pm.info()["steps_done"] == 2
        assert np.array_equal(pm.get_kinetic(), ps.get_kinetic())
    spec, W0 = cases[0]
    F, W = oracle.run(spec, W0, 2, threads=0)
    pt.check(members[0].moments(), W, members[0].get_kinetic(),
             np.ascontiguousarray(F.transpose(0, 2, 3, 1)), TOL["fp32"], label="degree-3 member")
    for pb in members + singles:
        pb.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_with_long_line_members(prec):
    """Members whose lines need rounds through the tile (512 cells along x at
    p = 2) beside ordinary members of the same degree and dimension: the
    batch puts them in a branch of their own, and every member still equals
    the same problem stepped alone, bit for bit."""
    import torch
    from paper_2212_11010_amd import kds, workloads as wl
    shapes = [([512, 4], [64, 4]), ([32, 24], [8, 6]), ([4, 512], [4, 128]), ([48, 16], [16, 8])]
    specs = []
    for i, (n, s) in enumerate(shapes):
        spec, W0 = wl.make_workload(2, n_cells=n, sub_cells=s, steps=3, seed=100 + i)
        specs.append((spec, W0))

    def build():
        out = []
        for spec, W0 in specs:
            pb = kds.Problem(spec, precision=prec)
            pb.set_state(torch.from_numpy(W0).cuda())
            out.append(pb)
        return out

    members, singles = build(), build()
    qmax = members[0].info()["line_qmax"]
    rounds = [max(pb.get_plan()["Q"]) > qmax for pb in members]
    assert rounds == [True, False, True, False], rounds
    with kds.Batch(members) as b:
        b.step(3)
        b.synchronize()
    for pb in singles:
        pb.step(3)
    for i, (pm, ps) in enumerate(zip(members, singles)):
        assert pm.info()["schedule"] == kds.KDS_SCHED_LINE
        assert np.array_equal(pm.get_kinetic(), ps.get_kinetic()), i
    for pb in members + singles:
        pb.close()
