"""The seeded many-problem workload (uneven sizes for batched launches)."""
from __future__ import annotations

import math

from paper_2212_11010_amd import workloads as wl


def test_batch_workload_is_seeded_and_within_budget():
    a = wl.make_batch_workload()
    b = wl.make_batch_workload()
    assert len(a) == 48
    assert [s["name"] for s in a] == [s["name"] for s in b]
    total = sum(wl.unknowns(s) for s in a)
    assert total <= 4.0e9
    kinds = {s["law"] for s in a}
    assert kinds == {wl.LAW_LINEAR, wl.LAW_EULER}


def test_batch_members_satisfy_the_subdomain_condition():
    """Every member: S divides N and the kinetic Courant number nu = lambda
    dt / h is at most S (the iteration condition of Sec. 5.1 with the kinetic
    speed), with the recipe's degree and size ranges."""
    for s in wl.make_batch_workload():
        d = s["dim"]
        N, S = s["n_cells"][0], s["sub_cells"][0]
        assert all(n == N for n in s["n_cells"][:d]) and all(x == S for x in s["sub_cells"][:d])
        assert N % S == 0
        nu = max(abs(v) for v in s["vel"]) * s["dt"] * N
        assert math.isclose(nu, s["kinetic_courant"], rel_tol=1e-12)
        assert nu <= S
        if d == 2:
            assert 1 <= s["degree"] <= 3 and N in wl.BATCH_ACOUSTICS_N
        else:
            assert 1 <= s["degree"] <= 2 and N in wl.BATCH_EULER_N


def test_batch_member_spec_matches_a_direct_build():
    """The state-free spec equals the spec built with the state (small member)."""
    specs = wl.make_batch_workload(n_problems=6, max_unknowns=2e6, acoustics_n=(16,),
                                   euler_n=(8,), seed=3)
    for s in specs:
        args = dict(s["member_args"])
        cfg = args.pop("cfg")
        full, W0 = wl.make_workload(cfg, speed_bound=(cfg == 3), **args)
        for k in full:
            if k != "name":
                assert full[k] == s[k], (k, full[k], s[k])
        assert W0.shape == (N_cells(s), (s["degree"] + 1) ** s["dim"], s["m"])
        assert (wl.batch_member_state(s) == W0).all()


def N_cells(s):
    n = 1
    for a in range(s["dim"]):
        n *= s["n_cells"][a]
    return n
