"""kds_moments_static, the entry point that allocates nothing: through the C
ABI, its output must equal kds_moments' (same kernel, same FP64 sums:
bitwise), on two calls in a row on one GPU, the second with a smaller input,
so that the second call reads only what it wrote into the shared static
scratch array.  Oversized and out-of-range requests are rejected on the host
(KDS_E_INVALID) before any device work."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _problem(cfg, **ov):
    import torch
    from paper_2212_11010_amd import kds
    from paper_2212_11010_amd import workloads as wl
    spec, W0 = wl.make_workload(cfg, **ov)
    pb = kds.Problem(spec, precision="fp32")
    pb.set_state(torch.from_numpy(W0).cuda())
    pb.step(spec["steps"])
    return pb


def _static(pb, begin, count):
    from paper_2212_11010_amd import kds
    out = np.full((count, pb.m), np.nan)
    st = kds.lib().kds_moments_static(pb.h, C.c_int64(begin), C.c_int64(count),
                                      C.c_void_p(out.ctypes.data))
    assert st == kds.KDS_OK, kds.kds_last_error(pb.h)
    return out


def test_moments_static_matches_moments_on_two_calls():
    big = _problem(2, n_cells=[64, 48], sub_cells=[16, 8], steps=3)       # 27648 nodes
    small = _problem(3, n_cells=[6, 4, 4], sub_cells=[3, 2, 2], steps=2)  # 2592 nodes
    try:
        Wb = big.moments().reshape(-1, big.m)
        Ws = small.moments().reshape(-1, small.m)
        print("nodes", Wb.shape[0], Ws.shape[0], flush=True)
        got_b = _static(big, 0, Wb.shape[0])
        assert np.array_equal(got_b, Wb)
        # second call, smaller input (another problem, other m): only its values
        got_s = _static(small, 0, Ws.shape[0])
        assert np.array_equal(got_s, Ws)
        # a range in the middle, again after the smaller call
        got_r = _static(big, 1000, 777)
        assert np.array_equal(got_r, Wb[1000:1777])
        assert _static(big, 5, 0).shape == (0, big.m)
    finally:
        big.close()
        small.close()


def test_moments_static_rejects_bad_ranges():
    from paper_2212_11010_amd import kds
    pb = _problem(2, n_cells=[16, 16], sub_cells=[8, 8], steps=1)
    try:
        n = pb.ncell * pb.nn
        out = np.zeros((n + 1, pb.m))
        L = kds.lib()
        for begin, count in ((0, n + 1), (-1, 4), (n, 1), (3, -2)):
            st = L.kds_moments_static(pb.h, C.c_int64(begin), C.c_int64(count),
                                      C.c_void_p(out.ctypes.data))
            assert st == kds.KDS_E_INVALID, (begin, count)
        assert L.kds_moments_static(pb.h, C.c_int64(0), C.c_int64(1), None) == kds.KDS_E_INVALID
    finally:
        pb.close()


def test_moments_static_full_scratch_and_oversize():
    """A problem with more nodes than the scratch holds: exactly the largest
    range (32 MiB of W) is served, one node more is rejected."""
    from paper_2212_11010_amd import kds
    pb = _problem(2, n_cells=[512, 512], sub_cells=[32, 32], steps=1)
    try:
        max_nodes = (32 << 20) // (8 * pb.m)
        assert pb.ncell * pb.nn > max_nodes + 1
        W = pb.moments().reshape(-1, pb.m)
        got = _static(pb, 7, max_nodes)
        assert np.array_equal(got, W[7:7 + max_nodes])
        out = np.zeros((max_nodes + 1, pb.m))
        st = kds.lib().kds_moments_static(pb.h, C.c_int64(0), C.c_int64(max_nodes + 1),
                                          C.c_void_p(out.ctypes.data))
        assert st == kds.KDS_E_INVALID
        assert "nodes per call" in kds.kds_last_error(pb.h)
    finally:
        pb.close()
