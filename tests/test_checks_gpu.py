"""State and stability checks of the C ABI (-m gpu): kds_set_state refuses
non-finite states; kds_info reports the sub-characteristic condition of
Sec. 2.1 (kinetic speeds above the largest wave speed) and the monotonicity
of the equilibrium (every dM_k/dW = a_k I + sum_i b_{k,i} A^i positive
semidefinite).  The expected values are closed forms of the workloads'
laws, not the library's own arithmetic:

* acoustics, velocities +-lambda e_i, M_{+-i} = W / (2d) +- A^i W / (2 lambda):
  the eigenvalues of dM are 1/(2d) +- c / (2 lambda) and 1/(2d), so the
  smallest is 1/(2d) - c/(2 lambda) (0 on the bound lambda = d c);
* D3Q4 with Maxwell (c = 1), V_k = lambda s_k, s_k in {+-1}^3:
  dM_k = I/4 + (sum_i s_k,i A^i) / (4 lambda), whose smallest eigenvalue is
  1/4 - sqrt(3) / (4 lambda) (0 at the paper's lambda = sqrt(3));
* Euler: the largest |u_i| + c over the nodes, recomputed here in numpy.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _problem(spec, prec="fp32"):
    from paper_2212_11010_amd import kds
    return kds.Problem(spec, precision=prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_set_state_refuses_nonfinite(prec):
    import torch
    from paper_2212_11010_amd import kds, workloads as wl
    spec, W0 = wl.make_workload(2, n_cells=[16, 8], sub_cells=[8, 8], steps=2)
    bad = [np.nan, np.inf, -np.inf] + ([1e300] if prec == "fp32" else [])
    with _problem(spec, prec) as pb:
        for v in bad:
            W = W0.copy()
            W[5, 3, 1] = v
            print("  W[5, 3, 1] =", v, flush=True)
            with pytest.raises(kds.KdsError) as ei:
                pb.set_state(torch.from_numpy(W).cuda())
            assert ei.value.status == kds.KDS_E_NONFINITE
            with pytest.raises(kds.KdsError) as ei:
                pb.step(1)
            assert ei.value.status == kds.KDS_E_STATE
        # a finite state afterwards is taken as usual (host copy path too)
        pb.set_state(W0)
        pb.step(1)
        assert pb.check_finite()


@pytest.mark.parametrize("scale", [1.0, 1.5, 0.25])
def test_acoustics_warnings_closed_form(scale):
    from paper_2212_11010_amd import workloads as wl
    spec, _ = wl.make_workload(2, n_cells=[16, 8], sub_cells=[8, 8], steps=2)
    spec = dict(spec, vel=[scale * v for v in spec["vel"]])
    lam, c, d = scale * spec["lam"], 1.0, 2   # A^i: c in the (0, i) and (i, 0) entries
    with _problem(spec) as pb:
        info = pb.info()
    want = 1.0 / (2 * d) - c / (2 * lam)
    print("  lambda %.3g: eq_min_eig %.6g (closed form %.6g), wave speed %.6g" %
          (lam, info["eq_min_eig"], want, info["max_wave_speed"]), flush=True)
    assert abs(info["eq_min_eig"] - want) <= 1e-13
    assert abs(info["max_wave_speed"] - c) <= 1e-13
    assert info["eq_monotone"] == (1 if want >= -1e-12 else 0)
    assert info["subchar_ok"] == (1 if lam > c else 0)


@pytest.mark.parametrize("scale", [1.0, 0.5])
def test_d3q4_maxwell_monotonicity_bound(scale):
    from paper_2212_11010_amd import workloads as wl
    spec, _ = wl.make_workload(6, n_cells=[4, 4, 4], sub_cells=[2, 2, 2], steps=1)
    spec = dict(spec, vel=[scale * v for v in spec["vel"]])
    lam = scale * spec["lam"]
    with _problem(spec) as pb:
        info = pb.info()
    want = 0.25 - math.sqrt(3.0) / (4.0 * lam)
    print("  lambda %.4g: eq_min_eig %.6g (closed form %.6g)" % (lam, info["eq_min_eig"], want),
          flush=True)
    assert abs(info["eq_min_eig"] - want) <= 1e-13
    assert info["eq_monotone"] == (1 if scale == 1.0 else 0)
    assert abs(info["max_wave_speed"] - 1.0) <= 1e-13   # Maxwell, c = 1
    assert info["subchar_ok"] == (1 if math.sqrt(3.0) * lam > 1.0 else 0)


def test_euler_wave_speed_of_the_state():
    import torch
    from paper_2212_11010_amd import workloads as wl
    spec, W0 = wl.make_workload(3, n_cells=[6, 4, 4], sub_cells=[3, 2, 2], steps=1)
    g = spec["law_params"][0]
    rho, mom, E = W0[..., 0], W0[..., 1:4], W0[..., 4]
    u = mom / rho[..., None]
    p = (g - 1.0) * (E - 0.5 * rho * (u * u).sum(-1))
    want = float(np.max(np.abs(u).max(-1) + np.sqrt(g * p / rho)))
    with _problem(spec) as pb:
        assert pb.info()["subchar_ok"] == -1            # no state yet
        pb.set_state(torch.from_numpy(W0).cuda())
        info = pb.info()
        print("  wave speed %.15g (numpy %.15g), min kinetic speed %.6g" %
              (info["max_wave_speed"], want, spec["lam"]), flush=True)
        assert abs(info["max_wave_speed"] - want) <= 1e-13 * want
        assert info["subchar_ok"] == 1 and info["eq_monotone"] == -1
        # a node with negative pressure has no real wave speed
        W = W0.copy()
        # (energy below the kinetic energy: p < 0; p = 0 where u = 0)
        W[7, 2, 4] = 0.25 * float((mom[7, 2] ** 2).sum() / rho[7, 2])
        pb.set_state(W)
        info = pb.info()
        assert math.isinf(info["max_wave_speed"]) and info["subchar_ok"] == 0
