"""The sampled two-step oracle of the full-size GPU checks (1-D line
transports + pointwise relaxation) reproduces the oracle's whole-grid steps
at every cell of small axis-aligned problems (2-D acoustics, 3-D Euler p = 2
and p = 3), to rounding: the reduction the full-size checks rely on."""
from __future__ import annotations

import numpy as np
import pytest

from tests.test_fullsize_gpu import TwoStepOracle, cell_id


@pytest.mark.parametrize("cfg,ov", [
    (2, dict(n_cells=[12, 8], sub_cells=[4, 4])),
    (3, dict(n_cells=[6, 6, 6], sub_cells=[3, 2, 3])),
    (4, dict(n_cells=[4, 4, 4], sub_cells=[2, 2, 4])),
])
def test_two_step_sampled_oracle_equals_whole_grid(orc, cfg, ov):
    from paper_2212_11010_amd import workloads as wl
    spec, W0 = wl.make_workload(cfg, **ov)
    c = orc.Config(spec)
    F = orc.init(c, W0)
    F1 = orc.step(c, F, 1)
    F2 = orc.step(c, F1, 1)
    Ns = spec["n_cells"][:spec["dim"]]
    rng = np.random.default_rng(3)
    two = TwoStepOracle(spec, W0)
    for _ in range(3):
        cc = [int(rng.integers(0, n)) for n in Ns]
        one, second = two.at(cc)
        i = cell_id(cc, Ns)
        scale = np.abs(F2).max()
        assert np.abs(one - F1[:, :, i]).max() <= 1e-13 * scale
        assert np.abs(second - F2[:, :, i]).max() <= 1e-13 * scale
