"""Host logic of the Gamma calibration harness: interface measures and the count threshold."""
import math

import numpy as np
import pytest

from paper_2412_14859_amd import calibrate as cal


def test_interface_measures():
    assert cal.interface_measure("sphere", R=2.0) == pytest.approx(16.0 * math.pi)
    assert cal.interface_measure("sphere", R=2.0, dim=2) == pytest.approx(4.0 * math.pi)
    assert cal.interface_measure("hemisphere", R=2.0) == pytest.approx(8.0 * math.pi)
    assert cal.interface_measure("hemisphere", R=2.0, dim=2) == pytest.approx(2.0 * math.pi)
    assert cal.interface_measure("flat", L=5.0) == 25.0
    assert cal.interface_measure("flat", L=5.0, dim=2) == 5.0
    with pytest.raises(ValueError):
        cal.interface_measure("torus", R=1.0)


def test_threshold_selects_exactly_k_fluid_nodes():
    rng = np.random.default_rng(3)
    f = rng.random((4, 5, 6))
    fluid = rng.random(f.shape) > 0.2
    for k in (1, 7, int(fluid.sum()) - 1):
        lo, hi = cal.gamma_interval(f, fluid, k)
        assert lo < hi
        for g in (lo, 0.5 * (lo + hi)):
            assert int((f[fluid] > g).sum()) == k
        assert int((f[fluid] > hi).sum()) == k - 1
    # tied values (one magnitude per row of a flat interface): a wide interval
    rows = np.repeat(np.array([0.5, 0.4, 0.3, 0.2, 0.1])[:, None], 8, axis=1)
    lo, hi = cal.gamma_interval(rows, np.ones(rows.shape, bool), 16)
    assert (lo, hi) == (0.3, 0.4)
    with pytest.raises(ValueError):
        cal.gamma_interval(rows, np.ones(rows.shape, bool), 0)
