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


def test_rate_threshold_pools_the_snapshots():
    """Summed over snapshots, the site count at Gamma is the number of pooled values above
    it; the calibrated threshold makes that sum Sbar * sum_t A(t)."""
    rng = np.random.default_rng(5)
    snaps = [rng.random(200) * 0.6 for _ in range(7)]
    target = 3.0 * 123.4
    g, (lo, hi) = cal.gamma_for_rate(snaps, target)
    assert lo < g < hi
    total = sum(int((s > g).sum()) for s in snaps)
    assert total == round(target)
    # a moving flat interface: rows whose magnitudes shift between snapshots give a narrow
    # pooled interval where one static snapshot is degenerate
    rows = [np.repeat(np.array([0.52, 0.45, 0.31, 0.12]) + d, 16) for d in (0.0, 0.01, 0.02)]
    s_lo, s_hi = cal.gamma_interval(rows[0], np.ones(rows[0].shape, bool), 48)
    g, (p_lo, p_hi) = cal.gamma_for_rate(rows, 3 * 48)
    assert p_hi - p_lo < s_hi - s_lo


def test_rate_calibration_rejects_bad_arguments_before_any_device_work():
    from paper_2412_14859_amd import inputs
    w = inputs.workload("contrast_flat3d", shape=(16, 4, 4), ratio=1.0)
    for kw in (dict(snapshots=0), dict(iterations=0), dict(phi=0.0), dict(kind="torus")):
        args = dict(kind="flat", phi=3e-3)
        args.update(kw)
        with pytest.raises(ValueError):
            cal.calibrate_dynamic(w, **args)
