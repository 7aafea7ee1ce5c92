"""Pins of the oracle's blue pressure outlet (Zou and He, on the end planes of the last lattice
axis; used with density contrast in Sec. III)."""
import numpy as np
import pytest

from oracle.oracle import Oracle, tables
from paper_2412_14859_amd import inputs


def _axis(Q):
    return 0 if Q == 19 else 1  # array axis of the last lattice axis (z, or y in 2D)


def _planes(Q, shape):
    ax = _axis(Q)
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[ax], hi[ax] = 0, shape[ax] - 1
    return tuple(lo), tuple(hi)


@pytest.mark.parametrize("Q,shape", [(9, (1, 14, 9)), (19, (9, 6, 7))])
def test_blue_at_rest_at_the_outlet_density_is_a_fixed_point(Q, shape):
    p = dict(inputs._base(Q, shape), phi=0.0)
    ora = Oracle(p)
    ora.init_equilibrium(np.zeros(shape), np.full(shape, 1.0))
    f0 = ora.populations()
    ora.set_outlet(True, True, 1.0)
    ora.step(5)
    assert np.abs(ora.populations() - f0).max() < 1e-15


@pytest.mark.parametrize("Q,shape", [(9, (1, 60, 12)), (19, (44, 8, 9))])
def test_outlet_planes_hold_the_blue_density_without_tangential_flow(Q, shape):
    """A drop in the middle, blue at 1.05 relaxing to 1.0 through the outlets.  The outflow
    carries some of the drop's red tail out, but no red enters, so the red mass falls by at
    least the sink."""
    t = tables(Q)
    c = np.asarray(t["c"])
    nz, ny, nx = shape
    centre = (nx / 2, ny / 2, nz / 2 if Q == 19 else 0.0)
    d = inputs.sphere_distance(shape, centre, 3.0)
    rr, rb = inputs.densities_from_distance(d, 2.0, (1.0, 1.05))
    p = dict(inputs._base(Q, shape), phi=1e-3, rho_in=(1.0, 1.0))
    ora = Oracle(p)
    ora.init_equilibrium(rr, rb)
    ora.set_outlet(True, True, 1.0)
    ax = _axis(Q)
    a = 2 if Q == 19 else 1  # lattice axis index of the outlet normal
    m0 = ora.observables()
    mean_b = []
    for _ in range(40):
        ora.step(1)
        f = ora.populations()
        for plane in _planes(Q, shape):
            fb = f[1][(slice(None),) + plane]
            fr = f[0][(slice(None),) + plane]
            assert np.abs(fb.sum(0) - 1.0).max() < 1e-14
            for tdir in range(3):
                if tdir == a or (Q == 9 and tdir == 2):
                    continue
                mom = np.tensordot(c[:, tdir], fb, axes=(0, 0))
                assert np.abs(mom).max() < 1e-14
            # no red enters through the plane
            sign = 1 if plane[ax] != 0 else -1
            entering = [i for i in range(Q) if sign * c[i, a] == -1]
            assert np.abs(fr[entering]).max() == 0.0
        mean_b.append(float(f[1].sum() / np.prod(shape)))
    # the excess blue leaves through the outlets
    assert mean_b[-1] < mean_b[0] < 1.05 and mean_b[-1] - 1.0 < 0.6 * (mean_b[0] - 1.0)
    # red leaves only through the sink
    m1 = ora.observables()
    dr = (m0["mass_r"] - m1["mass_r"]) - m1["sink_total"]
    assert dr > -1e-13 * m0["mass_r"], dr


@pytest.mark.parametrize("Q,shape", [(9, (1, 60, 12))])
def test_without_outflow_red_changes_only_by_the_sink(Q, shape):
    """Blue already at the outlet density and the outlets 27 nodes from the drop: nothing
    drives an outflow and the drop's red tail (which spreads by diffusion where the colour
    gradient is below the recolouring fade) does not reach them within the run, so the red
    mass falls by the sink alone (to 1e-8)."""
    nz, ny, nx = shape
    centre = (nx / 2, ny / 2, nz / 2 if Q == 19 else 0.0)
    d = inputs.sphere_distance(shape, centre, 3.0)
    rr, rb = inputs.densities_from_distance(d, 2.0, (1.0, 1.0))
    p = dict(inputs._base(Q, shape), phi=1e-3)
    ora = Oracle(p)
    ora.init_equilibrium(rr, rb)
    ora.set_outlet(True, True, 1.0)
    m0 = ora.observables()
    ora.step(40)
    m1 = ora.observables()
    dr = (m0["mass_r"] - m1["mass_r"]) - m1["sink_total"]
    assert m1["sink_total"] > 0 and abs(dr) < 1e-8 * m0["mass_r"], dr
