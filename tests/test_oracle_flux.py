"""Pins of the oracle's height-dependent flux (Eq. heated): Phi = phi_S / (K + h / h_s) with h
the red thickness of the column normal to the substrate."""
import numpy as np

from oracle.oracle import Oracle
from paper_2412_14859_amd import inputs


def _sharp_columns(Q, shape, heights):
    """Wall layer at index 0 of the substrate axis; pure red below height h(column) (counted
    in fluid nodes), pure blue above."""
    nz, ny, nx = shape
    p = inputs._base(Q, shape)
    solid = np.zeros(shape, np.uint8)
    rr = np.zeros(shape)
    if Q == 19:
        solid[0] = 1
        k = np.arange(nz)[:, None, None]
        red = (k >= 1) & (k <= heights[None])
    else:
        solid[:, 0, :] = 1
        k = np.arange(ny)[None, :, None]
        red = (k >= 1) & (k <= heights[None, None, :])
    rr[red & (solid == 0)] = 1.0
    rb = np.where((solid == 0) & ~red, 1.0, 0.0)
    return p, solid, rr, rb


def test_sharp_columns_give_the_closed_form_flux():
    rng = np.random.default_rng(7)
    for Q, shape in ((19, (9, 5, 6)), (9, (1, 11, 7))):
        ncol = shape[1] * shape[2] if Q == 19 else shape[2]
        hmax = (shape[0] if Q == 19 else shape[1]) - 1
        heights = rng.integers(0, hmax, size=ncol)
        h2 = heights.reshape(shape[1], shape[2]) if Q == 19 else heights
        p, solid, rr, rb = _sharp_columns(Q, shape, h2)
        ora = Oracle(p, solid=solid)
        ora.init_equilibrium(rr, rb)
        phi_s, K, hs = 2e-3, 0.5, 7.0
        ora.set_height_flux(phi_s, K, hs, every=1)
        ora.step(1)
        got = ora.phi_field()
        want_col = phi_s / (K + h2 / hs)
        want = np.broadcast_to(want_col[None] if Q == 19 else want_col[None, None, :], shape)
        assert np.abs(got - want).max() <= 1e-15 * phi_s


def test_flux_field_refreshes_every_m_steps():
    w = inputs.workload("sessile3d", shape=(10, 12, 12), radius=4.0)
    p = dict(w["params"], phi=1e-3)
    ora = Oracle(p, solid=w["solid"], phi_field=w["phi_field"])
    ora.init_equilibrium(w["rho_r"], w["rho_b"])
    ora.set_height_flux(1e-2, 1.0, 4.0, every=3)
    fields = []
    for _ in range(7):
        ora.step(1)
        fields.append(ora.phi_field())
    # refreshed before steps 0, 3 and 6: constant in between
    assert np.array_equal(fields[0], fields[1]) and np.array_equal(fields[1], fields[2])
    assert np.array_equal(fields[3], fields[4]) and np.array_equal(fields[4], fields[5])
    assert not np.array_equal(fields[2], fields[3])
    # constant along each column, larger where the drop is thin (at the rim) than at its top
    f = fields[-1]
    assert np.ptp(f, axis=0).max() == 0.0
    assert f[0].max() > f[0][6, 6]
