"""Interface measurements and analytical laws used by the evaporation benchmarks, checked
against closed forms on synthetic fields (no GPU)."""
import math

import numpy as np
import pytest

from paper_2412_14859_amd import analytic, inputs


def test_variable_density_radius_solves_its_equation_and_reduces_to_the_linear_law():
    R0, phi, g, sigma = 44.0, 3e-3, 2.0, 0.1
    t = np.linspace(0.0, 0.9 * R0 * g / phi, 12)
    R = analytic.sphere_radius_variable(t, R0, phi, g, sigma)
    c = 4.0 * sigma / (3.0 * (1.0 / 3.0))
    lhs = R + c * np.log(R / R0)
    assert np.allclose(lhs, R0 - phi * t / g, rtol=0, atol=1e-9)
    # the Laplace term slows the shrinking: R above the linear law, the gap growing as R falls
    lin = analytic.sphere_radius_constant(t, R0, phi, g)
    assert np.all(R[1:] > lin[1:]) and np.all(np.diff(R - lin) > 0)
    # without surface tension it is the linear law
    R1 = analytic.sphere_radius_variable(t, R0, phi, g, 0.0)
    assert np.allclose(R1, lin, rtol=1e-10)


def test_half_max_volume_of_a_diffuse_sphere():
    shape = (64, 64, 64)
    R = 20.0
    d = inputs.sphere_distance(shape, (32.0, 32.0, 32.0), R)
    rr, _ = inputs.densities_from_distance(d, 2.0, (2.0, 1.0))
    r = analytic.sphere_radius(analytic.half_max_volume(rr))
    assert abs(r - R) < 0.05 * 1.0  # within a twentieth of a node
    torch = pytest.importorskip("torch")
    assert analytic.half_max_volume(torch.as_tensor(rr)) == analytic.half_max_volume(rr)


def test_hemisphere_and_disc_radius_from_volume():
    assert math.isclose(analytic.sphere_radius(2.0 / 3.0 * math.pi * 8.0, half=True), 2.0)
    assert math.isclose(analytic.sphere_radius(math.pi * 9.0, dim=2), 3.0)


@pytest.mark.parametrize("h", [10.0, 17.3, 40.25])
def test_film_height_from_the_wall_surface(h):
    shape = (64, 4, 4)
    d = inputs.flat_distance(shape, h + 0.5, axis=0)  # wall surface at z = 0.5
    rr, _ = inputs.densities_from_distance(d, 2.0, (2.0, 1.0))
    rr[0] = 0.0  # the solid layer
    assert abs(analytic.film_height(rr, axis=0, wall=0) - h) < 0.02
    # mirrored: the wall at the last layer
    assert abs(analytic.film_height(rr[::-1].copy(), axis=0, wall=-1) - h) < 0.02
    # a wall two layers thick
    d2 = inputs.flat_distance(shape, h + 1.5, axis=0)
    r2, _ = inputs.densities_from_distance(d2, 2.0, (2.0, 1.0))
    r2[:2] = 0.0
    assert abs(analytic.film_height(r2, axis=0, solid_layers=2) - h) < 0.02


def test_height_flux_ode_with_a_large_K_is_the_linear_law():
    # ln(K R0 / (R + K R0)) = -ln(1 + R / (K R0)) = -R / (K R0) + O(K^-2), so for large K
    # dR/dt = -phi_S / K: the uniform flux phi_S / K
    R0, phi_s, K = 30.0, 1e-3, 1e6
    t = np.linspace(0.0, 1e9, 5)
    R = analytic.hemisphere_radius_height_flux(t, R0, phi_s, K)
    assert np.allclose(R, R0 - phi_s / K * t, rtol=1e-6)
