"""Interface positions measured from density fields, and the analytical laws the paper
compares them with (Sec. III).

The interface lies where the density of the evaporating (red) component is half its
maximum.  A drop's radius is that of the sphere (or hemisphere, or disc) of equal volume to
the region above half the maximum; a flat film's height is where the mean red profile along
the wall normal crosses half its maximum (linear interpolation), measured from the wall
surface, which sits halfway between the solid layer and the first fluid layer.

Laws (lattice units, c_s^2 = 1/3, rho_b the surrounding blue density):
  flat film, constant density:      h(t) = h0 - phi t / rho0                  (Sec. flat)
  sphere, constant density:         R(t) = R0 - phi t / rho0                  (Sec. sphere)
  sphere, Laplace-dependent density: R + (4 sigma / (3 c_s^2 rho_b)) ln(R / R0)
                                      = R0 - phi t / (gamma rho_b)            (Appendix)
  hemisphere with height flux:      dR/dt = (phi_S R0 / R) ln(K R0 / (R + K R0))
                                                                  (Sec. varying flux)
  pinned cap, constant density:     h(t) = h0 - 2 phi t / rho0                (Sec. pinned cap)
  pinned cap, Laplace-dependent density (contact radius a held):
      h + c [ln((a^2 + h^2) / (a^2 + h0^2)) - a^4 / (a^2 + h^2)^2]
        = h0 - 2 phi t / (gamma rho_b) - c a^4 / (a^2 + h0^2)^2,  c = 4 sigma / (3 c_s^2 rho_b)
                                                                  (Appendix B)
A cap's height is measured on the column through its axis from the top surface of the
cavity ring to the half-maximum crossing; its contact radius is the radius of the disc of
equal area to the part of the plane just above the ring where the red density exceeds half
its maximum.
"""
import math

import numpy as np

CS2 = 1.0 / 3.0


def _np(a):
    return a.detach().cpu().numpy() if hasattr(a, "detach") else np.asarray(a)


def half_max_volume(rho_r, solid=None):
    """Number of fluid nodes whose red density exceeds half of its maximum; the maximum is
    taken over the fluid nodes.  Accepts a numpy array or a torch tensor (reduced where it
    lives)."""
    if hasattr(rho_r, "detach"):
        r = rho_r if solid is None else rho_r.masked_fill(
            rho_r.new_tensor(np.asarray(solid) != 0, dtype=bool), 0.0)
        return float((r > 0.5 * r.max()).sum().item())
    r = np.asarray(rho_r, dtype=np.float64)
    if solid is not None:
        r = np.where(np.asarray(solid) != 0, 0.0, r)
    return float((r > 0.5 * r.max()).sum())


def sphere_radius(volume, dim=3, half=False):
    """Radius of the sphere (disc in 2D) of the given volume; half=True for a hemisphere
    (half disc)."""
    v = volume * (2.0 if half else 1.0)
    return (3.0 * v / (4.0 * math.pi)) ** (1.0 / 3.0) if dim == 3 else math.sqrt(v / math.pi)


def film_height(rho_r, axis=0, wall=0, solid_layers=1):
    """Height of a flat red film on a wall `solid_layers` thick at the start (wall=0) or end
    of `axis`: the mean red density over each layer normal to `axis`, the first crossing of
    half its maximum going away from the wall, interpolated linearly, measured from the wall
    surface."""
    r = _np(rho_r).astype(np.float64)
    other = tuple(i for i in range(r.ndim) if i != axis)
    prof = r.mean(axis=other)
    if wall != 0:
        prof = prof[::-1]
    prof = prof[solid_layers:]
    half = 0.5 * prof.max()
    k = 0
    while k < prof.size and prof[k] > half:
        k += 1
    if k == 0 or k == prof.size:
        return 0.0 if k == 0 else float(prof.size - 0.5)
    # crossing between fluid layers k - 1 and k (layer j is centred j + 1/2 from the surface)
    frac = (prof[k - 1] - half) / (prof[k - 1] - prof[k])
    return (k - 1 + frac) + 0.5


def flat_height(t, h0, phi, rho0):
    return h0 - phi * np.asarray(t, dtype=np.float64) / rho0


def sphere_radius_constant(t, R0, phi, rho0):
    return R0 - phi * np.asarray(t, dtype=np.float64) / rho0


def sphere_radius_variable(t, R0, phi, gamma, sigma, rho_b=1.0):
    """Root of R + (4 sigma / (3 c_s^2 rho_b)) ln(R / R0) = R0 - phi t / (gamma rho_b) for
    each t (the left side increases with R, so the root on (0, R0] is unique)."""
    from scipy.optimize import brentq
    c = 4.0 * sigma / (3.0 * CS2 * rho_b)
    out = []
    for ti in np.atleast_1d(np.asarray(t, dtype=np.float64)):
        rhs = R0 - phi * ti / (gamma * rho_b)
        g = lambda R: R + c * math.log(R / R0) - rhs
        out.append(R0 if ti == 0 else brentq(g, 1e-12 * R0, R0, xtol=1e-12 * R0))
    return np.array(out)


def hemisphere_radius_height_flux(t, R0, phi_s, K):
    """dR/dt = (phi_S R0 / R) ln(K R0 / (R + K R0)), integrated with RK45."""
    from scipy.integrate import solve_ivp
    t = np.asarray(t, dtype=np.float64)
    sol = solve_ivp(lambda _, r: [phi_s * R0 / r[0] * math.log(K * R0 / (r[0] + K * R0))],
                    (0.0, float(t[-1])), [R0], t_eval=t, method="RK45", rtol=1e-9, atol=1e-9)
    return sol.y[0]


def cap_height(rho_r, top, centre=None):
    """Apex height of a cap above the surface at z = top (between node layers): going up the
    column through `centre` (x, y node indices; default the middle node), the last crossing
    of half the red maximum, interpolated linearly, minus top."""
    r = _np(rho_r).astype(np.float64)
    nz, ny, nx = r.shape
    cx, cy = centre if centre is not None else (nx // 2, ny // 2)
    col = r[:, cy, cx]
    half = 0.5 * r.max()
    k = int(math.ceil(top))
    while k + 1 < nz and col[k + 1] > half:
        k += 1
    if col[k] <= half or k + 1 >= nz:
        return 0.0
    frac = (col[k] - half) / (col[k] - col[k + 1])
    return k + frac - top


def contact_radius(rho_r, z):
    """Radius of the disc of equal area to the nodes of plane z above half the red
    maximum."""
    if hasattr(rho_r, "detach"):
        half = 0.5 * rho_r.max()
        return math.sqrt(float((rho_r[z] > half).sum().item()) / math.pi)
    r = np.asarray(rho_r, dtype=np.float64)
    return math.sqrt(float((r[z] > 0.5 * r.max()).sum()) / math.pi)


def cap_height_constant(t, h0, phi, rho0):
    return h0 - 2.0 * phi * np.asarray(t, dtype=np.float64) / rho0


def cap_height_variable(t, h0, a, phi, gamma, sigma, rho_b=1.0):
    """Root h of the Laplace-dependent pinned-cap law for each t.  The left side
    h + c [ln(a^2 + h^2) - a^4 / (a^2 + h^2)^2] increases with h, so the root on (0, h0] is
    unique."""
    from scipy.optimize import brentq
    c = 4.0 * sigma / (3.0 * CS2 * rho_b)
    a2 = a * a

    def lhs(h):
        return h + c * (math.log((a2 + h * h) / (a2 + h0 * h0)) - a2 * a2 / (a2 + h * h) ** 2)

    out = []
    for ti in np.atleast_1d(np.asarray(t, dtype=np.float64)):
        rhs = h0 - 2.0 * phi * ti / (gamma * rho_b) - c * a2 * a2 / (a2 + h0 * h0) ** 2
        if ti == 0:
            out.append(h0)
            continue
        lo = 1e-9 * h0
        if lhs(lo) > rhs:
            out.append(0.0)  # evaporated
            continue
        out.append(brentq(lambda h: lhs(h) - rhs, lo, h0, xtol=1e-12 * h0))
    return np.array(out)
