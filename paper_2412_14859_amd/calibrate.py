"""Calibration of the site threshold Gamma (Sec. II.B and Sec. III).

The paper picks Gamma so that the mass-loss rate of the simulation equals the analytical one
(Eq. satisfy): with the per-site sink s = phi / Sbar, the number of sites must be Sbar times
the interface measure A (length in 2D, area in 3D).  For a drop at rest the sites are the
nodes with ||F|| > Gamma, so the calibrated Gamma lies between the k-th and (k+1)-th largest
gradient magnitude over the fluid nodes, k = round(Sbar A).

The harness equilibrates the drop on the GPU without flux (the soft site rule carries ||F||
per node, so the gradient field is read from the carried site data), then takes that
threshold on the host.  Geometry measures: `interface_measure`.
"""
import math

import numpy as np


def interface_measure(kind, R=None, L=None, dim=3):
    """Analytical interface measure: 'sphere' (4 pi R^2; circle 2 pi R in 2D), 'hemisphere'
    (cap on a wall: 2 pi R^2; half circle pi R in 2D), 'flat' (L^2, or L in 2D)."""
    if kind == "sphere":
        return 4.0 * math.pi * R * R if dim == 3 else 2.0 * math.pi * R
    if kind == "hemisphere":
        return 2.0 * math.pi * R * R if dim == 3 else math.pi * R
    if kind == "flat":
        return L * L if dim == 3 else L
    raise ValueError(kind)


def gamma_interval(fmag, fluid, k):
    """The thresholds with exactly k fluid nodes above them: [(k+1)-th, k-th largest value of
    fmag over the fluid nodes).  Where many nodes share a value (a flat interface has one
    gradient magnitude per row) the count jumps and the interval is wide."""
    v = np.sort(np.asarray(fmag)[np.asarray(fluid, bool)].ravel())[::-1]
    if not 0 < k < v.size:
        raise ValueError("site count out of range")
    return float(v[k]), float(v[k - 1])


def gamma_for_count(fmag, fluid, k):
    """Midpoint of gamma_interval."""
    lo, hi = gamma_interval(fmag, fluid, k)
    return 0.5 * (lo + hi)


def equilibrated_gradient(workload, steps, precision="fp64", device="cuda:0"):
    """||F|| per node after `steps` steps without flux, and the drop volume V = M_r/rho_r^in."""
    from paper_2412_14859_amd import cgevap
    w = workload
    p = dict(w["params"], phi=0.0, site_rule="soft", kappa=1.0)
    sim = cgevap.Simulation(p, w["rho_r"], w["rho_b"], solid=w["solid"], precision=precision,
                            device=device)
    sim.step(steps)
    fmag = sim.carry.cpu().numpy().copy()
    v = sim.observables()["v_mass"]
    sim.close()
    return fmag, v


def calibrate(workload, kind, steps, sbar=3.0, precision="fp64", radius_from_volume=True):
    """Gamma for which the equilibrated drop has Sbar * A sites.  The radius of a sphere or
    hemisphere is taken from the equilibrated volume (R = (3V / 4 pi)^(1/3) or
    (3V / 2 pi)^(1/3); r = (V / pi)^(1/2) or (2V / pi)^(1/2) in 2D) unless
    radius_from_volume is False, when the workload's radius is used.  Returns (Gamma, details)."""
    p = workload["params"]
    dim = 2 if int(p["Q"]) == 9 else 3
    fmag, v = equilibrated_gradient(workload, steps, precision)
    fluid = np.ones(fmag.shape, bool) if workload["solid"] is None else workload["solid"] == 0
    R = None
    if kind in ("sphere", "hemisphere"):
        if radius_from_volume:
            f = (2.0 if kind == "hemisphere" else 1.0)
            R = (3.0 * v * f / (4.0 * math.pi)) ** (1.0 / 3.0) if dim == 3 else \
                math.sqrt(v * f / math.pi)
        else:
            R = workload["radius"]
        A = interface_measure(kind, R=R, dim=dim)
    else:
        nz, ny, nx = p["shape"]
        A = interface_measure("flat", L=nx, dim=dim) if dim == 2 else nx * ny
    k = int(round(sbar * A))
    lo, hi = gamma_interval(fmag, fluid, k)
    return 0.5 * (lo + hi), {"sites": k, "measure": A, "radius": R, "volume": v,
                             "interval": (lo, hi),
                             "sites_at": lambda g: int((fmag[fluid] > g).sum())}
