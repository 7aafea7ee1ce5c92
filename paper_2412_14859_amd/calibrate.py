"""Calibration of the site threshold Gamma (Sec. II.B and Sec. III).

The paper picks Gamma so that the mass-loss rate of the simulation equals the analytical one
(Eq. satisfy): with the per-site sink s = phi / Sbar, the number of sites must be Sbar times
the interface measure A (length in 2D, area in 3D).  For a drop at rest the sites are the
nodes with ||F|| > Gamma, so the calibrated Gamma lies between the k-th and (k+1)-th largest
gradient magnitude over the fluid nodes, k = round(Sbar A).

The harness equilibrates the drop on the GPU without flux (the soft site rule carries ||F||
per node, so the gradient field is read from the carried site data), then takes that
threshold on the host.  Geometry measures: `interface_measure`.

`calibrate_dynamic` matches the rates over an evaporating run instead, which is the paper's
criterion: the mass the sink removes over the run, (phi / Sbar) times the site count summed
over the steps, must equal phi times the interface measure summed over the steps.  A moving
interface crosses the lattice, so the site count at a fixed Gamma changes as it moves (for a
flat film the static count is degenerate).  The run uses soft sites of small width, which
act as hard sites at a starting threshold while carrying ||F|| of every node; at each of a
set of evenly spaced snapshots it records ||F|| and the interface measure A(t) from the
half-maximum contour.  Summed over the snapshots, the site count at Gamma is the number of
pooled gradient values above Gamma, so the calibrated Gamma is the threshold with
Sbar * sum_t A(t) pooled values above it.  The trajectory depends weakly on the threshold it
ran with; `iterations` > 1 runs again from the previous result.

The criterion above needs the interface measure, and a measure taken from the half-maximum
radius is not the one whose rate of change fixes the mass: the drop's red mass is that of a
sphere of its equimolar radius, which lies outside the half-maximum contour by an amount that
grows with the interface width.  The paper compares the measured radius (or height) with the
analytical law directly, so `criterion="curve"` matches that instead: the least-squares slope
of the measured position over the run at the threshold it ran with, scaled by the pooled site
count at a trial threshold over that at the run's (the sink, and so the slope, is proportional
to the site count), must equal the law's slope -phi / rho0.
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


def gamma_for_rate(snapshots, target):
    """Thresholds with round(target) values of the pooled snapshots (1-D arrays of gradient
    magnitudes; values below any floor may be left out) above them: the interval of
    `gamma_interval` over the pool, and its midpoint."""
    v = np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in snapshots])
    lo, hi = gamma_interval(v, np.ones(v.shape, bool), int(round(target)))
    return 0.5 * (lo + hi), (lo, hi)


def _position(sim, kind, dim, solid_layers):
    from paper_2412_14859_amd import analytic
    rr = sim.fields()["rho_r"]
    if kind == "flat":
        return analytic.film_height(rr, axis=0 if dim == 3 else 1,
                                    solid_layers=solid_layers), float(rr.max())
    v = analytic.half_max_volume(rr)
    return analytic.sphere_radius(v, dim=dim, half=kind == "hemisphere"), float(rr.max())


def calibrate_dynamic(workload, kind, phi, equil=4000, t_star=0.8, snapshots=40, sbar=3.0,
                      gamma0=None, kappa=1e-4, precision="fp32s", outlet=None, solid_layers=1,
                      floor=0.05, iterations=1, criterion="rate", device="cuda:0"):
    """Gamma matching the mass-loss rate over an evaporating run (see the module notes).

    workload: an `inputs.workload` dict; kind: 'sphere', 'hemisphere' or 'flat' (the
    interface measure); phi: the flux of the run, which lasts until t* = t phi / (x0 rho0) =
    t_star (x0 the initial radius or film height, rho0 the equilibrium red density); outlet:
    (lo, hi) blue outlets switched on for the evaporation; solid_layers: wall thickness under
    a film; criterion: "rate" (sites against Sbar times the interface measure) or "curve"
    (the slope of the measured position against the law's).  Returns (Gamma, details)."""
    from paper_2412_14859_amd import cgevap
    if snapshots < 1 or iterations < 1 or not phi > 0:
        raise ValueError("snapshots and iterations must be >= 1 and phi > 0")
    if kind not in ("sphere", "hemisphere", "flat"):
        raise ValueError(kind)
    if criterion not in ("rate", "curve"):
        raise ValueError(criterion)
    w = workload
    p0 = w["params"]
    dim = 2 if int(p0["Q"]) == 9 else 3
    shape = p0["shape"]
    fluid = None if w["solid"] is None else (np.asarray(w["solid"]) == 0)
    g = float(p0["gamma"] if gamma0 is None else gamma0)
    history = []
    for _ in range(iterations):
        p = dict(p0, phi=0.0, site_rule="soft", kappa=kappa, gamma=g)
        sim = cgevap.Simulation(p, w["rho_r"], w["rho_b"], solid=w["solid"],
                                phi_field=np.zeros(shape), precision=precision, device=device)
        sim.step(equil)
        x0, rho0 = _position(sim, kind, dim, solid_layers)
        sim.set_counters()
        if outlet is not None:
            sim.set_outlet(*outlet, 1.0)
        sim.phi_field.fill_(phi)
        t_end = t_star * x0 * rho0 / phi
        chunk = max(1, int(t_end / snapshots))

        def measure(x):
            if kind == "flat":  # the film's area: nx * ny (the length nx in 2D)
                return float(shape[2] * shape[1]) if dim == 3 else float(shape[2])
            return interface_measure(kind, R=x, dim=dim)

        A0 = measure(x0)
        pool, measures, xs = [], [], [x0]
        for _ in range(snapshots):
            sim.step(chunk)
            fm = sim.carry.cpu().numpy()
            vals = fm if fluid is None else fm[fluid]
            pool.append(vals[vals > floor].copy())
            x, _ = _position(sim, kind, dim, solid_layers)
            xs.append(x)
            measures.append(measure(x))
        obs = sim.observables()
        sim.close()
        ts = chunk * np.arange(snapshots + 1, dtype=np.float64)
        slope = float(np.polyfit(ts, np.asarray(xs), 1)[0])  # measured position per step
        slope_law = -phi / rho0
        if criterion == "rate":
            target = sbar * float(np.sum(measures))
        else:
            n_run = float(sum(int((a > g).sum()) for a in pool))
            target = n_run * slope_law / slope
        g_new, interval = gamma_for_rate(pool, target)
        # the realised rate of this run against the analytical one, phi times the integral
        # of A over the run (trapezoidal rule over the snapshots and the start)
        integral = chunk * (0.5 * A0 + float(np.sum(measures[:-1])) + 0.5 * measures[-1])
        realised = obs["sink_total"] / (phi * integral)
        history.append({"gamma_run": g, "gamma": g_new, "interval": interval,
                        "realised_rate_ratio": realised, "slope_ratio": slope / slope_law,
                        "x0": x0, "rho0": rho0, "steps": chunk * snapshots, "x_end": x})
        g = g_new
    return g, {"history": history, "sites_target": target}
