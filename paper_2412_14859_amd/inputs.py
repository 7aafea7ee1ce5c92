"""Seeded synthetic inputs: initial component densities, solid flags, flux fields, targets.

This module holds geometry and random numbers only -- none of the lattice Boltzmann
arithmetic.  It serves both the HIP path and the test oracle.  Every field is float64 in
[nz][ny][nx] order (nz = 1 for two-dimensional lattices); node (x, y, z) sits at integer
coordinates.

Initial condition (the workloads' reading of "tanh profile of width w"): the red volume
fraction is c(x) = (1 + tanh(d(x)/w))/2, d the signed distance to the drop surface,
positive inside; rho_r = c rho_r_in, rho_b = (1 - c) rho_b_in; zero velocity.

The surface-tension parameter A of the workloads is the perturbation amplitude
A = (9/4) sigma / tau at tau = 1, hence sigma = 4A/9.
"""
import math

import numpy as np

RED, BLUE = 0, 1


def grid(shape):
    """Node coordinates (z, y, x) as float64 arrays of the given shape (nz, ny, nx)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return z, y, x


def densities_from_distance(d, width, rho_in):
    c = 0.5 * (1.0 + np.tanh(d / width))
    return c * rho_in[0], (1.0 - c) * rho_in[1]


def sphere_distance(shape, center, radius):
    """Signed distance to a circle (2D, shape[0] == 1) or sphere; center = (cx, cy, cz)."""
    z, y, x = grid(shape)
    cx, cy, cz = center
    r2 = (x - cx) ** 2 + (y - cy) ** 2
    if shape[0] > 1:
        r2 = r2 + (z - cz) ** 2
    return radius - np.sqrt(r2)


def flat_distance(shape, height, axis=1):
    """Signed distance to the plane coordinate == height along axis (0 z, 1 y, 2 x);
    red below the plane."""
    coords = grid(shape)
    return height - coords[axis]


def ellipse_distance(shape, center, a, b, iters=120):
    """Signed distance to the ellipse x^2/a^2 + y^2/b^2 = 1 (2D, a >= b), by bisection on the
    foot-point parameter (D. Eberly, "Distance from a point to an ellipse")."""
    assert a >= b
    with np.errstate(divide="ignore", invalid="ignore"):
        return _ellipse_distance(shape, center, a, b, iters)


def _ellipse_distance(shape, center, a, b, iters):
    _, y, x = grid(shape)
    y0 = np.abs(x - center[0])
    y1 = np.abs(y - center[1])
    z0, z1 = y0 / a, y1 / b
    g = z0 * z0 + z1 * z1 - 1.0
    r0 = (a / b) ** 2
    n0 = r0 * z0
    s0 = z1 - 1.0
    s1 = np.where(g < 0.0, 0.0, np.sqrt(n0 * n0 + z1 * z1) - 1.0)
    for _ in range(iters):
        s = 0.5 * (s0 + s1)
        gs = (n0 / (s + r0)) ** 2 + (z1 / (s + 1.0)) ** 2 - 1.0
        s0 = np.where(gs > 0.0, s, s0)
        s1 = np.where(gs > 0.0, s1, s)
    s = 0.5 * (s0 + s1)
    x0 = r0 * y0 / (s + r0)
    x1 = y1 / (s + 1.0)
    dist = np.sqrt((x0 - y0) ** 2 + (x1 - y1) ** 2)
    # points on the major axis (y1 == 0) inside the evolute segment
    on_axis = y1 == 0.0
    num, den = a * y0, a * a - b * b
    xde = np.clip(num / den, 0.0, 1.0)
    d_axis = np.where(num < den, np.sqrt((a * xde - y0) ** 2 + (b * np.sqrt(1.0 - xde * xde)) ** 2),
                      np.abs(y0 - a))
    dist = np.where(on_axis, d_axis, dist)
    return np.where(g < 0.0, dist, -dist)


def wall_layers(shape, axis, layers):
    """uint8 solid flags: the given index layers along axis (0 z, 1 y, 2 x) are solid."""
    s = np.zeros(shape, np.uint8)
    for layer in layers:
        idx = [slice(None)] * 3
        idx[axis] = layer
        s[tuple(idx)] = 1
    return s


def uniform_noise(shape, lo, hi, seed):
    return np.random.Generator(np.random.PCG64(seed)).uniform(lo, hi, size=shape)


def target_shape(shape, center, r0, width=2.0, modes=(2, 3, 4), amp=0.03, seed=1003):
    """Seeded wobbly target phase field tanh((r*(theta) - r)/width) with
    r*(theta) = r0 (1 + sum_m a_m cos(m theta + p_m)), a_m ~ U(0, amp), p_m ~ U(0, 2 pi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.0, amp, size=len(modes))
    p = rng.uniform(0.0, 2.0 * math.pi, size=len(modes))
    _, y, x = grid(shape)
    dx, dy = x - center[0], y - center[1]
    r = np.sqrt(dx * dx + dy * dy)
    th = np.arctan2(dy, dx)
    rs = np.ones_like(r)
    for m, am, pm in zip(modes, a, p):
        rs = rs + am * np.cos(m * th + pm)
    return np.tanh((r0 * rs - r) / width)


# ----------------------------------------------------------------------------- workloads

def _base(Q, shape, **kw):
    p = {"Q": Q, "shape": tuple(shape), "rho_in": (1.0, 1.0), "tau": (1.0, 1.0),
         "sigma": 4.0 * 1e-3 / 9.0, "beta": 0.7, "phi": 1e-5, "sbar": 3.0, "gamma": 0.305,
         "site_rule": "grad"}
    p.update(kw)
    return p


def workload(name, shape=None, radius=None, phi=None, seed=None, ratio=None, offset=None):
    """Workload dict: params (lattice + physics), rho_r, rho_b, solid (or None),
    phi_field (or None), steps.  shape/radius downscale a workload; phi overrides the flux;
    offset = (ox, oy, oz) moves the drop centre of the drop workloads off the box centre (a
    centre on a node puts the saddles of the phase field between the drop and its periodic
    images on nodes, where the gradient vanishes inside a mixture and its direction, and so the
    recolouring angle, is rounding noise; half a node moves every such saddle between nodes).

    Names: 'drop2d' (D2Q9 128^2 drop R 32, |rho^N| < 0.5 site rule), 'flat2d' (D2Q9 1024^2
    flat interface between walls), 'ellipse2d' (D2Q9 1024^2 ellipse 200 x 120),
    'sphere3d' (D3Q19 256^3 sphere R 64), 'sessile3d' (D3Q19 384x384x192 cap on a wall,
    density ratio 10, space-dependent flux), 'adjoint2d' (D2Q9 512^2 drop R 96 with a
    seeded flux field and target shape), 'hemisphere3d' / 'hemisphere2d' (drop on a wall for
    the height-dependent flux, D3Q19 192^3 R 66 / D2Q9 384x192 R 66), 'contrast3d' (D3Q19
    192^3 drop R 44 at density ratio `ratio`, blue outlets on both z planes) and
    'contrast_flat3d' (D3Q19 160^3 film of height 80 on a wall at z = 0, 1, blue outlet on
    the top plane), 'cap3d' (D3Q19 192^3 cap pinned on a cylindrical cavity, ring radii
    50 / 53, height 8)."""
    ox, oy, oz = offset or (0.0, 0.0, 0.0)
    if name == "drop2d":
        shape = shape or (1, 128, 128)
        R = radius or 32.0 * shape[2] / 128.0
        p = _base(9, shape, site_rule="phase", gamma=0.5)
        d = sphere_distance(shape, (shape[2] / 2 + ox, shape[1] / 2 + oy, 0.0), R)
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": None, "phi_field": None,
             "steps": 2000, "radius": R}
    elif name == "flat2d":
        shape = shape or (1, 1024, 1024)
        ny = shape[1]
        p = _base(9, shape)
        d = flat_distance(shape, ny / 2.0, axis=1)
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        solid = wall_layers(shape, 1, [0, ny - 1])
        rr = np.where(solid == 1, 0.0, rr)
        rb = np.where(solid == 1, 0.0, rb)
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": solid, "phi_field": None,
             "steps": 20000, "height": ny / 2.0}
    elif name == "ellipse2d":
        shape = shape or (1, 1024, 1024)
        s = shape[2] / 1024.0
        p = _base(9, shape)
        d = ellipse_distance(shape, (shape[2] / 2, shape[1] / 2), 200.0 * s, 120.0 * s)
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": None, "phi_field": None,
             "steps": 20000}
    elif name == "sphere3d":
        shape = shape or (256, 256, 256)
        R = radius or 64.0 * shape[2] / 256.0
        p = _base(19, shape, sigma=4.0 * 5e-4 / 9.0)
        d = sphere_distance(shape, (shape[2] / 2 + ox, shape[1] / 2 + oy, shape[0] / 2 + oz), R)
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": None, "phi_field": None,
             "steps": 10000, "radius": R}
    elif name == "sessile3d":
        shape = shape or (192, 384, 384)
        nz, ny, nx = shape
        R = radius or 96.0 * nx / 384.0
        p = _base(19, shape, sigma=4.0 * 5e-4 / 9.0, rho_in=(1.0, 0.1), tau=(1.0, 0.6))
        d = sphere_distance(shape, (nx / 2 + ox, ny / 2 + oy, 0.5), R)
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        solid = wall_layers(shape, 0, [0, nz - 1])
        rr = np.where(solid == 1, 0.0, rr)
        rb = np.where(solid == 1, 0.0, rb)
        _, y, x = grid(shape)
        rxy = np.sqrt((x - nx / 2 - ox) ** 2 + (y - ny / 2 - oy) ** 2)
        ph = 1e-5 * (1.0 + 0.2 * rxy / R) + uniform_noise(shape, -1e-7, 1e-7,
                                                            1001 if seed is None else seed)
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": solid, "phi_field": ph,
             "steps": 20000, "radius": R}
    elif name == "adjoint2d":
        shape = shape or (1, 512, 512)
        s = shape[2] / 512.0
        R = radius or 96.0 * s
        p = _base(9, shape)
        c = (shape[2] / 2 + ox, shape[1] / 2 + oy, 0.0)
        d = sphere_distance(shape, c, R)
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        ph = 1e-5 * uniform_noise(shape, 0.9, 1.1, 1002 if seed is None else seed)
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": None, "phi_field": ph,
             "steps": 2000, "radius": R, "target": target_shape(shape, c, 90.0 * s),
             "ckpt_every": 100, "kappa": 0.01}
    elif name == "flat3d":
        # flat film on a wall (the paper's flat-interface benchmark in three dimensions):
        # red below z = nz/2, walls at z = 0 and nz - 1
        shape = shape or (128, 64, 64)
        nz = shape[0]
        p = _base(19, shape)
        d = flat_distance(shape, nz / 2.0, axis=0)
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        solid = wall_layers(shape, 0, [0, nz - 1])
        rr = np.where(solid == 1, 0.0, rr)
        rb = np.where(solid == 1, 0.0, rb)
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": solid, "phi_field": None,
             "height": nz / 2.0}
    elif name in ("hemisphere3d", "hemisphere2d"):
        # the height-dependent flux benchmark (Sec. III, space- and time-varying flux): a
        # hemispherical drop (half disc in 2D) on a neutrally wetting wall at index 0 of the
        # last lattice axis, unit density ratio, beta 0.99, sigma 0.1, unit relaxation times;
        # the flux field is computed from the drop height (phi_S 1e-3, K, h_s = R0)
        three = name == "hemisphere3d"
        shape = shape or ((192, 192, 192) if three else (1, 192, 384))
        nz, ny, nx = shape
        R = radius or (66.0 * nx / 192.0 if three else 66.0 * nx / 384.0)
        p = _base(19 if three else 9, shape, sigma=0.1, beta=0.99)
        centre = (nx / 2 + ox, ny / 2 + oy, 0.5) if three else (nx / 2 + ox, 0.5, 0.0)
        d = sphere_distance(shape, centre, R)
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        # walls at both ends of the substrate axis: with one wall layer and periodic wrap,
        # the wetting value under the drop would average the drop base with the far side
        solid = wall_layers(shape, 0 if three else 1, [0, (nz if three else ny) - 1])
        rr = np.where(solid == 1, 0.0, rr)
        rb = np.where(solid == 1, 0.0, rb)
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": solid,
             "phi_field": np.full(shape, p["phi"]), "radius": R, "phi_s": 1e-3,
             "h_scale": R}
    elif name in ("contrast3d", "contrast_flat3d"):
        # density contrast (Sec. III, density contrast): red initialised at gamma, blue at 1,
        # beta 0.99, sigma 0.1, unit relaxation times, phi = 3e-3; the blue component leaves
        # through pressure outlets (rho_b = 1) on the end planes of z during evaporation.
        # Gamma: 0.32 (gamma 2) and 0.33 (gamma 4) for the sphere.  For the film the paper
        # gives only |Gamma_flat - Gamma_sphere| = 0.02 and 0.04; the film takes the value
        # matched to the mass-loss rate over an evaporating run (calibrate_dynamic: 0.312 at
        # ratio 2, 0.311 at ratio 4, where the same procedure gives the drop 0.319 and 0.333)
        g = float(ratio or 2.0)
        flat = name == "contrast_flat3d"
        shape = shape or ((160, 160, 160) if flat else (192, 192, 192))
        nz, ny, nx = shape
        gsph = {2.0: 0.32, 4.0: 0.33}.get(g, 0.32)
        gam = {2.0: 0.312, 4.0: 0.311}.get(g, 0.312) if flat else gsph
        p = _base(19, shape, sigma=0.1, beta=0.99, rho_in=(g, 1.0), phi=3e-3, gamma=gam)
        if flat:
            # the wall is two layers thick (z = 0, 1; surface at z = 1.5): z = 0 is also the
            # periodic neighbour of the outlet plane, and with a single layer its wetting value
            # would average the film with the blue at the outlet, a false gradient under the film
            h0 = 80.0 * nz / 160.0
            d = flat_distance(shape, h0 + 1.5, axis=0)
            rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
            solid = wall_layers(shape, 0, [0, 1])
            rr = np.where(solid == 1, 0.0, rr)
            rb = np.where(solid == 1, 0.0, rb)
            w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": solid, "phi_field": None,
                 "height": h0, "outlet": (False, True)}
        else:
            R = radius or 44.0 * nx / 192.0
            d = sphere_distance(shape, (nx / 2 + ox, ny / 2 + oy, nz / 2 + oz), R)
            rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
            w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": None, "phi_field": None,
                 "radius": R, "outlet": (True, True)}
    elif name == "cap3d":
        # pinned spherical cap (Sec. III, pinned cap): a cylindrical cavity (a ring of solid
        # nodes, inner radius 50, outer radius 53, height 8) on the bottom wall, filled with
        # red, and a spherical cap on it whose edge sits on the ring's outer rim with a contact
        # angle of 120 degrees; unit density ratio, beta 0.99, sigma 0.1, tau 1, walls at both
        # ends of z.  Downscaled, the ring keeps a thickness of at least 1.5 nodes and a height
        # of at least 2; `radius` overrides the outer radius
        shape = shape or (192, 192, 192)
        nz, ny, nx = shape
        s = min(nx, ny) / 192.0
        r_out = radius or 53.0 * s
        r_in = r_out - max(3.0 * s, 1.5)
        H = max(int(round(8.0 * s)), 2)
        theta = math.radians(120.0)
        Rs = r_out / math.sin(theta)
        hc = Rs * (1.0 - math.cos(theta))
        top = H + 0.5  # the ring's top surface
        zc = top + hc - Rs
        p = _base(19, shape, sigma=0.1, beta=0.99)
        z, y, x = grid(shape)
        r = np.sqrt((x - nx / 2 - ox) ** 2 + (y - ny / 2 - oy) ** 2)
        dsph = Rs - np.sqrt(r * r + (z - zc) ** 2)
        d = np.where(z > top, dsph, np.where(r < r_in, np.maximum(dsph, r_in - r),
                                             np.minimum(dsph, r_out - r)))
        rr, rb = densities_from_distance(d, 2.0, p["rho_in"])
        ring = (z >= 1) & (z <= H) & (r >= r_in) & (r <= r_out)
        solid = np.where(ring, 1, wall_layers(shape, 0, [0, nz - 1])).astype(np.uint8)
        rr = np.where(solid == 1, 0.0, rr)
        rb = np.where(solid == 1, 0.0, rb)
        w = {"params": p, "rho_r": rr, "rho_b": rb, "solid": solid, "phi_field": None,
             "radius": r_out, "inner_radius": r_in, "cavity_height": H, "cavity_top": top,
             "cap_height": hc}
    else:
        raise KeyError(name)
    if phi is not None:
        w["params"]["phi"] = phi
        if w["phi_field"] is not None:
            w["phi_field"] = w["phi_field"] * (phi / 1e-5)
    return w
