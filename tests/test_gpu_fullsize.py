"""Parity at the full workload sizes, in the step form the benchmark times (the automatic
choice), on sampled nodes.

One node's post-collision values depend only on its own pre-sink state and site data and on
rho^N at its neighbours (whose values depend only on their own state; with walls, a solid
neighbour takes the wetting mean over its own fluid neighbours).  So the FP64 oracle run for
one step on a small periodic box cut out around the node (3 nodes wide, 5 with walls) from the
GPU's exported state computes the node's outputs exactly.  They are compared with the GPU's
step on the whole domain: FP64 within 1e-12, FP32 storage within 1e-6 (one rounding of the
stored value) and FP16 storage within 5e-3, relative to t_i(alpha_k) rho_k^in."""
import numpy as np
import pytest

from oracle.oracle import Oracle, tables
from tests.helpers import case, gpu_for, pop_scale

pytestmark = [pytest.mark.gpu]

CASES = {
    # name: (workload, overrides, precision, tolerance)
    "sphere3d_256_fp32s": ("sphere3d", {}, "fp32s", 1e-6),
    "sphere3d_256_fp64": ("sphere3d", {}, "fp64", 1e-12),
    "sphere3d_256_fp16s": ("sphere3d", {}, "fp16s", 5e-3),
    "flat2d_1024_fp64": ("flat2d", {}, "fp64", 1e-12),
    "flat2d_1024_fp32s": ("flat2d", {}, "fp32s", 1e-6),
    "ellipse2d_1024_fp32s": ("ellipse2d", {}, "fp32s", 1e-6),
    "sessile3d_fp32s": ("sessile3d", {}, "fp32s", 1e-6),
    "adjoint2d_512_soft_fp32s": ("adjoint2d", {"site_rule": "soft", "kappa": 0.01}, "fp32s", 1e-6),
    "drop2d_128_phase_fp64": ("drop2d", {}, "fp64", 1e-12),
    # the pinned-cap cavity (ring of solid nodes on the bottom wall), 192^3
    "cap3d_192_fp64": ("cap3d", {}, "fp64", 1e-12),
    "cap3d_192_fp32s": ("cap3d", {}, "fp32s", 1e-6),
    # density ratio 2 with blue outlets on the end planes of z (drop 192^3; film 160^3 on a
    # wall with the outlet on top)
    "contrast3d_192_fp32s": ("contrast3d", {}, "fp32s", 1e-6),
    "contrast_flat3d_160_fp64": ("contrast_flat3d", {}, "fp64", 1e-12),
}


def _flush(msg):
    print(msg, flush=True)


def _samples(carry, solid, rng, k=24, zlim=None):
    """Seeded nodes: half at sites (or largest soft weights), half anywhere in the fluid;
    with zlim = (lo, hi) only planes lo <= z <= hi."""
    fluid = np.ones(carry.shape, bool) if solid is None else solid == 0
    if zlim is not None:
        zs = np.arange(carry.shape[0])[:, None, None]
        fluid = fluid & (zs >= zlim[0]) & (zs <= zlim[1])
    if carry.dtype == np.uint8:
        hot = np.argwhere((carry > 0) & fluid)
    else:  # soft rule: carried ||F||, take the interface
        hot = np.argwhere((carry > 0.05) & fluid)
    anyw = np.argwhere(fluid)
    pick = [] if len(hot) == 0 else \
        [hot[i] for i in rng.choice(len(hot), size=min(k // 2, len(hot)), replace=False)]
    pick += [anyw[i] for i in rng.choice(len(anyw), size=k - len(pick), replace=False)]
    return [tuple(int(v) for v in p) for p in pick]


def _box(shape, node, h, D):
    """Periodic index vectors of the box of half-width h around node (z, y, x)."""
    out = []
    for a, (n, c) in enumerate(zip(shape, node)):
        if D == 2 and a == 0:
            out.append(np.array([c]))
        else:
            out.append(np.arange(c - h, c + h + 1) % n)
    return out


def _center_outputs(f, centre, solid_box, c, opp):
    """Post-collision values computed at the box centre, read from a post-step state:
    direction i went to centre + c_i, or bounced back into the centre as opp(i)."""
    Q = c.shape[0]
    cz, cy, cx = centre
    out = np.empty((2, Q))
    for i in range(Q):
        z, y, x = cz + c[i, 2], cy + c[i, 1], cx + c[i, 0]
        if solid_box is not None and solid_box[z, y, x]:
            out[:, i] = f[:, opp[i], cz, cy, cx]
        else:
            out[:, i] = f[:, i, z, y, x]
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_sampled_nodes_match_the_oracle_at_full_size(name):
    import torch
    wl, over, precision, tol = CASES[name]
    w = case(wl, None, **over)
    p = w["params"]
    Q = int(p["Q"])
    D = 2 if Q == 9 else 3
    t = tables(Q)
    c, opp = np.asarray(t["c"]), np.asarray(t["opp"])
    scale = pop_scale(Q, p["rho_in"])
    walls = w["solid"] is not None
    h = 2 if walls else 1
    _flush(f"[full size] {name} shape={p['shape']} {precision}")
    sim = gpu_for(w, precision)
    zlim = None
    if w.get("outlet"):
        # the outlet fix-up writes slots on the end planes that only the outlet nodes read:
        # boxes stay clear of them
        sim.set_outlet(*w["outlet"], 1.0)
        zlim = (h + 1, p["shape"][0] - h - 2)
    kernel = sim.kernel_name()
    sim.step(10)
    rng = np.random.default_rng(2412)
    carry = sim.carry.cpu().numpy()
    nodes = _samples(carry, w["solid"], rng, zlim=zlim)
    f0 = sim.populations()
    boxes = []
    for node in nodes:
        iz, iy, ix = _box(p["shape"], node, h, D)
        tz, ty, tx = (torch.as_tensor(v, device=f0.device) for v in (iz, iy, ix))
        fb = f0[:, :, tz[:, None, None], ty[None, :, None], tx[None, None, :]].cpu().numpy()
        sel = np.ix_(iz, iy, ix)
        boxes.append((node, fb, carry[sel], None if not walls else w["solid"][sel],
                      None if w["phi_field"] is None else w["phi_field"][sel]))
    del f0
    sim.step(1)
    f1 = sim.populations()
    worst = 0.0
    for node, fb, cb, sb, phib in boxes:
        bp = dict(p, shape=fb.shape[2:])
        ora = Oracle(bp, solid=sb, phi_field=phib)
        ora.set_populations(fb)
        if p.get("site_rule", "grad") == "soft":
            ora.set_fmag(cb)
            ora.step(1)
        elif p.get("site_rule", "grad") == "grad":
            ora.step(1, masks=cb[None].astype(np.uint8))
        else:  # |rho^N| < Gamma uses the current state, which the box holds
            ora.step(1)
        centre = tuple(v // 2 for v in fb.shape[2:])
        if D == 2:
            centre = (0,) + centre[1:]
        want = _center_outputs(ora.populations(), centre, sb, c, opp)
        # the same entries of the GPU's post-step state
        iz, iy, ix = _box(p["shape"], node, h, D)
        tz, ty, tx = (torch.as_tensor(v, device=f1.device) for v in (iz, iy, ix))
        gb = f1[:, :, tz[:, None, None], ty[None, :, None], tx[None, None, :]].cpu().numpy()
        got = _center_outputs(gb, centre, sb, c, opp)
        e = float(np.max(np.abs(got - want) / scale))
        worst = max(worst, e)
        assert e < tol, (name, node, e)
    _flush(f"  {kernel}: {len(boxes)} nodes, worst e_pop {worst:.3e}")
    sim.close()
    del sim, f1
    torch.cuda.empty_cache()


@pytest.mark.parametrize("site_rule,precision,tol", [("grad", "fp64", 1e-11),
                                                     ("grad", "fp32s", 1e-11),
                                                     ("soft", "fp32s", None)])
def test_full_size_adjoint_mass_covectors(site_rule, precision, tol):
    """The adjoint workload at full size (D2Q9 512^2 drop, checkpoints every 100 steps over
    2000 steps), checked through properties that hold at any size.
    * L = final total mass (dL/drho = 1): every operator conserves it, so dL/dphi = 0.
    * Hard sites, L = final red mass (dL/drho^N = rho/2, dL/drho = (1 + rho^N)/2): every
      operator but the sink conserves red mass, so the per-step gradient is exactly
      dL/dphi(x, t) = -m(x, t)/Sbar, i.e. the values 0 and -1/Sbar at exactly the site-steps of
      the run, and sum_x phi(x) dL/dphi(x) is minus the mass the sink removed (the forward's
      FP64 bookkeeping).  The adjoint is the exact transpose of the step at the stored
      trajectory, so this holds to rounding at every storage precision.  With soft sites the
      weights depend on the state, so phi also acts through later weights and these
      identities do not hold."""
    import torch
    w = case("adjoint2d", None, site_rule=site_rule, kappa=0.01)
    p = w["params"]
    nsteps, K = 2000, 100
    _flush(f"[full-size adjoint] adjoint2d 512^2 {site_rule} {precision} n={nsteps} K={K}")
    sim = gpu_for(w, precision)
    ck = sim.forward_ckpt(nsteps, K)
    obs = sim.observables()
    fl = sim.fields()
    rho = fl["rho_r"] + fl["rho_b"]
    r0 = sim.backward(ck, nsteps, K, dL_drho=torch.ones_like(rho))
    z = float(r0["grad_phi"].abs().max())
    _flush(f"  total-mass covector: max |dL/dphi| = {z:.2e}")
    assert z < 1e-10 / p["sbar"]
    if site_rule == "grad":
        r = sim.backward(ck, nsteps, K, dL_drhoN=rho / 2, dL_drho=(1 + fl["rhoN"]) / 2,
                         per_step=True)
        phi = sim.phi_field.to(torch.float64)
        lhs = float((phi * r["grad_phi"]).sum())
        rel = abs(lhs + obs["sink_total"]) / obs["sink_total"]
        _flush(f"  sum phi dL/dphi = {lhs:.12e}, sink total {obs['sink_total']:.12e}, "
               f"rel {rel:.2e}")
        assert obs["sink_total"] > 0 and rel < tol
        g = r["grad_phi_t"]
        inv = 1.0 / p["sbar"]
        at_site = (g + inv).abs() < tol * inv
        assert bool(((g.abs() < tol * inv) | at_site).all())
        assert int(at_site.sum()) == obs["site_steps"]
        del g, at_site
    sim.close()
    torch.cuda.empty_cache()


def test_full_size_adjoint_central_differences():
    """The adjoint workload at full size with soft sites (D2Q9 512^2, 2000 steps, K = 100, the
    shape loss L = sum (rho^N_T - target)^2), FP64: the adjoint's directional derivatives along
    a seeded direction of phi(x) and along Gamma against central differences of the GPU's own
    forward runs (relative step 1e-3)."""
    import torch
    w = case("adjoint2d", None, site_rule="soft", kappa=0.01)
    p = w["params"]
    nsteps, K = 2000, 100
    target = torch.as_tensor(w["target"])
    _flush("[full-size adjoint FD] adjoint2d 512^2 soft fp64")
    sim = gpu_for(w, "fp64")
    start = sim.save_state().clone()
    dev = sim.device
    tgt = target.to(dev)
    ck = sim.forward_ckpt(nsteps, K)
    rn = sim.fields()["rhoN"]
    r = sim.backward(ck, nsteps, K, dL_drhoN=2.0 * (rn - tgt))
    phi0 = sim.phi_field.clone()

    def loss(phi, gamma):
        sim.phi_field.copy_(phi)
        sim.set_site_threshold(gamma)
        sim.load_state(start)
        sim.set_counters()
        sim.step(nsteps)
        v = float(((sim.fields()["rhoN"] - tgt) ** 2).sum())
        sim.phi_field.copy_(phi0)
        sim.set_site_threshold(p["gamma"])
        return v

    gen = torch.Generator(device="cpu").manual_seed(1004)
    v = (torch.randn(phi0.shape, generator=gen, dtype=torch.float64).to(dev) * phi0)
    ad = float((r["grad_phi"] * v).sum())
    eps = 1e-3
    fd = (loss(phi0 + eps * v, p["gamma"]) - loss(phi0 - eps * v, p["gamma"])) / (2 * eps)
    _flush(f"  phi: adjoint {ad:.10e} fd {fd:.10e}")
    assert abs(fd - ad) <= 1e-4 * abs(ad)
    eg = 1e-3 * p["gamma"]
    fdg = (loss(phi0, p["gamma"] + eg) - loss(phi0, p["gamma"] - eg)) / (2 * eg)
    _flush(f"  Gamma: adjoint {r['grad_gamma']:.10e} fd {fdg:.10e}")
    assert abs(fdg - r["grad_gamma"]) <= 1e-3 * abs(r["grad_gamma"])
    sim.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name,precision,tol", [("sphere3d", "fp32s", 1e-6),
                                                ("sphere3d", "fp64", 1e-13),
                                                ("cap3d", "fp32s", 1e-6)])
def test_record_calls_equal_split_steps_at_full_size(name, precision, tol):
    """The benchmark runs the record form (the automatic choice at unit relaxation times) in
    calls of many steps, whose intermediate states never leave the library.  At the full
    size, a call of 6 steps equals 6 split steps (which the sampled test above pins to the
    oracle) within the rounding of the record, with identical site data in FP64."""
    import torch
    from tests.helpers import e_pop
    w = case(name, None)
    p = w["params"]
    _flush(f"[full size record vs split] {name} shape={p['shape']} {precision}")
    a = gpu_for(w, precision)
    assert a.kernel_name() == "k_pull_record"
    a.step(6)
    fa = a.populations().cpu().numpy()
    ca = a.carry.cpu().numpy()
    oa = a.observables()
    a.close()
    del a
    torch.cuda.empty_cache()
    b = gpu_for(w, precision, kernel="split")
    b.step(6)
    fb = b.populations().cpu().numpy()
    cb = b.carry.cpu().numpy()
    ob = b.observables()
    b.close()
    del b
    torch.cuda.empty_cache()
    e = e_pop(fa, fb, int(p["Q"]), p["rho_in"], w["solid"])
    _flush(f"  e_pop(record, split) = {e:.3e}")
    assert e < tol, e
    if precision == "fp64":
        assert np.array_equal(ca, cb)
        assert oa["site_steps"] == ob["site_steps"]
    assert abs(oa["sink_total"] - ob["sink_total"]) <= 1e-9 * abs(ob["sink_total"])
