"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact rational
identities of the lattice tables, moment identities, a textbook single-phase BGK step,
the viscosity law, polynomial exactness of the gradient stencil, conservation laws,
lattice symmetries, translation equivariance and the analytic recession laws of
Sec. III.A.  A plausible slip anywhere in the oracle (dropped term, wrong sign or index,
transposed operand) breaks at least one of them.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle.oracle import Oracle, tables
from paper_2412_14859_amd import inputs

# Textbook velocity sets and weights, typed here independently of the oracle.
TEXTBOOK = {
    9: ([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (1, 1, 0), (-1, -1, 0),
         (1, -1, 0), (-1, 1, 0)],
        [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4),
    19: ([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
          (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)],
         [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12),
}


def params(Q, shape, **kw):
    p = {"Q": Q, "shape": shape, "rho_in": (1.0, 1.0), "tau": (1.0, 1.0), "sigma": 0.01,
         "beta": 0.7, "phi": 0.0, "sbar": 3.0, "gamma": 0.305, "site_rule": "grad"}
    p.update(kw)
    return p


def unstream(f, c):
    """Post-collision values from post-streaming ones, periodic: f*_i(x) = f_i(x + c_i)."""
    out = np.empty_like(f)
    for i, (cx, cy, cz) in enumerate(c):
        out[:, i] = np.roll(f[:, i], shift=(-cz, -cy, -cx), axis=(1, 2, 3))
    return out


# ----------------------------------------------------------------------------- tables

@pytest.mark.parametrize("Q", [9, 19])
def test_tables_textbook_and_rational_identities(Q):
    t = tables(Q)
    cs, Ws = TEXTBOOK[Q]
    assert [tuple(v) for v in t["c"]] == cs
    assert np.allclose(t["W"], [float(w) for w in Ws], rtol=0, atol=1e-17)
    for i in range(Q):
        assert tuple(-t["c"][t["opp"][i]]) == tuple(t["c"][i])
    c = np.array(cs)
    W0 = Ws[0]
    # weights: isotropy of the 2nd and 4th moments with c_s^2 = 1/3
    for a in range(3 if Q == 19 else 2):
        for b in range(3 if Q == 19 else 2):
            m2 = sum(Ws[i] * c[i, a] * c[i, b] for i in range(Q))
            assert m2 == (Fraction(1, 3) if a == b else 0)
    m4 = sum(Ws[i] * c[i, 0] ** 2 * c[i, 1] ** 2 for i in range(Q))
    assert m4 == Fraction(1, 9)
    # rest weights t_i(alpha) = A_i + B_i alpha: exact identities for rational alpha
    A = [Fraction(0)] + [Ws[i] / (1 - W0) for i in range(1, Q)]
    B = [Fraction(1)] + [-A[i] for i in range(1, Q)]
    assert np.allclose(t["A"], [float(a) for a in A], rtol=0, atol=1e-16)
    assert np.allclose(t["B"], [float(b) for b in B], rtol=0, atol=1e-16)
    zeta = sum(A[i] * c[i, 0] ** 2 for i in range(Q))
    assert zeta == (Fraction(3, 5) if Q == 9 else Fraction(1, 2))
    assert abs(t["zeta"] - float(zeta)) < 1e-15
    assert zeta * (1 - W0) == Fraction(1, 3)       # Appendix A: zeta (1 - W_0) = c_s^2
    for alpha in (Fraction(0), W0, Fraction(14, 15), Fraction(2, 7)):
        tw = [A[i] + B[i] * alpha for i in range(Q)]
        assert sum(tw) == 1
        assert sum(tw[i] * c[i, 0] ** 2 for i in range(Q)) == zeta * (1 - alpha)
        assert sum(tw[i] * c[i, 0] * c[i, 1] for i in range(Q)) == 0
    assert [A[i] + B[i] * W0 for i in range(Q)] == Ws       # t_i(W_0) = W_i
    # published D3Q19 / D2Q9 rest weights of the generalized colour-gradient model
    a = Fraction(1, 4)
    tw = [A[i] + B[i] * a for i in range(Q)]
    if Q == 19:
        assert tw[1] == (1 - a) / 12 and tw[7] == (1 - a) / 24
    else:
        assert tw[1] == (1 - a) / 5 and tw[5] == (1 - a) / 20
    # perturbation constants: sum C = c_s^2, sum C c_a c_b = c_s^2 delta_ab
    Cc = t["C"]
    assert abs(Cc.sum() - 1 / 3) < 1e-15
    assert abs((Cc * c[:, 0] ** 2).sum() - 1 / 3) < 1e-15
    assert abs((Cc * c[:, 0] * c[:, 1]).sum()) < 1e-16


# ----------------------------------------------------------------------------- equilibrium

@pytest.mark.parametrize("Q,shape", [(9, (1, 6, 7)), (19, (4, 5, 6))])
def test_equilibrium_moments(Q, shape):
    rng = np.random.default_rng(7)
    D = 2 if Q == 9 else 3
    rho_in = (1.0, 0.1)
    o = Oracle(params(Q, shape, rho_in=rho_in))
    rr = rng.uniform(0.2, 1.0, shape)
    rb = rng.uniform(0.01, 0.1, shape)
    u = rng.uniform(-0.05, 0.05, (D,) + shape)
    o.init_equilibrium(rr, rb, u)
    f = o.populations()
    t = tables(Q)
    c = t["c"].astype(float)
    zeta = t["zeta"]
    alpha = (1 - (1 - t["W"][0]) / 10.0, t["W"][0])    # gamma_r = 10, blue least dense
    for k, rho in enumerate((rr, rb)):
        assert np.allclose(f[k].sum(0), rho, rtol=0, atol=1e-15)
        for a in range(D):
            ja = np.tensordot(c[:, a], f[k], axes=(0, 0))
            assert np.allclose(ja, rho * u[a], rtol=0, atol=1e-15)
            for b in range(D):
                pab = np.tensordot(c[:, a] * c[:, b], f[k], axes=(0, 0))
                ref = rho * u[a] * u[b] + (rho * zeta * (1 - alpha[k]) if a == b else 0.0)
                assert np.allclose(pab, ref, rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------- single phase

def textbook_bgk_step(f, tau, Q):
    """Single-component BGK step with the textbook equilibrium, then periodic streaming."""
    cs, Ws = TEXTBOOK[Q]
    c = np.array(cs, dtype=float)
    W = np.array([float(w) for w in Ws])
    rho = f.sum(0)
    u = np.tensordot(c.T, f, axes=(1, 0)) / rho
    uu = (u * u).sum(0)
    out = np.empty_like(f)
    for i in range(Q):
        cu = c[i, 0] * u[0] + c[i, 1] * u[1] + c[i, 2] * u[2]
        feq = W[i] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
        post = f[i] - (f[i] - feq) / tau
        out[i] = np.roll(post, shift=(cs[i][2], cs[i][1], cs[i][0]), axis=(0, 1, 2))
    return out


@pytest.mark.parametrize("Q,shape,tau", [(9, (1, 8, 10), 0.8), (19, (5, 6, 7), 1.3)])
def test_single_component_is_textbook_bgk(Q, shape, tau):
    rng = np.random.default_rng(11)
    D = 2 if Q == 9 else 3
    o = Oracle(params(Q, shape, tau=(tau, tau), phi=1e-3, sigma=0.1))
    rr = rng.uniform(0.9, 1.1, shape)
    u = rng.uniform(-0.03, 0.03, (D,) + shape)
    o.init_equilibrium(rr, np.zeros(shape), u)
    f = o.populations()
    f[0] += rng.uniform(-1e-3, 1e-3, f[0].shape)      # off-equilibrium start
    o.set_populations(f)
    o.recompute_fmag()
    ref = f[0].copy()
    for _ in range(3):
        o.step(1)
        ref = textbook_bgk_step(ref, tau, Q)
        g = o.populations()
        assert np.abs(g[1]).max() == 0.0
        assert np.allclose(g[0], ref, rtol=0, atol=2e-15)


def test_shear_wave_decay_gives_viscosity():
    # nu = c_s^2 (tau - 1/2) (Sec. II.A); sinusoidal shear wave decays as exp(-nu k^2 t)
    ny, tau, U = 64, 0.8, 1e-3
    shape = (1, ny, 4)
    o = Oracle(params(9, shape, tau=(tau, tau)))
    y = np.arange(ny, dtype=float)
    k = 2 * np.pi / ny
    u = np.zeros((2,) + shape)
    u[0] = U * np.sin(k * y)[None, :, None]
    o.init_equilibrium(np.ones(shape), np.zeros(shape), u)
    amps = []
    for t in (100, 300):
        o.step(t - (100 if amps else 0))
        ux = o.fields()["u"][0, 0, :, 0]
        amps.append((ux * np.sin(k * y)).sum() * 2 / ny)
    nu_meas = -np.log(amps[1] / amps[0]) / (k * k * 200)
    assert abs(nu_meas / ((tau - 0.5) / 3) - 1) < 5e-3


# ----------------------------------------------------------------------------- gradient

@pytest.mark.parametrize("Q,shape", [(9, (1, 12, 12)), (19, (10, 10, 10))])
def test_gradient_stencil_polynomial_exactness(Q, shape):
    z, y, x = inputs.grid(shape)
    xc, yc = x - shape[2] / 2, y - shape[1] / 2
    interior = (slice(2, -2) if shape[0] > 1 else slice(None), slice(2, -2), slice(2, -2))
    cases = [
        (0.03 * xc - 0.02 * yc, np.full(shape, np.hypot(0.03, 0.02))),       # linear
        (0.004 * xc ** 2, np.abs(0.008 * xc)),                                # quadratic
        (0.05 * xc + 0.002 * yc ** 2, np.sqrt(0.05 ** 2 + (0.004 * yc) ** 2)),  # mixed
        (1e-3 * xc ** 3, np.abs(3e-3 * xc ** 2 + 1e-3)),                     # cubic: +c_s^2-term
    ]
    for g, ref in cases:
        o = Oracle(params(Q, shape))
        o.init_equilibrium((1 + g) / 2, (1 - g) / 2)
        fl = o.fields()
        assert np.allclose(fl["rhoN"], g, rtol=0, atol=1e-15)
        assert np.allclose(fl["gradmag"][interior], ref[interior], rtol=1e-12, atol=1e-15)
        assert np.allclose(o.fmag()[interior], ref[interior], rtol=1e-12, atol=1e-15)


# ----------------------------------------------------------------------------- perturbation, recolouring

@pytest.mark.parametrize("n", [16, 64])
@pytest.mark.parametrize("Q,axis", [(9, 2), (9, 1), (19, 0)])
def test_perturbation_and_recolouring_moments(Q, axis, n):
    # n = 64 reaches the far tail of the profile, where ||F|| falls to 1e-11: Eq. recolor
    # holds there as everywhere (cos(theta) is cut only at F.F <= 1e-24)
    shape = [1, 16, 16] if Q == 9 else [16, 4, 4]
    shape[axis] = n
    shape = tuple(shape)
    sigma, beta, tau = 0.02, 0.7, 1.0
    coords = inputs.grid(shape)
    s = coords[axis] - shape[axis] / 2 + 0.3
    g = np.tanh(s / 2.5)
    rr, rb = (1 + g) / 2, (1 - g) / 2
    t = tables(Q)
    c = t["c"].astype(float)
    # the profile varies along `axis`: index into (x, y, z) of the lattice vectors
    a_n = {2: 0, 1: 1, 0: 2}[axis]
    for b in (0.0, beta):
        o = Oracle(params(Q, shape, sigma=sigma, beta=b))
        o.init_equilibrium(rr, rb)
        gm = o.fields()["gradmag"]
        o.step(1)
        fs = unstream(o.populations(), t["c"])
        f2 = fs[0] + fs[1]                             # colour-blind post-perturbation
        rho = rr + rb
        Wt = t["A"][:, None, None, None] + t["B"][:, None, None, None] * t["W"][0]
        delta = f2 - rho[None] * Wt                    # tau = 1: collision gives f^eq(rho, 0)
        assert np.allclose(delta.sum(0), 0, atol=1e-15)
        for a in range(3):
            assert np.allclose(np.tensordot(c[:, a], delta, axes=(0, 0)), 0, atol=1e-15)
            for bb in range(3):
                if Q == 9 and (a == 2 or bb == 2):
                    continue
                m = np.tensordot(c[:, a] * c[:, bb], delta, axes=(0, 0))
                nn = 1.0 if (a == a_n and bb == a_n) else 0.0
                ref = -(sigma / (2 * tau)) * gm * ((1.0 if a == bb else 0.0) - nn)
                assert np.allclose(m, ref, rtol=1e-12, atol=1e-15)
        # recolouring conserves each component and splits the colour-blind population (to the
        # rounding of a sum of Q terms of at most 1: Q ulp(1) / 2 < 2.2e-15)
        assert np.allclose(fs[0].sum(0), rr, rtol=0, atol=2.2e-15)
        assert np.allclose(fs[1].sum(0), rb, rtol=0, atol=2.2e-15)
        sep = fs[0] - (rr / rho)[None] * f2
        if b == 0.0:
            assert np.abs(sep).max() < 1e-15
        else:
            # red is pushed up its own gradient: momentum of the separation term along +F,
            # sum_i cos(theta_i) t_i c_i = n sum_i t_i (c_i.n)^2/|c_i|  (closed form)
            cn = np.sqrt((c ** 2).sum(1))
            k = sum(Wt[i, 0, 0, 0] * c[i, a_n] ** 2 / cn[i] for i in range(1, Q))
            dg = np.gradient(g, axis=axis)
            mom = np.tensordot(c[:, a_n], sep, axes=(0, 0))
            ref = b * rr * rb / rho * k * np.sign(dg) * (gm > 1e-12)
            inner = [slice(None)] * 3
            inner[axis] = slice(2, -2)                 # away from the periodic wrap's jump
            inner = tuple(inner)
            assert np.allclose(mom[inner], ref[inner], rtol=1e-12, atol=1e-15)


# ----------------------------------------------------------------------------- conservation

@pytest.mark.parametrize("case", ["drop_grad", "drop_phase", "walls_field"])
def test_mass_bookkeeping(case):
    if case == "walls_field":
        w = inputs.workload("flat2d", shape=(1, 40, 12))
        rng = np.random.default_rng(3)
        phi = rng.uniform(0.5e-3, 1.5e-3, w["rho_r"].shape)
        w["phi_field"] = phi
    else:
        w = inputs.workload("drop2d", shape=(1, 48, 48))
        if case == "drop_grad":
            w["params"].update(site_rule="grad", gamma=0.305)
        phi = np.full(w["rho_r"].shape, 1e-3)
    p = dict(w["params"], phi=1e-3)
    o = Oracle(p, solid=w["solid"], phi_field=w["phi_field"])
    o.init_equilibrium(w["rho_r"], w["rho_b"])
    ob0 = o.observables()
    m_tot0 = ob0["mass_r"] + ob0["mass_b"]
    prev = ob0["mass_r"]
    sink = 0.0
    for _ in range(30):
        mask = o.step(1, log_masks=True)[0]
        ob = o.observables()
        removed = (phi * mask).sum() / p["sbar"]
        sink += removed
        assert mask.sum() > 0
        assert abs((prev - ob["mass_r"]) - removed) < 1e-12 * ob0["mass_r"]
        assert abs(ob["mass_r"] + ob["mass_b"] - m_tot0) < 1e-12 * m_tot0
        prev = ob["mass_r"]
    assert abs(ob["sink_total"] - sink) < 1e-12 * sink
    # sink off: each component conserved
    o2 = Oracle(dict(p, phi=0.0), solid=w["solid"])
    o2.init_equilibrium(w["rho_r"], w["rho_b"])
    a = o2.observables()
    o2.step(30)
    b = o2.observables()
    assert abs(a["mass_r"] - b["mass_r"]) < 1e-12 * a["mass_r"]
    assert abs(a["mass_b"] - b["mass_b"]) < 1e-12 * a["mass_b"]


def test_momentum_conserved_with_sink():
    w = inputs.workload("drop2d", shape=(1, 40, 40))
    w["params"].update(phi=2e-3)
    o = Oracle(w["params"])
    rng = np.random.default_rng(5)
    u = rng.uniform(-0.01, 0.01, (2, 1, 40, 40))
    o.init_equilibrium(w["rho_r"], w["rho_b"], u)

    def momentum():
        f = o.populations()
        c = tables(9)["c"].astype(float)
        return np.array([np.tensordot(c[:, a], f.sum(0), axes=(0, 0)).sum() for a in range(2)])

    j0 = momentum()
    o.step(20)
    assert np.abs(momentum() - j0).max() < 1e-13


def test_translation_equivariance_bitwise():
    w = inputs.workload("drop2d", shape=(1, 32, 40), radius=9.0)
    p = dict(w["params"], site_rule="grad", gamma=0.305, phi=1e-3)
    runs = []
    for shift in ((0, 0), (5, 11)):
        o = Oracle(p)
        o.init_equilibrium(np.roll(w["rho_r"], shift, axis=(1, 2)),
                           np.roll(w["rho_b"], shift, axis=(1, 2)))
        o.step(12)
        runs.append(o.populations())
    assert np.array_equal(np.roll(runs[0], (5, 11), axis=(3, 4)), runs[1])


@pytest.mark.parametrize("Q", [9, 19])
def test_centred_drop_keeps_lattice_symmetry(Q):
    if Q == 9:
        w = inputs.workload("drop2d", shape=(1, 32, 32), radius=9.0)
    else:
        w = inputs.workload("sphere3d", shape=(16, 16, 16), radius=5.0)
    p = dict(w["params"], site_rule="grad", gamma=0.305, phi=1e-3)
    o = Oracle(p)
    o.init_equilibrium(w["rho_r"], w["rho_b"])
    o.step(15)
    rN = o.fields()["rhoN"]
    mirror = np.roll(rN[:, :, ::-1], 1, axis=2)            # x -> n - x
    assert np.abs(rN - mirror).max() < 1e-13
    assert np.abs(rN - np.swapaxes(rN, 1, 2)).max() < 1e-13  # x <-> y
    if Q == 19:
        assert np.abs(rN - np.swapaxes(rN, 0, 2)).max() < 1e-13


@pytest.mark.parametrize("Q", [9, 19])
def test_uniform_state_is_a_fixed_point(Q):
    shape = (1, 6, 5) if Q == 9 else (4, 5, 3)
    o = Oracle(params(Q, shape, phi=1e-3))
    o.init_equilibrium(np.full(shape, 0.7), np.full(shape, 0.3))
    f0 = o.populations()
    o.step(3)
    assert np.allclose(o.populations(), f0, rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------- physics laws

def test_laplace_pressure_jump_2d():
    # Young-Laplace in 2D: p_in - p_out = sigma / R, pressures from the EOS (Eq. EOS)
    sigma = 0.01
    Rs, dps = [], []
    for R in (12.0, 16.0, 20.0):
        w = inputs.workload("drop2d", shape=(1, 64, 64), radius=R)
        o = Oracle(dict(w["params"], sigma=sigma, phi=0.0))
        o.init_equilibrium(w["rho_r"], w["rho_b"])
        o.step(2500)
        ob = o.observables()
        fl = o.fields()
        Rs.append(np.sqrt((fl["rho_r"] / 1.0).sum() / np.pi))
        dps.append(ob["p_in"] - ob["p_out"])
    slope = np.polyfit(1.0 / np.array(Rs), np.array(dps), 1)[0]
    assert abs(slope / sigma - 1) < 0.05


def interface_height(rho_r):
    """Height where the column-averaged rho_r crosses half its maximum (linear interp.)."""
    prof = rho_r.mean(axis=(0, 2))
    half = 0.5 * prof.max()
    j = np.nonzero((prof[:-1] > half) & (prof[1:] <= half))[0][-1]
    return j + (prof[j] - half) / (prof[j] - prof[j + 1])


def test_flat_interface_recedes_at_phi_over_rho():
    # h(t) = h0 - phi t / rho0  (Sec. III.A.1); uncalibrated Gamma -> 10 % tolerance
    phi = 1e-3
    w = inputs.workload("flat2d", shape=(1, 96, 4), phi=phi)
    o = Oracle(w["params"], solid=w["solid"])
    o.init_equilibrium(w["rho_r"], w["rho_b"])
    o.step(500)
    h0 = interface_height(o.fields()["rho_r"])
    o.step(12000)
    h1 = interface_height(o.fields()["rho_r"])
    rate = (h0 - h1) / 12000
    assert abs(rate / phi - 1) < 0.10
    # sites per unit interface length close to Sbar = 3 (Sec. II.B)
    ob = o.observables()
    assert abs(ob["n_sites"] / 4 - 3) <= 1


def test_circle_radius_falls_linearly():
    # dR/dt = -phi / rho_l for a circle at unit density ratio (2D analogue of Eq. sphere_r)
    phi = 3e-3
    w = inputs.workload("drop2d", shape=(1, 72, 72), radius=24.0, phi=phi)
    p = dict(w["params"], site_rule="grad", gamma=0.305)
    o = Oracle(p)
    o.init_equilibrium(w["rho_r"], w["rho_b"])
    o.step(300)
    r0 = np.sqrt(o.observables()["v_mass"] / np.pi)
    o.step(3000)
    r1 = np.sqrt(o.observables()["v_mass"] / np.pi)
    rate = (r0 - r1) / 3000
    assert abs(rate / phi - 1) < 0.10


# ----------------------------------------------------------------------------- mixed nodes

# Rest weights of the generalized colour-gradient equilibrium, typed here from their published
# closed forms: t_0 = alpha, axis (1 - alpha)/5 (D2Q9) or /12 (D3Q19), diagonals /20 or /24.
def textbook_rest_weight(Q, i, alpha):
    n2 = sum(v * v for v in TEXTBOOK[Q][0][i])
    if n2 == 0:
        return alpha
    return (1 - alpha) / ((5 if n2 == 1 else 20) if Q == 9 else (12 if n2 == 1 else 24))


def component_alpha(Q, rho_in):
    """Appendix A: the least dense component takes W_0, the others 1 - (1 - W_0)/gamma_k."""
    W0 = float(TEXTBOOK[Q][1][0])
    rmin = min(rho_in)
    return [W0 if r == rmin else 1 - (1 - W0) / (r / rmin) for r in rho_in]


@pytest.mark.parametrize("Q,shape", [(9, (1, 7, 9)), (19, (5, 4, 6))])
def test_collision_of_a_mixed_node(Q, shape):
    """One collision of a uniform mixture at density ratio 10 (alpha_r = 1 - (1 - W_0)/10,
    alpha_b = W_0) with tau_r = 1, tau_b = 0.6, random velocities and an off-equilibrium
    shear part: the colour-blind post-collision population is
        f^eq_i(rho, u, abar) + (1 - omega) (f_i - f^eq_i),
        rho t_i(abar) = sum_k rho_k t_i(alpha_k),   omega = sum_k (rho_k / rho) / tau_k
    (Sec. II.A: the density-weighted alpha of the equilibrium and the harmonic relaxation time)
    and red keeps its share rho_r / rho of it (the phase field is uniform, so F = 0: no
    perturbation, no recolouring).  An arithmetic mean of tau, an unweighted or swapped
    weighting of alpha, or a dropped velocity term moves the result by 1e-5 or more."""
    rng = np.random.default_rng(17)
    D = 2 if Q == 9 else 3
    rho_in, tau = (1.0, 0.1), (1.0, 0.6)
    cs = np.array(TEXTBOOK[Q][0], dtype=float)
    W = np.array([float(w) for w in TEXTBOOK[Q][1]])
    a_r, a_b = component_alpha(Q, rho_in)
    rr, rb = np.full(shape, 0.6), np.full(shape, 0.04)
    u = rng.uniform(-0.04, 0.04, (D,) + shape)
    o = Oracle(params(Q, shape, rho_in=rho_in, tau=tau, sigma=0.05, phi=0.0))
    o.init_equilibrium(rr, rb, u)
    f = o.populations()
    # an off-equilibrium part with no mass and no momentum: the shear mode c_x c_y and the
    # normal-stress mode c_x^2 - c_y^2, added to red only (each component keeps its mass)
    g = rng.uniform(-1e-3, 1e-3, (2,) + shape)
    f[0] += (cs[:, 0] * cs[:, 1])[:, None, None, None] * g[0] + \
        (cs[:, 0] ** 2 - cs[:, 1] ** 2)[:, None, None, None] * g[1]
    o.set_populations(f)
    o.recompute_fmag()
    o.step(1)
    post = unstream(o.populations(), [tuple(int(v) for v in ci) for ci in cs])
    rho = rr + rb
    fcb = f[0] + f[1]
    uu = (u * u).sum(0)
    omega = (rr / rho) / tau[0] + (rb / rho) / tau[1]
    for i in range(Q):
        cu = sum(cs[i, a] * u[a] for a in range(D))
        feq = rr * textbook_rest_weight(Q, i, a_r) + rb * textbook_rest_weight(Q, i, a_b) + \
            rho * W[i] * (3 * cu + 4.5 * cu * cu - 1.5 * uu)
        ref = feq + (1 - omega) * (fcb[i] - feq)
        # a few ulps of values below 1
        assert np.allclose(post[0, i] + post[1, i], ref, rtol=0, atol=1e-15), i
        assert np.allclose(post[0, i], (rr / rho) * ref, rtol=0, atol=1e-15), i


def test_shear_wave_of_a_mixture_decays_with_the_harmonic_tau():
    """A uniform mixture (rho_r / rho = 0.3) with tau_r = 1, tau_b = 0.6: its shear wave decays
    at nu = c_s^2 (tau_eff - 1/2) with 1/tau_eff = sum_k (rho_k / rho) / tau_k (Sec. II.A),
    i.e. tau_eff = 0.682; the arithmetic mean 0.72 would give a 21 % larger rate."""
    ny, U = 64, 1e-3
    shape = (1, ny, 4)
    tau = (1.0, 0.6)
    o = Oracle(params(9, shape, tau=tau))
    y = np.arange(ny, dtype=float)
    k = 2 * np.pi / ny
    u = np.zeros((2,) + shape)
    u[0] = U * np.sin(k * y)[None, :, None]
    o.init_equilibrium(np.full(shape, 0.3), np.full(shape, 0.7), u)
    amps = []
    for t in (100, 300):
        o.step(t - (100 if amps else 0))
        ux = o.fields()["u"][0, 0, :, 0]
        amps.append((ux * np.sin(k * y)).sum() * 2 / ny)
    nu_meas = -np.log(amps[1] / amps[0]) / (k * k * 200)
    tau_eff = 1.0 / (0.3 / tau[0] + 0.7 / tau[1])
    assert abs(nu_meas / ((tau_eff - 0.5) / 3) - 1) < 5e-3


# ----------------------------------------------------------------------------- walls

def _contact_angle(rhoN, wall_surface=0.5, first_row=3):
    """Contact angle (degrees, through the red) of a half disc on the wall y = 0: a circle
    fitted (least squares) to the rho^N = 0 contour away from the wall, theta = arccos of
    minus the height of its centre above the wall surface over its radius."""
    ny, nx = rhoN.shape
    pts = []
    for y in range(first_row, ny - 1):
        row = rhoN[y]
        for x in range(nx - 1):
            if (row[x] > 0) != (row[x + 1] > 0):
                pts.append((x + row[x] / (row[x] - row[x + 1]), y))
    for x in range(nx):
        col = rhoN[:, x]
        for y in range(first_row, ny - 2):
            if (col[y] > 0) != (col[y + 1] > 0):
                pts.append((x, y + col[y] / (col[y] - col[y + 1])))
    P = np.array(pts)
    A = np.c_[2 * P[:, 0], 2 * P[:, 1], np.ones(len(P))]
    cx, cy, c = np.linalg.lstsq(A, (P ** 2).sum(1), rcond=None)[0]
    return float(np.degrees(np.arccos(-(cy - wall_surface) / np.sqrt(c + cx * cx + cy * cy))))


def test_neutral_wall_keeps_a_90_degree_contact_angle():
    """Neutral wetting (Sec. III, walls): a half disc (R = 20) on a wall relaxes to a contact
    angle of 90 degrees (measured 89.8) at unit density ratio; a wall value biased towards one
    colour (e.g. the red fraction in place of rho^N) tilts it by degrees."""
    w = inputs.workload("hemisphere2d", shape=(1, 48, 96), radius=20.0, offset=(0.5, 0, 0))
    o = Oracle(dict(w["params"], phi=0.0), solid=w["solid"])
    o.init_equilibrium(w["rho_r"], w["rho_b"])
    o.step(4000)
    theta = _contact_angle(o.fields()["rhoN"][0])
    assert abs(theta - 90.0) < 1.0, theta


def test_wall_thickness_does_not_change_the_fluid():
    """A solid node's wetting value comes from its fluid neighbours only, and a fluid node
    reads only its nearest neighbours: a drop on a wall evolves bitwise the same between
    walls two and three layers thick (the box grows by the extra layers, so the fluid rows
    are the same), with the sink on."""
    runs = []
    for layers in (2, 3):
        ny = 26 + 2 * layers
        shape = (1, ny, 40)
        d = inputs.sphere_distance(shape, (20.5, layers - 0.5, 0.0), 9.0)
        rr, rb = inputs.densities_from_distance(d, 2.0, (1.0, 1.0))
        solid = inputs.wall_layers(shape, 1, list(range(layers)) +
                                   list(range(ny - layers, ny)))
        rr = np.where(solid == 1, 0.0, rr)
        rb = np.where(solid == 1, 0.0, rb)
        o = Oracle(params(9, shape, phi=1e-3, sigma=0.01), solid=solid)
        o.init_equilibrium(rr, rb)
        o.step(40)
        runs.append(o.populations()[:, :, :, layers:ny - layers, :])
    assert np.array_equal(runs[0], runs[1])


def test_threads_do_not_change_the_oracle():
    """The per-node loops may run on several threads (the CPU baseline's mode): the same bits
    as one thread, observables included."""
    w = inputs.workload("sessile3d", shape=(12, 14, 18), radius=5.0, phi=1e-3)
    runs = []
    for t in (1, 4):
        o = Oracle(w["params"], solid=w["solid"], phi_field=w["phi_field"])
        o.set_threads(t)
        o.init_equilibrium(w["rho_r"], w["rho_b"])
        o.step(6)
        runs.append((o.populations(), o.observables()))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1] == runs[1][1]
