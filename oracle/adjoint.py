"""Differentiable FP64 CPU reference of the colour-gradient step with reaction-limited
evaporation, and its gradients by reverse-mode automatic differentiation.

TEST INFRASTRUCTURE ONLY: the test suite uses it to check the GPU adjoint.  It is written in
plain PyTorch CPU operations (float64), independently of the C oracle and of the HIP path, and
is itself pinned against the C oracle's forward step, central finite differences, and the
exact red-mass sensitivity of the sink (tests/test_adjoint_oracle.py).

The step, in the order of the method summary at the end of Sec. II.B (periodic domains,
optionally with solid nodes):
  sink s = m phi / Sbar at site weight m (Eq. relation, Eq. exchange): f0^r -= s, f0^b += s
  moments rho_k, rho, u, rho^N (Sec. II.A)
  colour gradient F = (1/c_s^2) sum_i W_i rho^N(x + c_i) c_i (Eq. cg)
  BGK with harmonic tau and alpha-equilibrium (Eqs. collision, feq)
  perturbation (Eq. perturb), recolouring (Eq. recolor)
  streaming (Eq. Stream)
with the readings used throughout: t_i(a) = A_i + B_i a, C_0 = c_s^2 - (1 - W_0), C_i = W_i;
cos(theta_i) = F.c_i / (|F| |c_i|) and the perturbation taken as 0 where F.F <= 1e-24 (their
limit at F = 0); cos(theta_0) = 0; the optional regularisation params['recolor_fade'] = w > 0
(off by default, not the paper's model) multiplies cos(theta_i) by clamp(|F|/w - 1, 0, 1),
as the C oracle does.  Solid nodes (Sec. III,
walls) carry no populations: streaming bounces back halfway from them, and in the gradient
stencil a solid node takes the W-weighted mean of rho^N over its fluid neighbours (neutral
wetting); the sink acts at fluid nodes only.

Site weights: 'hard' masks are given per step (taken from a forward run; the threshold has
zero derivative almost everywhere, so the sites are held fixed); 'soft' weights are the
logistic function of (||F_{n-1}|| - Gamma) / kappa, differentiable in Gamma and in the state.
"""
import torch

DT = torch.float64


def lattice(Q):
    """Directions, weights and derived constants of D2Q9 / D3Q19 (canonical order)."""
    if Q == 9:
        c = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
             (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0)]
        w = {0: 4.0 / 9.0, 1: 1.0 / 9.0, 2: 1.0 / 36.0}
    elif Q == 19:
        c = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
        for a, b in ((0, 1), (0, 2), (1, 2)):
            for sa, sb in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
                v = [0, 0, 0]
                v[a], v[b] = sa, sb
                c.append(tuple(v))
        w = {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}
    else:
        raise ValueError(Q)
    n2 = [sum(x * x for x in ci) for ci in c]
    W = torch.tensor([w[k] for k in n2], dtype=DT)
    cs2 = 1.0 / 3.0
    A = torch.where(torch.arange(Q) == 0, torch.zeros(Q, dtype=DT), W / (1.0 - W[0]))
    B = torch.where(torch.arange(Q) == 0, torch.ones(Q, dtype=DT), -A)
    C = W.clone()
    C[0] = cs2 - (1.0 - W[0])
    clen = torch.tensor([x ** 0.5 for x in n2], dtype=DT)
    return {"Q": Q, "c": c, "ct": torch.tensor(c, dtype=DT), "W": W, "A": A, "B": B, "C": C,
            "cs2": cs2, "clen": clen}


def alphas(W0, rho_in):
    rmin = min(rho_in)
    return [W0 if r == rmin else 1.0 - (1.0 - W0) / (r / rmin) for r in rho_in]


def shift(a, c, sign):
    """a(x - sign * c) for a field a[..., z, y, x] (periodic): sign=+1 pulls from x - c."""
    return torch.roll(a, shifts=(sign * c[2], sign * c[1], sign * c[0]), dims=(-3, -2, -1))


def opposite(Q):
    """opp(0) = 0; opp(i) = i + 1 for odd i, i - 1 for even i >= 2 (canonical order)."""
    return [0] + [i + 1 if i % 2 else i - 1 for i in range(1, Q)]


def wetted(L, rhoN, solid):
    """rho^N with the neutral-wetting value at solid nodes (fluid values unchanged)."""
    if solid is None:
        return rhoN
    fl = (~solid).to(DT)
    num = torch.zeros_like(rhoN)
    den = torch.zeros_like(rhoN)
    for i, ci in enumerate(L["c"]):
        if i == 0:
            continue
        num = num + L["W"][i] * shift(fl * rhoN, ci, -1)
        den = den + L["W"][i] * shift(fl, ci, -1)
    wet = num / torch.where(den > 0, den, torch.ones_like(den))
    return torch.where(solid, wet, rhoN)


def phase_gradient(L, rhoN):
    F = []
    for a in range(3):
        acc = torch.zeros_like(rhoN)
        for i, ci in enumerate(L["c"]):
            if ci[a]:
                acc = acc + L["W"][i] * ci[a] * shift(rhoN, ci, -1)
        F.append(acc / L["cs2"])
    return F


def phase_field(f, solid=None):
    """rho^N of the fluid nodes (0 at solid nodes)."""
    rr, rb = f[0].sum(0), f[1].sum(0)
    if solid is None:
        return (rr - rb) / (rr + rb)
    rho = rr + rb
    return torch.where(solid, torch.zeros_like(rr),
                       (rr - rb) / torch.where(solid, torch.ones_like(rho), rho))


def step(L, p, f, fprev, phi, weight, stored=None, solid=None):
    """One step.  f: [2, Q, nz, ny, nx] pre-sink state; fprev: ||F_{n-1}|| [nz, ny, nx];
    phi: flux field of this step; weight: site weights m.  Returns (next state, ||F_n||).
    stored: optional function of the post-sink moments (rho, [j_x, j_y, j_z], rho^N) returning
    the values the rest of the step uses instead (a test uses it to reproduce a storage
    rounding); by default they are used as computed.  solid: optional bool [nz, ny, nx]."""
    Q = L["Q"]
    s = weight * phi / p["sbar"]
    if solid is not None:
        s = torch.where(solid, torch.zeros_like(s), s)
    fr = torch.cat([(f[0, 0] - s)[None], f[0, 1:]])
    fb = torch.cat([(f[1, 0] + s)[None], f[1, 1:]])
    rr, rb = fr.sum(0), fb.sum(0)
    rho = rr + rb
    if solid is not None:  # solid nodes hold nothing; keep the quotients finite there
        rho = torch.where(solid, torch.ones_like(rho), rho)
    fcb = fr + fb
    j = [sum(L["c"][i][a] * fcb[i] for i in range(Q) if L["c"][i][a]) for a in range(3)]
    rhoN = (rr - rb) / rho
    if stored is not None:
        rho, j, rhoN = stored(rho, j, rhoN)
        rr, rb = rho * (1.0 + rhoN) / 2.0, rho * (1.0 - rhoN) / 2.0
    u = [j[a] / rho for a in range(3)]
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    F = phase_gradient(L, wetted(L, rhoN, solid))
    F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2]
    # ||F|| itself (carried to the next step's site weight) is exact; the perturbation and
    # cos(theta) are 0/0 forms at F = 0 and are cut where F.F <= 1e-24
    nz = F2 > 0
    Fn = torch.where(nz, torch.sqrt(torch.where(nz, F2, torch.ones_like(F2))),
                     torch.zeros_like(F2))
    pos = F2 > 1e-24
    Fp = torch.where(pos, Fn, torch.zeros_like(Fn))
    invFn = torch.where(pos, 1.0 / torch.where(pos, Fn, torch.ones_like(Fn)), torch.zeros_like(Fn))
    w = p.get("recolor_fade", 0.0)
    fade = torch.clamp(Fn / w - 1.0, 0.0, 1.0) if w > 0 else torch.ones_like(Fn)
    a_r, a_b = alphas(float(L["W"][0]), p["rho_in"])
    inv_tau = (rr / rho) / p["tau"][0] + (rb / rho) / p["tau"][1]
    abar = (rr / rho) * a_r + (rb / rho) * a_b
    out_r, out_b = [], []
    for i in range(Q):
        ci = L["c"][i]
        cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2]
        t_i = L["A"][i] + L["B"][i] * abar
        feq = rho * (t_i + L["W"][i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu))
        f1 = fcb[i] - inv_tau * (fcb[i] - feq)
        Fc = ci[0] * F[0] + ci[1] * F[1] + ci[2] * F[2]
        f1 = f1 + 2.25 * p["sigma"] * inv_tau * (L["W"][i] * Fc * Fc * invFn - L["C"][i] * Fp)
        cos = Fc * invFn * fade / L["clen"][i] if i != 0 else torch.zeros_like(Fc)
        sep = p["beta"] * rr * rb / (rho * rho) * cos * rho * t_i
        out_r.append(rr / rho * f1 + sep)
        out_b.append(rb / rho * f1 - sep)
    post = torch.stack([torch.stack(out_r), torch.stack(out_b)])
    if solid is None:
        nxt = torch.stack([torch.stack([shift(post[k, i], L["c"][i], +1) for i in range(Q)])
                           for k in range(2)])
        return nxt, Fn
    # pull with halfway bounce-back: f_i(x) = f*_i(x - c_i), or f*_opp(i)(x) where x - c_i is
    # solid; solid nodes stay empty
    fl = ~solid
    post = torch.where(fl, post, torch.zeros_like(post))
    opp = opposite(Q)
    rows = []
    for k in range(2):
        col = []
        for i in range(Q):
            src_solid = shift(solid, L["c"][i], +1)
            v = torch.where(src_solid, post[k, opp[i]], shift(post[k, i], L["c"][i], +1))
            col.append(torch.where(fl, v, torch.zeros_like(v)))
        rows.append(torch.stack(col))
    Fn = torch.where(fl, Fn, torch.zeros_like(Fn))
    return torch.stack(rows), Fn


def equilibrium_state(L, p, rho_r, rho_b):
    a_r, a_b = alphas(float(L["W"][0]), p["rho_in"])
    t_r = L["A"] + L["B"] * a_r
    t_b = L["A"] + L["B"] * a_b
    fr = t_r[:, None, None, None] * rho_r[None]
    fb = t_b[:, None, None, None] * rho_b[None]
    return torch.stack([fr, fb])


def gradient_magnitude(L, f, solid=None):
    F = phase_gradient(L, wetted(L, phase_field(f, solid), solid))
    g = torch.sqrt(F[0] ** 2 + F[1] ** 2 + F[2] ** 2)
    return g if solid is None else torch.where(solid, torch.zeros_like(g), g)


def run(params, rho_r, rho_b, phi, nsteps, gamma=None, masks=None, return_masks=False,
        solid=None):
    """Forward run.  phi: [nz, ny, nx] (held over time) or [nsteps, nz, ny, nx] tensor.
    Soft rule when params['site_rule'] == 'soft' (gamma: 0-d tensor, kappa from params);
    otherwise hard masks, given as [nsteps, nz, ny, nx] or taken from ||F_{n-1}|| > Gamma.
    solid: optional [nz, ny, nx] flags (nonzero = solid).  Returns the final state (and the
    masks used)."""
    if params.get("site_rule", "grad") not in ("grad", "soft"):
        raise ValueError("the reference implements the gradient-threshold site rules only")
    L = lattice(int(params["Q"]))
    sd = None if solid is None else torch.as_tensor(solid) != 0
    f = equilibrium_state(L, params, torch.as_tensor(rho_r, dtype=DT),
                          torch.as_tensor(rho_b, dtype=DT))
    if sd is not None:
        f = torch.where(sd, torch.zeros_like(f), f)
    fprev = gradient_magnitude(L, f, sd).detach()
    soft = params.get("site_rule") == "soft"
    if gamma is None:
        gamma = torch.tensor(params["gamma"], dtype=DT)
    used = []
    for n in range(nsteps):
        ph = phi[n] if phi.dim() == 4 else phi
        if soft:
            w = torch.sigmoid((fprev - gamma) / params.get("kappa", 0.01))
        elif masks is not None:
            w = torch.as_tensor(masks[n], dtype=DT)
        else:
            w = (fprev > float(gamma.detach())).to(DT)
        used.append(w.detach())
        f, fprev = step(L, params, f, fprev, ph, w, solid=sd)
    return (f, torch.stack(used)) if return_masks else f


def loss_rhoN(f, target, solid=None):
    """sum over the fluid nodes of (rho^N - target)^2."""
    d = phase_field(f, None if solid is None else torch.as_tensor(solid) != 0) - target
    if solid is not None:
        d = torch.where(torch.as_tensor(solid) != 0, torch.zeros_like(d), d)
    return (d ** 2).sum()


def gradients(params, rho_r, rho_b, phi, nsteps, target, gamma=None, masks=None,
              space_time=False, solid=None):
    """dL/dphi (and dL/dGamma in the soft rule) of L = sum_x (rho^N_T - target)^2.
    phi is a fixed [nz, ny, nx] field; with space_time the gradient is per step."""
    phi0 = torch.as_tensor(phi, dtype=DT)
    if space_time:
        ph = phi0.expand((nsteps,) + phi0.shape).clone().requires_grad_(True)
    else:
        ph = phi0.clone().requires_grad_(True)
    g = torch.tensor(params["gamma"] if gamma is None else gamma, dtype=DT, requires_grad=True)
    f = run(params, rho_r, rho_b, ph, nsteps, gamma=g, masks=masks, solid=solid)
    L = loss_rhoN(f, torch.as_tensor(target, dtype=DT), solid)
    L.backward()
    L = L.detach()
    return {"loss": L.item(), "grad_phi": ph.grad.detach(),
            "grad_gamma": None if g.grad is None else float(g.grad)}
