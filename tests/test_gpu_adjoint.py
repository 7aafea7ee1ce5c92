"""GPU adjoint (cge_forward_ckpt / cge_backward) against the FP64 CPU autograd reference on
the same seeded inputs, against central finite differences of the GPU's own forward run, and
through the torch.autograd.Function wrapper.

Loss: L = sum_x (rho^N_T - target)^2, so dL/drho^N_T = 2 (rho^N_T - target).  Hard sites
(||F_{n-1}|| > Gamma) are held at the forward run's; soft sites are logistic in
(||F_{n-1}|| - Gamma) / kappa and also give dL/dGamma."""
import numpy as np
import pytest

from oracle import adjoint as A
from tests.helpers import case, gpu_for

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def _target(shape, r):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) - (nz - 1) / 2.0, np.arange(ny) - ny / 2.0,
                          np.arange(nx) - nx / 2.0, indexing="ij")
    rr = np.sqrt(x * x + y * y + (z * z if nz > 1 else 0.0))
    return np.tanh((r - rr) / 2.0)


CASES = {
    # name: (workload, shape, overrides, target radius)
    "d2q9_hard": ("adjoint2d", (1, 16, 18), dict(radius=5.0, phi=3e-3, site_rule="grad"), 5.5),
    "d2q9_soft": ("adjoint2d", (1, 16, 18), dict(radius=5.0, phi=3e-3, site_rule="soft",
                                                 kappa=0.02), 5.5),
    "d2q9_soft_ratio": ("adjoint2d", (1, 20, 22), dict(radius=6.0, phi=3e-3, site_rule="soft",
                                                       kappa=0.02, rho_in=(1.0, 0.5),
                                                       tau=(1.0, 0.7), beta=0.6), 6.5),
    "d3q19_soft": ("sphere3d", (8, 9, 10), dict(radius=3.0, phi=3e-3, site_rule="soft",
                                                kappa=0.02), 3.3),
    "d3q19_hard": ("sphere3d", (8, 9, 10), dict(radius=3.0, phi=3e-3), 3.3),
    # relaxation times other than 1: the reverse step recomputes from stored populations
    "d3q19_tau": ("sphere3d", (8, 9, 10), dict(radius=3.0, phi=3e-3, tau=(1.0, 0.8)), 3.3),
    # solid nodes: bounce-back pairs and wetting values in the transpose
    "d2q9_walls_hard": ("flat2d", (1, 20, 22), dict(phi=3e-3, site_rule="grad"), 6.0),
    "d2q9_walls_soft_tau": ("flat2d", (1, 20, 22), dict(phi=3e-3, site_rule="soft", kappa=0.02,
                                                        tau=(1.0, 0.8)), 6.0),
    "d3q19_walls_ratio": ("sessile3d", (8, 12, 14), dict(radius=4.0, phi=3e-3), 4.0),
    "d3q19_walls_soft": ("hemisphere3d", (10, 12, 12), dict(radius=4.0, phi=3e-3,
                                                            site_rule="soft", kappa=0.02), 4.5),
}


def _setup(name):
    wl, shape, over, r = CASES[name]
    w = case(wl, shape, **over)
    if w["phi_field"] is None:  # a seeded field around the uniform flux
        rng = np.random.default_rng(5)
        w["phi_field"] = w["params"]["phi"] * rng.uniform(0.8, 1.2, shape)
    return w, _target(shape, r)


def _gpu_gradients(w, target, nsteps, K, precision="fp64", per_step=False, kernel="auto"):
    import torch
    sim = gpu_for(w, precision, kernel=kernel)
    ck = sim.forward_ckpt(nsteps, K)
    rn = sim.fields()["rhoN"]
    g = 2.0 * (rn - torch.as_tensor(target, device=rn.device))
    d2 = (rn.cpu().numpy() - target) ** 2
    if w["solid"] is not None:  # the loss runs over the fluid nodes (seeds at solid ones are ignored)
        d2 = np.where(w["solid"] != 0, 0.0, d2)
    loss = float(d2.sum())
    r = sim.backward(ck, nsteps, K, g, per_step=per_step)
    step = sim.observables()["step"]
    out = {"loss": loss, "grad_phi": r["grad_phi"].cpu().numpy(), "grad_gamma": r["grad_gamma"],
           "grad_phi_t": None if r["grad_phi_t"] is None else r["grad_phi_t"].cpu().numpy(),
           "step_after": step}
    sim.close()
    return out


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_gradients_match_the_autograd_reference(name):
    w, target = _setup(name)
    p = w["params"]
    nsteps, K = 25, 7  # segments 7, 7, 7, 4
    _flush(f"[adjoint fp64] {name} {w['rho_r'].shape} n={nsteps} K={K}")
    got = _gpu_gradients(w, target, nsteps, K)
    ref = A.gradients(p, w["rho_r"], w["rho_b"], w["phi_field"], nsteps, target,
                      solid=w["solid"])
    assert abs(got["loss"] - ref["loss"]) <= 1e-12 * ref["loss"]
    gr = ref["grad_phi"].numpy()
    assert np.abs(gr).max() > 0
    e = _rel(got["grad_phi"], gr)
    _flush(f"  grad_phi rel err {e:.2e}")
    assert e < 1e-10, e
    if p["site_rule"] == "soft":
        eg = abs(got["grad_gamma"] - ref["grad_gamma"]) / abs(ref["grad_gamma"])
        _flush(f"  grad_gamma {got['grad_gamma']:.6e} ref {ref['grad_gamma']:.6e} rel {eg:.2e}")
        assert eg < 1e-10, eg
    else:
        assert got["grad_gamma"] == 0.0
    assert got["step_after"] == nsteps  # the step counter is restored


def test_per_step_flux_gradient_matches_the_reference():
    w, target = _setup("d2q9_soft")
    p = w["params"]
    nsteps, K = 12, 5
    _flush("[adjoint fp64] per-step dL/dphi(x, t)")
    got = _gpu_gradients(w, target, nsteps, K, per_step=True)
    ref = A.gradients(p, w["rho_r"], w["rho_b"], w["phi_field"], nsteps, target,
                      space_time=True)["grad_phi"].numpy()
    assert got["grad_phi_t"].shape == ref.shape
    e = _rel(got["grad_phi_t"], ref)
    assert e < 1e-10, e
    # the time-constant gradient is the sum over the steps
    assert np.abs(got["grad_phi_t"].sum(0) - got["grad_phi"]).max() <= 1e-15 * nsteps * \
        np.abs(got["grad_phi"]).max()


def test_checkpoint_interval_does_not_change_the_gradients():
    w, target = _setup("d2q9_soft")
    _flush("[adjoint] K in (1, 4, 9, 30) for 9 steps")
    res = [_gpu_gradients(w, target, 9, K) for K in (1, 4, 9, 30)]
    for r in res[1:]:
        assert np.array_equal(r["grad_phi"], res[0]["grad_phi"])
        assert r["grad_gamma"] == res[0]["grad_gamma"]


def _reference_fp32_storage(w, target, nsteps):
    """The autograd reference on the trajectory of FP32 storage: after every step the state is
    rounded to nearest float32 in the stored encoding (ft_i = f_i^r + f_i^b - rho_b^in
    t_i(alpha_b), dd_i = f_i^r - f_i^b), as is the flux field.  Within a step the phase
    field rho^N is stored in float32 too, and the step continues from the stored value; at
    unit relaxation times the split step also stores rho - rho_b^in and j (rho^N computed
    with the unrounded rho).  All of that is reproduced.  The roundings pass gradients
    through unchanged."""
    import torch
    DT = torch.float64
    p = w["params"]
    L = A.lattice(int(p["Q"]))
    a_b = A.alphas(float(L["W"][0]), p["rho_in"])[1]
    tref = ((L["A"] + L["B"] * a_b) * p["rho_in"][1])[:, None, None, None]

    def rnd(x):
        return x + (x.float().double() - x).detach()

    def store(f):
        ft, dd = rnd(f[0] + f[1] - tref), rnd(f[0] - f[1])
        return torch.stack([(ft + tref + dd) / 2, (ft + tref - dd) / 2])

    rho_ref = float(p["rho_in"][1])

    def stored_rhoN(rhoN, rho, rho_lin):
        # the value rounded to float32; the derivatives those of D / rho (D = rho_r - rho_b)
        # taken at the stored value, 1 / rho and -rhoN_stored / rho with rho = rho_lin: the
        # adjoint linearises the stored field, as the exact quotient is not kept
        D = rho * rhoN
        c = rhoN.float().double().detach()
        r0 = rho_lin.detach()
        e = D - c * rho_lin
        return c + e / r0 - e.detach() / r0

    def split_moments(rho, j, rhoN):  # (j_z of D2Q9 is the constant 0)
        rho_s = rho_ref + rnd(rho - rho_ref)
        return (rho_s, [rnd(a) if torch.is_tensor(a) else a for a in j],
                stored_rhoN(rhoN, rho, rho_s))

    def stored_phase(rho, j, rhoN):
        return rho, j, stored_rhoN(rhoN, rho, rho)

    unit = tuple(p["tau"]) == (1.0, 1.0)
    ph = torch.as_tensor(w["phi_field"], dtype=torch.float32).double().requires_grad_(True)
    g = torch.tensor(p["gamma"], dtype=DT, requires_grad=True)
    f = store(A.equilibrium_state(L, p, torch.as_tensor(w["rho_r"], dtype=DT),
                                  torch.as_tensor(w["rho_b"], dtype=DT))).detach()
    fprev = A.gradient_magnitude(L, f).detach()
    for _ in range(nsteps):
        m = torch.sigmoid((fprev - g) / p["kappa"])
        f, fprev = A.step(L, p, f, fprev, ph, m,
                          stored=split_moments if unit else stored_phase)
        f = store(f)
    A.loss_rhoN(f, torch.as_tensor(target, dtype=DT)).backward()
    return ph.grad.numpy(), float(g.grad)


@pytest.mark.parametrize("name,tol", [("d2q9_soft_ratio", 1e-9), ("d2q9_soft", 1e-9)])
def test_fp32_storage_gradients(name, tol):
    """FP32 storage: the adjoint of the FP32-storage trajectory against the reference on the
    trajectory rounded the same way: the populations after every step, and at unit
    relaxation times also the split step's stored moments (rho, j, rho^N).  Against FP64 the
    gradients move by what rounding the state moves them (~2e-4 on the equal-density case,
    in the reference as well), so that comparison bounds the size only."""
    w, target = _setup(name)
    _flush(f"[adjoint fp32s] {name}")
    g32 = _gpu_gradients(w, target, 25, 7, "fp32s")
    rp, rg = _reference_fp32_storage(w, target, 25)
    e = _rel(g32["grad_phi"], rp)
    eg = abs(g32["grad_gamma"] - rg) / abs(rg)
    g64 = _gpu_gradients(w, target, 25, 7, "fp64")
    e64 = _rel(g32["grad_phi"], g64["grad_phi"])
    _flush(f"  vs rounded reference: grad_phi {e:.2e} grad_gamma {eg:.2e}; vs fp64 {e64:.2e}")
    assert e < tol and eg < tol, (e, eg)
    assert e64 < 5e-3


@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_checkpointed_run_does_not_depend_on_the_context_step_form(precision):
    """At unit relaxation times the checkpointed forward and its recomputation use the split
    step whatever step form the context runs, so the gradients are the same bit for bit."""
    w, target = _setup("d3q19_hard")
    _flush(f"[adjoint] d3q19 hard {precision}, two-pass / fused / split contexts")
    res = [_gpu_gradients(w, target, 10, 4, precision, kernel=k)
           for k in ("twopass", "fused", "split")]
    for r in res[1:]:
        assert np.array_equal(r["grad_phi"], res[0]["grad_phi"])
        assert r["loss"] == res[0]["loss"]


def test_c5_instance_central_differences():
    """The adjoint benchmark's finite-difference instance (tests/test_adjoint_oracle.py,
    _c5_instance: 32 x 32, R = 6, soft sites kappa = 0.01, 200 steps, FP64, checkpoints every
    100 steps): the GPU adjoint against central differences of the GPU's own FP64 forward
    with relative step 1e-3, for the three random directions and the eight interface nodes
    (within 1e-6: the loss is linear in phi to below its rounding over that step) and for
    Gamma (within 2e-3: the truncation of the curved Gamma dependence is 3e-5), and against
    the CPU adjoint reference on the same instance within 1e-10."""
    import torch
    from oracle import adjoint as A
    from tests.test_adjoint_oracle import _c5_instance
    w, p, phi, target, dirs = _c5_instance()
    target = target.numpy()
    nsteps, K = 200, 100
    _flush("[adjoint FD] C5 instance: d2q9 32x32 soft, 200 steps")
    got = _gpu_gradients(w, target, nsteps, K)
    ref = A.gradients(p, w["rho_r"], w["rho_b"], phi, nsteps, target)
    assert _rel(got["grad_phi"], ref["grad_phi"].numpy()) < 1e-10
    assert abs(got["grad_gamma"] - ref["grad_gamma"]) <= 1e-10 * abs(ref["grad_gamma"])
    assert abs(got["loss"] - ref["loss"]) <= 1e-12 * abs(ref["loss"])

    def loss(phi_field, gamma):
        ww = dict(w, phi_field=phi_field, params=dict(p, gamma=gamma))
        sim = gpu_for(ww, "fp64")
        sim.step(nsteps)
        rn = sim.fields()["rhoN"].cpu().numpy()
        sim.close()
        return float(((rn - target) ** 2).sum())

    eps = 1e-3
    for k, v in enumerate(dirs):
        v = v.numpy()
        ad = float((got["grad_phi"] * v).sum())
        fd = (loss(w["phi_field"] + eps * v, p["gamma"]) -
              loss(w["phi_field"] - eps * v, p["gamma"])) / (2 * eps)
        _flush(f"  probe {k}: adjoint {ad:.10e} fd {fd:.10e}")
        assert abs(fd - ad) <= 1e-6 * abs(ad), (k, fd, ad)
    eg = eps * p["gamma"]
    fd = (loss(w["phi_field"], p["gamma"] + eg) - loss(w["phi_field"], p["gamma"] - eg)) / (2 * eg)
    _flush(f"  gamma: adjoint {got['grad_gamma']:.10e} fd {fd:.10e}")
    assert abs(fd - got["grad_gamma"]) <= 2e-3 * abs(got["grad_gamma"])
    del torch


def test_autograd_function_wrapper():
    import torch
    from paper_2412_14859_amd import cgevap
    w, target = _setup("d2q9_soft")
    _flush("[adjoint] torch.autograd.Function")
    sim = gpu_for(w, "fp64")
    start = sim.save_state().clone()
    dev = sim.device
    phi = torch.as_tensor(w["phi_field"], device=dev).requires_grad_(True)
    gamma = torch.tensor(w["params"]["gamma"], dtype=torch.float64, device=dev,
                         requires_grad=True)
    tgt = torch.as_tensor(target, device=dev)
    for _ in range(2):  # the start state is reloaded on every call
        phi.grad = gamma.grad = None
        rn = cgevap.evaporate(sim, phi, gamma, 25, 7, start)
        loss = ((rn - tgt) ** 2).sum()
        loss.backward()
        ref = A.gradients(w["params"], w["rho_r"], w["rho_b"], w["phi_field"], 25, target)
        assert abs(float(loss.detach()) - ref["loss"]) <= 1e-12 * ref["loss"]
        assert _rel(phi.grad.cpu().numpy(), ref["grad_phi"].numpy()) < 1e-10
        assert abs(float(gamma.grad) - ref["grad_gamma"]) <= 1e-10 * abs(ref["grad_gamma"])
    sim.close()


def test_autograd_function_interleaved_runs():
    """Two differentiable runs on one simulation, both forwards before either backward, with
    different flux fields and thresholds: each backward gives the gradient of its own run, the
    one the same run gives when its backward follows its forward directly."""
    import torch
    from paper_2412_14859_amd import cgevap
    w, target = _setup("d2q9_soft")
    _flush("[adjoint] interleaved evaporate calls")
    sim = gpu_for(w, "fp64")
    start = sim.save_state().clone()
    dev = sim.device
    tgt = torch.as_tensor(target, device=dev)
    base = torch.as_tensor(w["phi_field"], device=dev)
    runs = [(base, w["params"]["gamma"]), (base * 1.3, w["params"]["gamma"] + 0.01)]

    def leaves(ph, g):
        return (ph.clone().requires_grad_(True),
                torch.tensor(g, dtype=torch.float64, device=dev, requires_grad=True))

    seq = []
    for ph, g in runs:  # each backward right after its forward
        phi, gamma = leaves(ph, g)
        ((cgevap.evaporate(sim, phi, gamma, 25, 7, start) - tgt) ** 2).sum().backward()
        seq.append((phi.grad.clone(), float(gamma.grad)))
    ins = [leaves(ph, g) for ph, g in runs]
    losses = [((cgevap.evaporate(sim, phi, gamma, 25, 7, start) - tgt) ** 2).sum()
              for phi, gamma in ins]
    for k in (1, 0):  # the later run's backward first, then the earlier one's
        losses[k].backward()
        assert torch.equal(ins[k][0].grad, seq[k][0]), k
        assert float(ins[k][1].grad) == seq[k][1], k
    sim.close()


@pytest.mark.parametrize("name", ["d2q9_soft", "d2q9_soft_ratio"])
def test_backward_is_repeatable_and_restores_the_state(name):
    """The backward seeds from the final checkpoint and leaves the context at the final state
    with its counters, so a second backward (another loss) is independent of the first."""
    import torch
    w, target = _setup(name)
    _flush(f"[adjoint] repeat + restore {name}")
    sim = gpu_for(w, "fp32s")
    ck = sim.forward_ckpt(20, 6)
    f_end, obs_end = sim.populations().cpu(), sim.observables()
    fl = sim.fields()
    g = 2.0 * (fl["rhoN"] - torch.as_tensor(target, device=sim.device))
    rho = fl["rho_r"] + fl["rho_b"]
    a = sim.backward(ck, 20, 6, g)
    assert torch.equal(sim.populations().cpu(), f_end)
    obs = sim.observables()
    for k in ("step", "sink_total", "site_steps", "mass_r"):
        assert obs[k] == obs_end[k], k
    sim.backward(ck, 20, 6, dL_drho=torch.ones_like(rho))  # another loss in between
    b = sim.backward(ck, 20, 6, g)
    assert torch.equal(a["grad_phi"], b["grad_phi"]) and a["grad_gamma"] == b["grad_gamma"]
    sim.close()


def test_unsupported_configurations_are_rejected():
    """The |rho^N| < Gamma site rule has no adjoint (the outlets and the height flux are
    refused by the checkpointed forward: tests/test_gpu_outlet.py)."""
    import torch
    from paper_2412_14859_amd import cgevap
    w = case("drop2d", (1, 12, 16), radius=4.0, phi=1e-3)  # |rho^N| < Gamma site rule
    sim = gpu_for(w, "fp64")
    ck = sim.forward_ckpt(2, 2)
    with pytest.raises(cgevap.CgeError) as e:
        sim.backward(ck, 2, 2, torch.zeros(sim.shape, dtype=torch.float64, device=sim.device))
    assert e.value.status == cgevap.EUNSUPPORTED
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
def test_red_mass_covector_with_walls(precision):
    """A hemispherical drop on a wall (64^3, walls at both ends, 300 steps, K = 50, hard
    sites).  Every operator but the sink conserves red mass, bounce-back and wetting
    included, so for L = final red mass the per-step gradient is exactly dL/dphi(x, t) =
    -m(x, t)/Sbar: 0 or -1/Sbar at fluid nodes, 0 at solid ones, and sum_x phi dL/dphi is
    minus the mass the sink removed."""
    import torch
    w = case("hemisphere3d", (64, 64, 64), radius=20.0, phi=3e-3)
    p = w["params"]
    nsteps, K = 300, 50
    _flush(f"[adjoint walls] hemisphere 64^3 red-mass covector {precision}")
    sim = gpu_for(w, precision)
    ck = sim.forward_ckpt(nsteps, K)
    obs = sim.observables()
    fl = sim.fields()
    rho = fl["rho_r"] + fl["rho_b"]
    r = sim.backward(ck, nsteps, K, dL_drhoN=rho / 2, dL_drho=(1 + fl["rhoN"]) / 2,
                     per_step=True)
    gt = r["grad_phi_t"].cpu().numpy() * p["sbar"]
    solid = w["solid"] != 0
    assert np.abs(gt[:, solid]).max() == 0.0
    vals = gt[:, ~solid]
    dist = np.minimum(np.abs(vals), np.abs(vals + 1.0))
    _flush(f"  |Sbar dL/dphi - {{0, -1}}| max {dist.max():.2e}; sites {int((vals < -0.5).sum())}")
    assert dist.max() < 1e-11
    assert (vals < -0.5).sum() > 0
    phi = sim.phi_field.to(torch.float64)
    lhs = float((phi * r["grad_phi"]).sum())
    rel = abs(lhs + obs["sink_total"]) / obs["sink_total"]
    _flush(f"  sum phi dL/dphi {lhs:.12e}, sink total {obs['sink_total']:.12e}, rel {rel:.2e}")
    assert rel < 1e-11
    sim.close()
