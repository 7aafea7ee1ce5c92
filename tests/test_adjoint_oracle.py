"""Pins of the FP64 CPU adjoint reference (oracle/adjoint.py, autograd through a plain
PyTorch CPU step): its forward equals the C oracle's, its gradients equal central finite
differences, and the red-mass sensitivity equals the closed form -m(x,t)/Sbar."""
import numpy as np
import pytest
import torch

from oracle import adjoint as A
from oracle.oracle import tables
from tests.helpers import case, oracle_for

DT = torch.float64


@pytest.mark.parametrize("Q", [9, 19])
def test_tables_agree_with_the_c_oracle(Q):
    L = A.lattice(Q)
    t = tables(Q)
    assert np.array_equal(L["ct"].numpy().astype(int), t["c"])
    for k in ("W", "A", "B", "C"):
        assert np.allclose(L[k].numpy(), t[k], rtol=0, atol=1e-16), k


@pytest.mark.parametrize("wl,shape,over", [
    ("drop2d", (1, 20, 26), dict(radius=6.0, phi=1e-3, site_rule="grad", gamma=0.305)),
    ("sphere3d", (8, 9, 10), dict(radius=3.0, phi=1e-3)),
    ("drop2d", (1, 20, 26), dict(radius=6.0, phi=1e-3, site_rule="soft", gamma=0.305,
                                 kappa=0.01)),
    ("drop2d", (1, 20, 26), dict(radius=6.0, phi=1e-3, tau=(1.0, 0.7), beta=0.5,
                                 site_rule="grad", gamma=0.305)),
    # solid nodes: a film between walls; a cap on a wall at density ratio 10 with a flux field
    ("flat2d", (1, 20, 26), dict(phi=1e-3)),
    ("sessile3d", (8, 12, 14), dict(radius=4.0, phi=1e-3)),
    ("hemisphere3d", (10, 12, 12), dict(radius=4.0, phi=1e-3, site_rule="soft", kappa=0.02)),
])
def test_forward_equals_the_c_oracle(wl, shape, over):
    w = case(wl, shape, **over)
    p = w["params"]
    ora = oracle_for(w)
    ora.step(8)
    phi = torch.full(shape, p["phi"], dtype=DT) if w["phi_field"] is None else \
        torch.as_tensor(w["phi_field"], dtype=DT)
    f = A.run(p, w["rho_r"], w["rho_b"], phi, 8, solid=w["solid"])
    assert np.abs(f.detach().numpy() - ora.populations()).max() < 1e-14


def _instance(site_rule="grad"):
    w = case("adjoint2d", (1, 16, 18), radius=5.0, phi=3e-3)
    p = dict(w["params"], site_rule=site_rule, kappa=0.02)
    rng = np.random.default_rng(11)
    target = np.tanh((5.5 - np.hypot(*np.meshgrid(np.arange(18) - 9.0, np.arange(16) - 8.0))) / 2.0)
    return w, p, torch.as_tensor(w["phi_field"], dtype=DT), torch.as_tensor(target[None]), rng


def test_gradient_wrt_flux_matches_central_differences():
    """Hard sites, held fixed at the base run's masks for the perturbed runs."""
    w, p, phi, target, rng = _instance()
    n = 25
    _, masks = A.run(p, w["rho_r"], w["rho_b"], phi, n, return_masks=True)
    g = A.gradients(p, w["rho_r"], w["rho_b"], phi, n, target, masks=masks)["grad_phi"]
    assert float(g.abs().max()) > 0
    # central differences carry an O(eps^2) truncation error; a wrong gradient would leave a
    # floor that does not shrink, so the error must also fall ~100x when eps falls 10x, unless
    # both are already at the rounding floor (below 1e-7: the loss is linear in phi to ~1e-10
    # over +-1e-3 relative on this instance), far below any wrong gradient's floor
    for trial in range(3):
        v = torch.as_tensor(rng.standard_normal(phi.shape), dtype=DT) * phi
        ad = float((g * v).sum())
        err = []
        for eps in (1e-3, 1e-4):
            lp = A.loss_rhoN(A.run(p, w["rho_r"], w["rho_b"], phi + eps * v, n, masks=masks),
                             target)
            lm = A.loss_rhoN(A.run(p, w["rho_r"], w["rho_b"], phi - eps * v, n, masks=masks),
                             target)
            err.append(abs(float(lp - lm) / (2 * eps) - ad) / abs(ad))
        assert err[0] < 2e-3 and err[1] < 2e-5, (trial, err)
        assert err[1] < err[0] / 30 or max(err) < 1e-7, (trial, err)


def test_gradient_wrt_gamma_matches_central_differences_soft_sites():
    w, p, phi, target, _ = _instance("soft")
    n = 25
    res = A.gradients(p, w["rho_r"], w["rho_b"], phi, n, target)
    assert res["grad_gamma"] != 0.0
    err = []
    for rel in (1e-3, 1e-4):
        eps = rel * p["gamma"]
        lp = A.loss_rhoN(A.run(p, w["rho_r"], w["rho_b"], phi, n,
                               gamma=torch.tensor(p["gamma"] + eps, dtype=DT)), target)
        lm = A.loss_rhoN(A.run(p, w["rho_r"], w["rho_b"], phi, n,
                               gamma=torch.tensor(p["gamma"] - eps, dtype=DT)), target)
        err.append(abs(float(lp - lm) / (2 * eps) - res["grad_gamma"]) / abs(res["grad_gamma"]))
    assert err[0] < 2e-3 and err[1] < 2e-5, err
    assert err[1] < err[0] / 30 or max(err) < 1e-7, err


def test_red_mass_sensitivity_is_minus_mask_over_sbar():
    """Every operator but the sink conserves red mass, so dM_r(T)/dphi(x, t) = -m(x, t)/Sbar
    exactly (hard sites)."""
    w, p, phi, _, _ = _instance()
    n = 12
    _, masks = A.run(p, w["rho_r"], w["rho_b"], phi, n, return_masks=True)
    ph = phi.expand((n,) + phi.shape).clone().requires_grad_(True)
    f = A.run(p, w["rho_r"], w["rho_b"], ph, n, masks=masks)
    f[0].sum().backward()
    expect = -masks / p["sbar"]
    assert masks.sum() > 0
    assert float((ph.grad - expect).abs().max()) < 1e-13


def test_red_mass_sensitivity_with_walls():
    """With solid nodes too (a film between walls: bounce-back and wetting), every operator but
    the sink conserves red mass, so dM_r(T)/dphi(x, t) = -m(x, t)/Sbar exactly, and 0 at solid
    nodes."""
    w = case("flat2d", (1, 20, 22), phi=3e-3)
    p = w["params"]
    phi = torch.full(p["shape"], 3e-3, dtype=DT)
    n = 10
    _, masks = A.run(p, w["rho_r"], w["rho_b"], phi, n, return_masks=True, solid=w["solid"])
    ph = phi.expand((n,) + phi.shape).clone().requires_grad_(True)
    f = A.run(p, w["rho_r"], w["rho_b"], ph, n, masks=masks, solid=w["solid"])
    f[0].sum().backward()
    fl = torch.as_tensor(w["solid"] == 0, dtype=DT)
    expect = -masks * fl / p["sbar"]
    assert float((masks * fl).sum()) > 0
    assert float((ph.grad - expect).abs().max()) < 1e-13


def _c5_instance():
    """The adjoint benchmark's finite-difference instance: the D2Q9 drop scaled to 32 x 32
    (R = 6), flux 1e-5 U(0.9, 1.1) (seed 1002), the wobbly target of seed 1003 scaled the same
    way (r0 = 5.625), soft sites with kappa = 0.01, 200 steps, FP64.  Probes: three random
    directions (seed 1004) scaled by phi, and eight interface nodes (|rho^N| < 0.5 at the
    start) drawn with the same generator."""
    w = case("adjoint2d", (1, 32, 32), site_rule="soft", kappa=0.01)
    p = w["params"]
    phi = torch.as_tensor(w["phi_field"], dtype=DT)
    rng = np.random.default_rng(1004)
    dirs = [torch.as_tensor(rng.standard_normal(phi.shape), dtype=DT) * phi for _ in range(3)]
    rhoN0 = (w["rho_r"] - w["rho_b"]) / (w["rho_r"] + w["rho_b"])
    iface = np.flatnonzero(np.abs(rhoN0) < 0.5)
    nodes = rng.choice(iface, size=8, replace=False)
    for k in nodes:
        v = torch.zeros(phi.numel(), dtype=DT)
        v[int(k)] = phi.reshape(-1)[int(k)]
        dirs.append(v.reshape(phi.shape))
    return w, p, phi, torch.as_tensor(w["target"], dtype=DT), dirs


def test_c5_instance_gradients_match_central_differences():
    """On the finite-difference instance of the adjoint benchmark, <dL/dphi, v> for the three
    random directions and the eight single interface nodes equals central differences with
    relative step 1e-3 within 1e-6: over +-1e-3 the loss is linear in phi to below its
    rounding (the differences agree to 4e-10 .. 3e-8, and move away as the step shrinks and
    the rounding of L ~ 6.5 grows against the difference), so any wrong term shows far above
    this bound; at step 1e-4 they still agree within 2e-5.  dL/dGamma is curved enough for
    the O(eps^2) truncation to show: within 2e-3 at 1e-3 and falling ~100x at 1e-4."""
    w, p, phi, target, dirs = _c5_instance()
    n = 200
    res = A.gradients(p, w["rho_r"], w["rho_b"], phi, n, target)
    g = res["grad_phi"]

    def loss(ph, gamma=None):
        gm = None if gamma is None else torch.tensor(gamma, dtype=DT)
        return float(A.loss_rhoN(A.run(p, w["rho_r"], w["rho_b"], ph, n, gamma=gm), target))

    for k, v in enumerate(dirs):
        ad = float((g * v).sum())
        assert ad != 0.0, k
        err = []
        for eps in (1e-3, 1e-4):
            fd = (loss(phi + eps * v) - loss(phi - eps * v)) / (2 * eps)
            err.append(abs(fd - ad) / abs(ad))
        assert err[0] < 1e-6 and err[1] < 2e-5, (k, err)
    gg = res["grad_gamma"]
    err = []
    for rel in (1e-3, 1e-4):
        eps = rel * p["gamma"]
        fd = (loss(phi, p["gamma"] + eps) - loss(phi, p["gamma"] - eps)) / (2 * eps)
        err.append(abs(fd - gg) / abs(gg))
    assert err[0] < 2e-3 and err[1] < 2e-5, err
    assert err[1] < err[0] / 30 or max(err) < 1e-7, err
