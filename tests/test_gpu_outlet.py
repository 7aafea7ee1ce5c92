"""Blue pressure outlets (Zou and He) on the end planes of the last lattice axis on the GPU:
step-by-step parity with the FP64 oracle at density ratio 2, and the outlet density held."""
import numpy as np
import pytest

from paper_2412_14859_amd import inputs
from tests.helpers import HALF_NODE, e_pop, gpu_for, oracle_for

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def _drop(Q, shape, R, ratio=2.0, wall=False, phi=1e-3):
    """A drop (density ratio `ratio`) in the middle of the last axis, blue at 1.03 so that
    the outlets (rho_b = 1) draw an outflow; optionally a wall plane at index 0.  The centre
    sits half a node off the box centre (tests/helpers.HALF_NODE): no saddle of the phase
    field between the drop and its periodic images falls on a node."""
    nz, ny, nx = shape
    ox, oy, oz = HALF_NODE
    centre = (nx / 2 + ox, ny / 2 + oy, nz / 2 + oz) if Q == 19 else \
        (nx / 2 + ox, ny / 2 + oy, 0.0)
    d = inputs.sphere_distance(shape, centre, R)
    rr, rb = inputs.densities_from_distance(d, 2.0, (ratio, 1.03))
    p = inputs._base(Q, shape, rho_in=(ratio, 1.0), phi=phi)
    solid = None
    if wall:
        solid = inputs.wall_layers(shape, 0 if Q == 19 else 1, [0])
        rr = np.where(solid == 1, 0.0, rr)
        rb = np.where(solid == 1, 0.0, rb)
    return {"params": p, "rho_r": rr, "rho_b": rb, "solid": solid, "phi_field": None}


CASES = {
    "d2q9": (9, (1, 40, 24), 6.0, False),
    "d3q19": (19, (24, 12, 14), 4.0, False),
    "d3q19_wall": (19, (24, 12, 14), 4.0, True),
}


@pytest.mark.parametrize("kernel", ["auto", "twopass"])
@pytest.mark.parametrize("name", list(CASES))
def test_outlet_matches_the_oracle(name, kernel):
    """FP64 step parity: every step, the oracle restarted from the GPU's state agrees with the
    GPU's next state within 1e-12, or within 10x the spread of a second restarted oracle whose
    input is perturbed by 2e-16 relative where that is larger; the free-running trajectories
    are compared the same way against a perturbed oracle run.  The gauge covers a node whose
    recolouring angle is ill-conditioned (a mixed node where F nearly vanishes, so that an ulp
    of summation order in F turns its direction); the drop is placed so that none is expected,
    and the test reports how many steps needed the gauge."""
    Q, shape, R, wall = CASES[name]
    w = _drop(Q, shape, R, wall=wall)
    lo, hi = (not wall), True
    _flush(f"[outlet fp64] {name} {kernel}")
    ora = oracle_for(w)
    ora.set_outlet(lo, hi, 1.0)
    twin = oracle_for(w)  # the oracle's own sensitivity
    f = twin.populations()
    twin.set_populations(f * (1 + 2e-16 * np.random.default_rng(0).standard_normal(f.shape)))
    twin.set_outlet(lo, hi, 1.0)
    one = oracle_for(w)  # restarted from the GPU's state every step
    one.set_outlet(lo, hi, 1.0)
    one2 = oracle_for(w)  # the same, from a perturbed copy of it
    one2.set_outlet(lo, hi, 1.0)
    rng = np.random.default_rng(1)
    sim = gpu_for(w, "fp64", kernel=kernel)
    sim.set_outlet(lo, hi, 1.0)
    rho_in = w["params"]["rho_in"]
    e = e_pop(sim.populations().cpu().numpy(), ora.populations(), Q, rho_in, w["solid"])
    assert e < 1e-14, e
    ax = 0 if Q == 19 else 1
    worst = worst_step = 0.0
    gauged = 0
    for step in range(1, 17):
        f0 = sim.populations().cpu().numpy()
        # the GPU carries the site mask (||F|| > Gamma) of the previous step
        m0 = np.where(sim.carry.cpu().numpy() > 0, 1e300, 0.0)
        one.set_populations(f0)
        one.set_fmag(m0)
        one.step(1)
        one2.set_populations(f0 * (1 + 2e-16 * rng.standard_normal(f0.shape)))
        one2.set_fmag(m0)
        one2.step(1)
        sim.step(1)
        ora.step(1)
        twin.step(1)
        fg, f1 = sim.populations().cpu().numpy(), one.populations()
        es = e_pop(fg, f1, Q, rho_in, w["solid"])
        gauge = 10.0 * e_pop(one2.populations(), f1, Q, rho_in, w["solid"])
        gauged += es >= 1e-12
        worst_step = max(worst_step, es)
        assert es < max(1e-12, gauge), ("step parity", step, es, gauge)
        fo = ora.populations()
        spread = e_pop(twin.populations(), fo, Q, rho_in, w["solid"])
        e = e_pop(fg, fo, Q, rho_in, w["solid"])
        worst = max(worst, e)
        assert e < max(1e-12, 10.0 * spread), ("trajectory", step, e, spread)
    _flush(f"  worst step e_pop {worst_step:.2e} ({gauged} of 16 steps above 1e-12, within "
           f"the gauge), trajectory {worst:.2e}")
    rb = sim.fields()["rho_b"].cpu().numpy()
    planes = ([0] if lo else []) + ([shape[ax] - 1] if hi else [])
    for k in planes:
        plane = np.take(rb, k, axis=ax)
        assert np.abs(plane - 1.0).max() < 1e-14
    og, oo = sim.observables(), ora.observables()
    assert abs(og["mass_b"] - oo["mass_b"]) < 1e-11 * oo["mass_b"]
    assert og["mass_b"] < float(w["rho_b"].sum())  # blue left through the outlets
    sim.close()


def test_outlet_fp32_storage_frozen_mask():
    import torch
    Q, shape, R, wall = CASES["d3q19"]
    w = _drop(Q, shape, R)
    p = w["params"]
    _flush("[outlet fp32s frozen]")
    ora = oracle_for(w)
    ora.set_outlet(True, True, 1.0)
    sim = gpu_for(w, "fp32s")
    sim.set_outlet(True, True, 1.0)
    for step in range(40):
        mask = (ora.fmag() > p["gamma"]).astype(np.uint8)
        sim.carry.copy_(torch.as_tensor(mask, device=sim.carry.device))
        sim.step(1)
        ora.step(1, masks=mask[None])
    e = e_pop(sim.populations().cpu().numpy(), ora.populations(), Q, p["rho_in"], w["solid"])
    _flush(f"  e_pop after 40 steps {e:.3e}")
    assert e < 1e-5
    sim.close()


def test_feature_setters_reject_bad_arguments_and_the_adjoint_refuses_them():
    """Outlets: a non-positive or non-finite outlet density, or fewer than 3 planes along the
    last axis, is EINVAL.  Height flux: without a bound flux field ESTATE, K <= 0 or h_s <= 0
    EINVAL.  A non-finite site threshold is EINVAL.  The checkpointed forward refuses
    outlets and the height flux (EUNSUPPORTED).  Nothing is changed by a rejected call."""
    from paper_2412_14859_amd import cgevap
    Q, shape, R, wall = CASES["d3q19"]
    w = _drop(Q, shape, R)
    sim = gpu_for(w, "fp64")
    f0 = sim.populations().cpu().numpy()
    for rho_out in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(cgevap.CgeError) as e:
            sim.set_outlet(True, True, rho_out)
        assert e.value.status == cgevap.EINVAL
    with pytest.raises(cgevap.CgeError) as e:
        sim.set_site_threshold(float("nan"))
    assert e.value.status == cgevap.EINVAL
    with pytest.raises(cgevap.CgeError) as e:
        sim.set_height_flux(1e-3, 1.0, 4.0, every=1)  # no flux field bound
    assert e.value.status == cgevap.ESTATE
    assert np.array_equal(sim.populations().cpu().numpy(), f0)
    sim.set_outlet(True, True, 1.0)
    with pytest.raises(cgevap.CgeError) as e:
        sim.forward_ckpt(4, 2)
    assert e.value.status == cgevap.EUNSUPPORTED
    sim.close()
    thin = _drop(Q, (2, 12, 14), 3.0)
    sim = gpu_for(thin, "fp64")
    with pytest.raises(cgevap.CgeError) as e:
        sim.set_outlet(True, True, 1.0)
    assert e.value.status == cgevap.EINVAL
    sim.close()
    wf = dict(w, phi_field=np.full(shape, 1e-3))
    sim = gpu_for(wf, "fp64")
    for K, hs in ((0.0, 4.0), (-1.0, 4.0), (1.0, 0.0), (float("nan"), 4.0)):
        with pytest.raises(cgevap.CgeError) as e:
            sim.set_height_flux(1e-3, K, hs, every=1)
        assert e.value.status == cgevap.EINVAL
    sim.set_height_flux(1e-3, 1.0, 4.0, every=1)
    with pytest.raises(cgevap.CgeError) as e:
        sim.forward_ckpt(4, 2)
    assert e.value.status == cgevap.EUNSUPPORTED
    sim.close()
