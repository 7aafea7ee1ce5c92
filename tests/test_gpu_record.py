"""The record form of the unit-relaxation step (kernel "record", CGE_KERNEL_RECORD).

Between the steps of one call each node keeps a 14-value post-collision record instead of
its 2Q populations; the first step of a call pulls populations and the last writes them.
A call of n steps therefore computes the same arithmetic as n steps of the split form, up to
the rounding of the record and of the rebuilt populations:
  * FP64: against the FP64 oracle within 1e-12 (the parity bar), calls of several steps;
    against the split form within 1e-13 with identical site masks and counters;
  * FP32 storage: against the split form within 1e-6 of the population scale (the record's
    FP32 values and the FP32 rebuild of each pulled population, against the split form's
    FP32-stored populations), the same sites and sink total to 1e-9 (1e-7 with the soft
    site rule, whose logistic weights amplify rounding differences of ||F|| by 1 / kappa);
  * FP16 storage (FP32 or FP64 arithmetic): half records with stochastic rounding against the
    split form's half populations within 5e-3, site-steps and sink totals within 1 %.
Shapes cover the z-marching pull of D3Q19 at every storage precision (64 x 8 tiles) with
ragged tiles, chunks of 1, 3, 5 and 32 planes (forced with cge_set_zchunk: on a 256-CU device
the automatic choice gives these small grids one plane per chunk) with ragged last chunks, one
and two planes and solid nodes, and the general pull: D2Q9, D3Q19 with an odd nx at FP16
storage (the half-record z-march takes two nodes per lane and needs an even nx), the
|rho^N| < Gamma and soft site rules."""
import numpy as np
import pytest

from tests.helpers import case, e_pop, gpu_for, oracle_for

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


ORACLE_CASES = {
    # name: (workload, shape (z, y, x), overrides)
    "d3q19_sphere": ("sphere3d", (20, 12, 40), dict(radius=4.5, phi=1e-3)),
    "d2q9_phase": ("drop2d", (1, 40, 52), dict(radius=11.0, phi=1e-3)),
    # a ring of solid nodes on the bottom wall (the pinned-cap cavity)
    "d3q19_walls": ("cap3d", (24, 32, 70), dict(radius=9.0, phi=1e-3)),
    "d2q9_walls_field": ("flat2d", (1, 40, 70), dict(phi=1e-3)),
    "d2q9_soft": ("adjoint2d", (1, 48, 70), dict(radius=14.0, phi=1e-3, site_rule="soft",
                                                 gamma=0.305, kappa=0.01)),
}


@pytest.mark.parametrize("name", list(ORACLE_CASES))
def test_record_calls_match_the_oracle_fp64(name):
    wl, shape, over = ORACLE_CASES[name]
    w = case(wl, shape, **over)
    Q, rho_in = w["params"]["Q"], w["params"]["rho_in"]
    _flush(f"[record fp64 vs oracle] {name} shape={shape}")
    ora = oracle_for(w)
    sim = gpu_for(w, "fp64", kernel="record")
    assert sim.kernel_name() == "k_pull_record"
    for calls in range(3):
        sim.step(4)
        ora.step(4)
        e = e_pop(sim.populations().cpu().numpy(), ora.populations(), Q, rho_in, w["solid"])
        assert e < 1e-12, (calls, e)
        if w["params"]["site_rule"] == "grad":
            mask = (ora.fmag() > w["params"]["gamma"]).astype(np.uint8)
            assert np.array_equal(sim.carry.cpu().numpy(), mask), calls
    og, oo = sim.observables(), ora.observables()
    for k in ("n_sites", "site_steps", "step"):
        assert og[k] == oo[k], k
    for k in ("mass_r", "mass_b", "sink_total"):
        assert abs(og[k] - oo[k]) <= 1e-12 * max(1.0, abs(oo[k])), (k, og[k], oo[k])
    assert og["site_steps"] > 0
    sim.close()


SPLIT_CASES = {
    # z-marching pull: ragged x, y and z tiles (70 planes: 32 + 32 + 6 at 32 planes per
    # chunk, 23 x 3 + 1 at 3); one and two planes
    "zm_ragged": ("sphere3d", (70, 10, 70), dict(radius=4.0, phi=1e-3)),
    "zm_aligned": ("sphere3d", (33, 8, 64), dict(radius=3.5, phi=1e-3)),
    "zm_one_plane": ("sphere3d", (1, 24, 64), dict(radius=6.0, phi=1e-3)),
    "zm_two_planes": ("sphere3d", (2, 20, 66), dict(radius=6.0, phi=1e-3)),
    # with solid nodes (the z-marching pull with walls at every storage precision): the
    # cavity ring, and a hemisphere on a wall with a flux field, ragged in x and z
    "walls": ("cap3d", (24, 32, 70), dict(radius=9.0, phi=1e-3)),
    "walls_hemisphere": ("hemisphere3d", (40, 20, 70), dict(radius=8.0, phi=1e-3)),
    # general pull
    "d3q19_odd_nx": ("sphere3d", (12, 10, 33), dict(radius=3.5, phi=1e-3)),
    "d2q9": ("drop2d", (1, 40, 52), dict(radius=11.0, phi=1e-3)),
    "soft": ("adjoint2d", (1, 48, 70), dict(radius=14.0, phi=1e-3, site_rule="soft",
                                            gamma=0.305, kappa=0.01)),
}


# planes per z-chunk of the z-marching pull: 0 lets the library choose (one plane per chunk
# for these small grids on a 256-CU device); 3 and 32 march through several planes per block,
# with a ragged last chunk where nz is not a multiple
ZCHUNKS = {"zm_ragged": (0, 3, 32), "zm_aligned": (0, 3, 32), "walls": (0, 3, 32),
           "walls_hemisphere": (0, 3, 32)}
SPLIT_PARAMS = [(name, zc) for name in SPLIT_CASES for zc in ZCHUNKS.get(name, (0,))]


@pytest.mark.parametrize("precision", ["fp64", "fp32s", "fp16s", "fp16s64"])
@pytest.mark.parametrize("name,zc", SPLIT_PARAMS)
def test_record_call_equals_split_steps(name, zc, precision):
    wl, shape, over = SPLIT_CASES[name]
    w = case(wl, shape, **over)
    Q, rho_in = w["params"]["Q"], w["params"]["rho_in"]
    _flush(f"[record vs split] {name} {precision} shape={shape} zchunk={zc}")
    a = gpu_for(w, precision, kernel="record")
    a.set_zchunk(zc)
    b = gpu_for(w, precision, kernel="split")
    for n in (7, 1, 5):  # calls of several steps, and one (the split step itself)
        a.step(n)
        b.step(n)
        e = e_pop(a.populations().cpu().numpy(), b.populations().cpu().numpy(), Q, rho_in,
                  w["solid"])
        tol = {"fp64": 1e-13, "fp32s": 1e-6, "fp16s": 5e-3, "fp16s64": 5e-3}[precision]
        assert e < tol, (n, e)
    oa, ob = a.observables(), b.observables()
    assert oa["step"] == ob["step"] == 13
    soft = w["params"]["site_rule"] == "soft"
    if precision.startswith("fp16s"):
        # half records and half populations round differently (stochastically, with other
        # random bits), so a site decision near the threshold may differ: the sink totals
        # agree to the share of one site-step
        _flush(f"  e_pop {e:.2e}, site-steps {oa['site_steps']} / {ob['site_steps']}")
        assert abs(oa["site_steps"] - ob["site_steps"]) <= 0.01 * ob["site_steps"] + 2
        assert abs(oa["sink_total"] - ob["sink_total"]) <= (
            0.01 * abs(ob["sink_total"]) + 2.0 * w["params"]["phi"] / w["params"]["sbar"])
    elif precision == "fp64":
        if soft:  # the carried ||F||, rounded in a different order
            assert float((a.carry - b.carry).abs().max()) < 1e-12
        else:
            assert bool((a.carry == b.carry).all())
        for k in ("n_sites", "site_steps"):
            assert oa[k] == ob[k], k
        assert abs(oa["sink_total"] - ob["sink_total"]) <= 1e-13 * abs(ob["sink_total"])
    else:
        assert oa["site_steps"] == ob["site_steps"]
        # soft weights pass rounding differences of ||F|| on amplified by 1 / kappa = 100
        rel = 1e-7 if soft else 1e-9
        assert abs(oa["sink_total"] - ob["sink_total"]) <= rel * abs(ob["sink_total"])
    a.close()
    b.close()


def test_automatic_choice_of_the_step_form():
    from paper_2412_14859_amd import cgevap
    w = case("sphere3d", (8, 8, 64), radius=3.0, phi=1e-3)
    for precision in ("fp64", "fp32s", "fp16s"):  # D3Q19 at unit tau: the record form
        s = gpu_for(w, precision)
        assert s.kernel_name() == "k_pull_record", precision
        s.close()
    w9 = case("drop2d", (1, 40, 52), radius=11.0, phi=1e-3)
    for precision in ("fp64", "fp32s", "fp16s"):  # D2Q9: the split step
        s = gpu_for(w9, precision)
        assert s.kernel_name() == "k_finish", precision
        s.close()
    w2 = case("sphere3d", (8, 8, 64), radius=3.0, phi=1e-3, tau=(1.0, 0.8))
    s = gpu_for(w2, "fp32s")
    assert s.kernel_name() != "k_pull_record"
    s.close()
    with pytest.raises(cgevap.CgeError):
        gpu_for(w2, "fp32s", kernel="record")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32s", 1e-5), ("fp16s", 5e-3),
                                           ("fp16s64", 5e-3)])
def test_z_marching_pull_against_the_oracle(precision, tol):
    """The benchmark's kernel pair (the z-marching pull, FP64, FP32 or half records) against
    the FP64 oracle directly, in calls of several steps: FP64 within the 1e-12 parity bar; with
    soft sites no site decision can flip between precisions, so FP32 storage stays within the
    1e-5 bar without imposing the oracle's masks, and half storage within 5e-3 (a few
    half-precision units of the largest scaled population, as the split step's half
    populations).  The shape spans ragged tiles in x and y and several planes."""
    w = case("sphere3d", (14, 16, 70), radius=5.0, phi=1e-3, site_rule="soft", kappa=0.01)
    Q, rho_in = w["params"]["Q"], w["params"]["rho_in"]
    _flush(f"[record {precision} vs oracle] d3q19 soft 14x16x70")
    ora = oracle_for(w)
    sim = gpu_for(w, precision, kernel="record")
    sim.set_zchunk(5)  # 14 planes: chunks of 5, 5 and 4
    worst = 0.0
    for _ in range(3):
        sim.step(5)
        ora.step(5)
        e = e_pop(sim.populations().cpu().numpy(), ora.populations(), Q, rho_in)
        worst = max(worst, e)
        assert e < tol, e
    _flush(f"  worst e_pop {worst:.3e}")
    og, oo = sim.observables(), ora.observables()
    assert abs(og["sink_total"] - oo["sink_total"]) <= tol * abs(oo["sink_total"])
    sim.close()
