"""The fused single-pass step with plane walls (every z-plane wholly solid or wholly fluid, no
solid plane with fluid on both sides): against the FP64 oracle every call, with z-chunks that
start and end on and next to the walls (a chunk of one plane, chunks ending on the lid, a
march that starts below a lid), the general collision at density ratio 10 with tau_v = 0.6
(the sessile-drop workload), a channel one fluid plane high; against the two-pass step at
FP32 and FP16 storage; and the choice of the step form (solid nodes that are not plane walls
fall back to the two-pass step, or are refused when the fused step is asked for)."""
import numpy as np
import pytest

from paper_2412_14859_amd import cgevap
from tests.helpers import case, e_pop, gpu_for, oracle_for

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


CASES = {
    # name: (workload, shape (z, y, x), overrides)
    "flat": ("flat3d", (21, 12, 70), dict(phi=1e-3)),
    "sessile_ratio10": ("sessile3d", (14, 18, 70), dict(radius=6.0, phi=1e-3)),
    "hemisphere_field": ("hemisphere3d", (24, 20, 70), dict(radius=6.0, phi=1e-3)),
}
# planes per chunk: one plane; two; five (ragged last chunk); nz - 1 (the second chunk is the
# lid alone); automatic
ZCHUNKS = (1, 2, 5, -1, 0)


@pytest.mark.parametrize("zc", ZCHUNKS)
@pytest.mark.parametrize("name", list(CASES))
def test_fused_plane_walls_match_the_oracle_fp64(name, zc):
    wl, shape, over = CASES[name]
    w = case(wl, shape, **over)
    zchunk = shape[0] - 1 if zc == -1 else zc
    _flush(f"[fused walls fp64] {name} shape={shape} zchunk={zchunk}")
    ora = oracle_for(w)
    sim = gpu_for(w, "fp64", kernel="fused")
    assert sim.kernel_name() == "k_fused"
    sim.set_zchunk(zchunk)
    for calls in range(2):
        sim.step(3)
        ora.step(3)
        e = e_pop(sim.populations().cpu().numpy(), ora.populations(), 19, w["params"]["rho_in"],
                  w["solid"])
        assert e < 1e-12, (calls, e)
        mask = (ora.fmag() > w["params"]["gamma"]).astype(np.uint8)
        mask[w["solid"] != 0] = 0
        assert np.array_equal(sim.carry.cpu().numpy(), mask), calls
    og, oo = sim.observables(), ora.observables()
    for k in ("n_sites", "site_steps", "step"):
        assert og[k] == oo[k], k
    for k in ("mass_r", "mass_b", "sink_total"):
        assert abs(og[k] - oo[k]) <= 1e-12 * max(1.0, abs(oo[k])), (k, og[k], oo[k])
    assert og["site_steps"] > 0
    sim.close()


def test_channel_one_fluid_plane_high():
    """Floor at z = 0, lid at z = 2: the one fluid plane bounces back on both sides, and both
    walls take their wetting values from it."""
    w = case("flat3d", (3, 12, 70), phi=1e-3)
    _flush("[fused walls fp64] channel nz = 3")
    ora = oracle_for(w)
    sim = gpu_for(w, "fp64", kernel="fused")
    assert sim.kernel_name() == "k_fused"
    sim.step(4)
    ora.step(4)
    e = e_pop(sim.populations().cpu().numpy(), ora.populations(), 19, w["params"]["rho_in"],
              w["solid"])
    assert e < 1e-12, e
    sim.close()


@pytest.mark.parametrize("precision,tol", [("fp32s", 1e-6), ("fp16s", 2e-2), ("fp16s64", 1e-6)])
def test_fused_plane_walls_match_twopass(precision, tol):
    """The same arithmetic as the two-pass step: states agree to the rounding of the storage
    (and of FP64 sums in another order); with FP64 arithmetic (FP32 storage, and FP16
    storage with fp16_arith64) they agree bitwise (measured 0), with FP32 arithmetic on FP16
    storage to 8.8e-4."""
    w = case("sessile3d", (14, 18, 70), radius=6.0, phi=1e-3)
    _flush(f"[fused vs twopass, walls] {precision}")
    sims = [gpu_for(w, precision, kernel=k, seed=7) for k in ("twopass", "fused")]
    assert sims[1].kernel_name() == "k_fused"
    for s in sims:
        s.step(9)
    e = e_pop(sims[0].populations().cpu().numpy(), sims[1].populations().cpu().numpy(), 19,
              w["params"]["rho_in"], w["solid"])
    _flush(f"  e_pop(fused, twopass) = {e:.3e}")
    assert e < tol, e
    for s in sims:
        s.close()


def test_step_form_choice_with_walls():
    # tau != 1 with plane walls: the fused step; with the cavity's mixed planes: two-pass
    w = case("sessile3d", (14, 18, 70), radius=6.0, phi=1e-3)
    s = gpu_for(w, "fp32s")
    assert s.kernel_name() == "k_fused"
    s.close()
    wc = case("cap3d", (24, 32, 70), radius=9.0, phi=1e-3)
    wc["params"]["tau"] = (1.0, 0.8)
    s = gpu_for(wc, "fp32s")
    assert s.kernel_name() == "k_collide"
    s.close()
    with pytest.raises(cgevap.CgeError) as e:
        gpu_for(wc, "fp32s", kernel="fused")
    assert e.value.status == cgevap.EUNSUPPORTED
    # a single solid plane with fluid on both sides: not plane walls either
    wf = case("flat3d", (12, 12, 70), phi=1e-3)
    solid = np.zeros_like(wf["solid"])
    solid[0] = 1
    wf["solid"] = solid
    wf["rho_r"], wf["rho_b"] = wf["rho_r"].copy(), wf["rho_b"].copy()
    wf["rho_r"][-1], wf["rho_b"][-1] = wf["rho_r"][-2], wf["rho_b"][-2]  # the old lid: fluid
    wf["params"]["tau"] = (1.0, 0.8)
    s = gpu_for(wf, "fp32s")
    assert s.kernel_name() == "k_collide"
    s.close()
