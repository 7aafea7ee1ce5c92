"""cge_observables_noalloc (the observables with the library's static scratch, for callers that
cannot allocate) against cge_observables of a context on the same state: two calls in a row,
the second on a smaller grid than the first, so the second reads scratch the first left
behind.  Integer fields must be equal, floating-point fields within 1e-13 relative (the same
kernels run in the same order, so they are expected bit-equal)."""
import ctypes as C

import pytest

from tests.helpers import case, gpu_for

pytestmark = pytest.mark.gpu

STATE_FIELDS_INT = ("n_sites", "v_half", "n_negative")
STATE_FIELDS_FP = ("mass_r", "mass_b", "v_mass", "perim_sites", "perim_grad", "max_u", "p_in",
                   "p_out", "max_rho_r")


def _flush(msg):
    print(msg, flush=True)


def _compare(sim, label):
    import torch
    from paper_2412_14859_amd import cgevap
    ref = sim.observables()
    cp = cgevap.make_params(sim.params, sim.precision)
    pb = cgevap.lib().cge_population_bytes(C.byref(cp))
    snap = sim.save_state()
    off = (pb + 255) & ~255
    pop, carry = snap[:pb], snap[off:]
    out = cgevap.observables_noalloc(sim.params, sim.precision, pop, carry, sim.flags,
                                     stream=torch.cuda.current_stream(sim.device))
    got = cgevap.obs_from_device(out)
    bitwise = all(got[k] == ref[k] for k in STATE_FIELDS_INT + STATE_FIELDS_FP)
    _flush(f"  {label}: mass_r {got['mass_r']:.15e} vs {ref['mass_r']:.15e}, "
           f"sites {got['n_sites']} vs {ref['n_sites']}, bit-equal {bitwise}")
    for k in STATE_FIELDS_INT:
        assert got[k] == ref[k], (label, k, got[k], ref[k])
    for k in STATE_FIELDS_FP:
        assert abs(got[k] - ref[k]) <= 1e-13 * max(1.0, abs(ref[k])), (label, k, got[k], ref[k])
    assert got["step"] == 0 and got["site_steps"] == 0 and got["sink_total"] == 0.0
    assert ref["n_sites"] > 0


def test_noalloc_observables_match_the_context_two_calls():
    # first call: D3Q19 cap on a wall at density ratio 10 with a flux field (solid nodes, the
    # wetting pass), FP32 storage; second call: a smaller D2Q9 drop in FP64
    w1 = case("sessile3d", (24, 40, 70), radius=9.0, phi=1e-3)
    w2 = case("drop2d", (1, 30, 50), radius=8.0, phi=1e-3, site_rule="grad", gamma=0.305)
    _flush("[noalloc] sessile3d 24x40x70 fp32s, then drop2d 30x50 fp64")
    s1 = gpu_for(w1, "fp32s")
    s1.step(7)
    _compare(s1, "first call (67200 nodes)")
    s2 = gpu_for(w2, "fp64")
    s2.step(5)
    _compare(s2, "second call (1500 nodes)")
    s1.close()
    s2.close()
