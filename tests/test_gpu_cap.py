"""Pinned cap on a cylindrical cavity (Sec. III, pinned cap), downscaled to 96^3 (ring radii
25 / 26.5, height 4): the cap stays pinned on the rim while its height follows
h0 - 2 phi t / rho0.  The full-size runs (192^3, both fluxes, Gamma 0.305 and 0.29) are
`bench.py --cap-benchmark`."""
import numpy as np
import pytest

from paper_2412_14859_amd import analytic, cgevap, inputs

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def test_cap_stays_pinned_and_follows_the_height_law():
    """phi = 3e-3, Gamma = 0.29.  Up to t* = 0.6 the height is within 4 % of the law
    (measured: 3.1 % at most, in the start-up transient at t* = 0.1, then falling to 0.1 %)
    and the contact radius drifts inwards but stays above 0.85 a0 (measured 0.886 at
    t* = 0.6).  The ring here is 1.5 nodes thick, half the full-size one, and holds the
    contact line less firmly: a / a0 passes 0.95 near t* = 0.2 instead of 0.4-0.6."""
    w = inputs.workload("cap3d", shape=(96, 96, 96))
    p = dict(w["params"], phi=0.0, gamma=0.29)
    top, zp = w["cavity_top"], w["cavity_height"] + 1
    _flush("[cap] 96^3 ring 25/26.5 height 4, phi 3e-3, Gamma 0.29")
    sim = cgevap.Simulation(p, w["rho_r"], w["rho_b"], solid=w["solid"],
                            phi_field=np.zeros(p["shape"]), precision="fp32s")

    def measure():
        rr = sim.fields()["rho_r"]
        return analytic.cap_height(rr, top), analytic.contact_radius(rr, zp), float(rr.max())

    sim.step(3000)
    h0, a0, rho0 = measure()
    phi = 3e-3
    sim.set_counters()
    sim.phi_field.fill_(phi)
    te = h0 * rho0 / (2 * phi)
    ts, hs, as_ = [0.0], [h0], [a0]
    for k in range(1, 13):
        sim.step(int(0.05 * te))
        ts.append(k * int(0.05 * te))
        h, a, _ = measure()
        hs.append(h)
        as_.append(a)
    obs = sim.observables()
    sim.close()
    ts, hs, as_ = np.array(ts, float), np.array(hs), np.array(as_)
    tstar = ts / te
    lin = analytic.cap_height_constant(ts, h0, phi, rho0)
    err = np.abs(hs - lin) / lin
    _flush(f"  h0 {h0:.2f} a0 {a0:.2f} rho0 {rho0:.4f}; t*: h err, a/a0: " +
           " ".join(f"{q:.2f}:{e:.4f},{r:.3f}" for q, e, r in zip(tstar, err, as_ / a0)))
    assert 40.0 < h0 < 50.0 and 25.0 < a0 < 30.0
    assert np.all(np.diff(hs) < 0)
    assert err.max() < 0.04
    assert np.all(as_ / a0 > 0.85) and np.all(np.diff(as_) <= 0.05)
    assert obs["site_steps"] > 0
