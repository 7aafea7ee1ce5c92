"""Pins of the stored oracle record of the 64^3 drop over 10000 steps
(tests/golden/c3_downscale_64cube_oracle.txt, written by tests/golden/make_c3_downscale.py),
against what the method fixes (Sec. II.B):
  * total mass is conserved (the sink moves red to blue): mass_r + mass_b = N rho at every
    record, N = 64^3 nodes at unit density;
  * the red mass lost equals the sink (Eq. exchange) at every record;
  * with a uniform flux and hard sites every sink term is phi / Sbar, so the sink total is
    site-steps x phi / Sbar (Eq. relation), to the rounding of a sum of 1e8 terms;
  * sites are the S-fold layer around the interface: the site count per step over the
    interface area 4 pi R^2 of the equivalent sphere is Sbar within 5 %;
  * the equivalent radius (3V / 4 pi)^(1/3) falls by phi t / rho_l (Sec. III, the linear law
    at unit density ratio), within 1 % of the drop over the run."""
import math
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PHI, SBAR, N = 1e-5, 3.0, 64 ** 3


def _rows():
    rows, keys = [], None
    with open(os.path.join(HERE, "golden", "c3_downscale_64cube_oracle.txt")) as f:
        for line in f:
            if line.startswith("# step "):
                keys = line[2:].split()
            elif line.strip() and not line.startswith("#"):
                rows.append({k: float(v) for k, v in zip(keys, line.split())})
    return rows


@pytest.fixture(scope="module")
def rows():
    r = _rows()
    assert r[0]["step"] == 0 and r[-1]["step"] == 10000 and len(r) == 21
    return r


def test_total_mass_is_conserved(rows):
    # to the FP64 rounding of 10000 steps (the record drifts to 1.5e-12 of N)
    for r in rows:
        assert abs(r["mass_r"] + r["mass_b"] - N) <= 1e-11 * N, r["step"]


def test_red_mass_lost_equals_the_sink(rows):
    # against site-steps x phi / Sbar (within 1e-10 of it); the summed sink total, added in
    # node and step order, is itself up to 1.25e-9 off (next test)
    m0 = rows[0]["mass_r"]
    for r in rows[1:]:
        exact = r["site_steps"] * PHI / SBAR
        assert abs((m0 - r["mass_r"]) - exact) <= 1e-9 * exact, r["step"]


def test_sink_total_is_site_steps_times_phi_over_sbar(rows):
    for r in rows[1:]:
        exact = r["site_steps"] * PHI / SBAR
        assert abs(r["sink_total"] - exact) <= 1.1e-8 * exact, r["step"]


def test_sites_per_unit_interface_area(rows):
    for a, b in zip(rows[1:], rows[2:]):
        per_step = (b["site_steps"] - a["site_steps"]) / (b["step"] - a["step"])
        R = (3.0 * b["v_mass"] / (4.0 * math.pi)) ** (1.0 / 3.0)
        assert abs(per_step / (4.0 * math.pi * R * R) / SBAR - 1.0) < 0.05, b["step"]


def test_radius_follows_the_linear_law(rows):
    radius = [(3.0 * r["v_mass"] / (4.0 * math.pi)) ** (1.0 / 3.0) for r in rows]
    drop = radius[0] - radius[-1]
    law = PHI * 10000 / 1.0
    assert abs(drop - law) < 0.01 * law, (drop, law)
