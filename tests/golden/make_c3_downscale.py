"""Writes tests/golden/c3_downscale_64cube_oracle.txt: the FP64 oracle's observables on the
64^3 downscale of the D3Q19 256^3 drop workload (R = 16, the drop centre half a node off the
box centre, parameters of the full workload: unit density ratio, tau 1, surface-tension
parameter 5e-4, beta 0.7, phi 1e-5, Gamma 0.305, S = 3), every 500 steps over 10000 steps.
Only the oracle and the seeded input generator run here.

    python tests/golden/make_c3_downscale.py [threads]

Takes about four minutes on eight cores."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_2412_14859_amd import inputs  # noqa: E402

STEPS, EVERY = 10000, 500
OFFSET = (0.5, 0.5, 0.5)
KEYS = ("v_mass", "mass_r", "mass_b", "sink_total", "site_steps", "n_sites")


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else len(os.sched_getaffinity(0))
    w = inputs.workload("sphere3d", shape=(64, 64, 64), radius=16.0, offset=OFFSET)
    o = Oracle(w["params"], solid=w["solid"], phi_field=w["phi_field"])
    o.set_threads(threads)
    o.init_equilibrium(w["rho_r"], w["rho_b"])
    rows = []
    for step in range(0, STEPS + 1, EVERY):
        if step:
            o.step(EVERY)
        ob = o.observables()
        rows.append((step,) + tuple(ob[k] for k in KEYS))
        print(f"step {step}: v_mass {ob['v_mass']:.12f}", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_downscale_64cube_oracle.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle, D3Q19 64^3 drop R = 16 centred at (32.5, 32.5, 32.5), the 256^3 drop\n")
        f.write("# workload scaled 1/4 (unit density ratio, tau 1, beta 0.7, phi 1e-5, Gamma 0.305,\n")
        f.write("# Sbar 3); written by tests/golden/make_c3_downscale.py\n")
        f.write("# step " + " ".join(KEYS) + "\n")
        for r in rows:
            f.write(f"{r[0]} " + " ".join(repr(float(v)) if isinstance(v, float) else str(v)
                                         for v in r[1:]) + "\n")
    print(out)


if __name__ == "__main__":
    main()
