"""Shared helpers of the GPU tests: oracle/GPU pairs on the same seeded inputs, error metrics."""
import numpy as np

from oracle.oracle import Oracle, tables
from paper_2412_14859_amd import inputs


def alphas(Q, rho_in):
    W0 = 4.0 / 9.0 if Q == 9 else 1.0 / 3.0
    rmin = min(rho_in)
    return [W0 if r == rmin else 1.0 - (1.0 - W0) / (r / rmin) for r in rho_in]


def pop_scale(Q, rho_in):
    """t_i(alpha_k) rho_k^in per (k, i): the normaliser of the population error."""
    t = tables(Q)
    a = alphas(Q, rho_in)
    return np.stack([(t["A"] + t["B"] * a[k]) * rho_in[k] for k in range(2)])


def e_pop(f_gpu, f_ora, Q, rho_in, solid=None):
    """max_{k,i,x} |f_gpu - f_oracle| / (t_i(alpha_k) rho_k^in) over fluid nodes."""
    s = pop_scale(Q, rho_in)[:, :, None, None, None]
    err = np.abs(np.asarray(f_gpu) - np.asarray(f_ora)) / s
    if solid is not None:
        err = err[:, :, solid == 0]
    return float(err.max())


# Drop-shaped workloads whose centre can move off the box centre (inputs.workload's offset).
OFFSET_WORKLOADS = ("drop2d", "sphere3d", "adjoint2d", "sessile3d", "hemisphere3d",
                    "hemisphere2d", "contrast3d", "cap3d")
# Downscaled drops sit half a node off the box centre, so that no symmetry saddle of the phase
# field (between a drop and its periodic images, or at the centre of a small drop) falls on a
# node: there the gradient vanishes inside a mixture and the recolouring angle of Eq. recolor
# is rounding noise, which the two sides of a parity test need not share.
HALF_NODE = (0.5, 0.5, 0.5)


def case(name, shape, **over):
    """A workload with parameter overrides (Q, shape set by the workload).  shape None is the
    full-size workload as specified (centred); a downscaled drop workload takes offset
    HALF_NODE unless an offset is given."""
    if shape is not None and name in OFFSET_WORKLOADS:
        over.setdefault("offset", HALF_NODE)
    kw = {k: over.pop(k) for k in ("radius", "phi", "seed", "offset") if k in over}
    w = inputs.workload(name, shape=shape, **kw)
    w["params"].update(over)
    return w


def oracle_for(w):
    o = Oracle(w["params"], solid=w["solid"], phi_field=w["phi_field"])
    o.init_equilibrium(w["rho_r"], w["rho_b"])
    return o


def gpu_for(w, precision="fp64", kernel="auto", seed=0):
    from paper_2412_14859_amd import cgevap
    return cgevap.Simulation(w["params"], w["rho_r"], w["rho_b"], solid=w["solid"],
                             phi_field=w["phi_field"], precision=precision, kernel=kernel,
                             seed=seed)
