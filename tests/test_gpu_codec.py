"""FP16 storage rounds stochastically: a value between two half numbers is stored as the
upper one with probability equal to its distance from the lower one over their spacing, so
the expected stored value is the value itself.

Checked through the import path (cge_set_populations), which rounds with the same routine as
the step kernels.  The populations are chosen so that the colour-blind channel is exactly
representable (f^r + f^b = t_i(alpha_b) rho_b^in, so ft_i = 0) and the colour difference
dd_i = f^r - f^b = v carries the value; the decoded f^r - f^b is then the stored dd_i.
Over 19 x 16^3 slots and four seeds every stored value is one of the two half numbers around
v, and their mean is v within 6 standard errors of the rounding noise, in the normal and
subnormal half ranges and below the smallest subnormal."""
import numpy as np
import pytest

from paper_2412_14859_amd import cgevap, inputs

pytestmark = pytest.mark.gpu


def _half_neighbours(v):
    """The half numbers below and above |v| (with v's sign), and their spacing."""
    a = abs(v)
    sp = 2.0 ** (np.floor(np.log2(a)) - 10) if a >= 2.0 ** -14 else 2.0 ** -24
    lo = np.floor(a / sp) * sp
    return np.sign(v) * lo, np.sign(v) * (lo + sp), sp


@pytest.mark.parametrize("v", [0.1234567, 3.0e-3 + 1.7e-7, 2.0e-5 + 3.1e-9, 4.0e-8, 1.3e-8,
                               -7.77e-6])
def test_fp16_storage_rounding_is_unbiased(v):
    shape = (16, 16, 16)
    Q = 19
    w = inputs.workload("sphere3d", shape=shape, radius=4.0)
    W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)  # t_i(alpha_b) at unit ratio
    f = np.empty((2, Q) + shape)
    f[0] = ((W + v) / 2.0)[:, None, None, None]
    f[1] = ((W - v) / 2.0)[:, None, None, None]
    lo, hi, sp = _half_neighbours(v)
    samples = []
    for seed in range(4):
        sim = cgevap.Simulation(w["params"], w["rho_r"], w["rho_b"], precision="fp16s",
                                seed=seed)
        sim.set_populations(f)
        got = sim.populations().cpu().numpy()
        sim.close()
        samples.append((got[0] - got[1]).ravel())
    d = np.concatenate(samples)
    # every stored value is one of the two half numbers around v
    near = np.minimum(np.abs(d - lo), np.abs(d - hi))
    assert near.max() < 1e-9 * sp
    p_up = float(np.mean(np.abs(d - hi) < np.abs(d - lo)))
    se = sp * np.sqrt(max(p_up * (1.0 - p_up), 1.0 / d.size)) / np.sqrt(d.size)
    print(f"v {v:.6e}: half numbers {lo:.6e} / {hi:.6e}, up {p_up:.4f} "
          f"(exact {(abs(v) - abs(lo)) / sp:.4f}), mean - v {d.mean() - v:.3e}, se {se:.3e}",
          flush=True)
    assert abs(d.mean() - v) < 6.0 * se + 1e-15 * abs(v)
