"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every symbol
the header declares, validates parameters before touching a device, and its lattice
tables agree with the oracle's independently written ones."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.oracle import tables as oracle_tables
from paper_2412_14859_amd import cgevap, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "cgevap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cge_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = cgevap.lib()
    names = header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert sorted(cgevap.EXPORTS) == names


def _params(**over):
    p = cgevap.make_params(inputs.workload("drop2d", shape=(1, 8, 8))["params"])
    for k, v in over.items():
        if k in ("tau", "rho_in"):
            getattr(p, k)[0] = v
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("over", [dict(lattice=7), dict(nx=0), dict(nz=2), dict(tau=0.5),
                                  dict(rho_in=0.0), dict(beta=1.5), dict(sbar=0.5),
                                  dict(precision=3), dict(site_rule=3), dict(kernel=9),
                                  dict(kernel=5), dict(kernel=-1),
                                  dict(site_rule=2, kappa=0.0), dict(site_rule=2, kappa=float("nan")),
                                  dict(sigma=-1.0), dict(phi=float("nan")),
                                  dict(gamma=float("inf")),
                                  # FP64 arithmetic on half storage: 0 or 1, FP16S only
                                  dict(fp16_arith64=1), dict(precision=1, fp16_arith64=1),
                                  dict(precision=2, fp16_arith64=2)])
def test_invalid_parameters_are_rejected_on_the_host(over):
    L = cgevap.lib()
    p = _params(**over)
    ctx = C.c_void_p()
    assert L.cge_create(C.byref(p), None, C.byref(ctx)) == cgevap.EINVAL
    assert ctx.value is None
    assert L.cge_population_bytes(C.byref(p)) == 0


@pytest.mark.parametrize("kernel", ["auto", "twopass", "fused", "split", "record"])
def test_every_step_form_passes_host_validation(kernel):
    """The binding's kernel names map onto the header's enumeration: each passes the host
    check (cge_population_bytes returns the population size without a device)."""
    L = cgevap.lib()
    p = _params(kernel=cgevap.KERNELS[kernel])
    assert L.cge_population_bytes(C.byref(p)) == 2 * 9 * 8 * 8 * 8
    assert cgevap.KERNELS["record"] == 4


def test_null_arguments():
    L = cgevap.lib()
    p = _params()
    assert L.cge_create(C.byref(p), None, None) == cgevap.EINVAL
    assert L.cge_create(None, None, C.byref(C.c_void_p())) == cgevap.EINVAL
    for fn in ("cge_step", "cge_reset_sites"):
        args = (None, 1) if fn == "cge_step" else (None,)
        assert getattr(L, fn)(*args) == cgevap.EINVAL
    assert L.cge_last_error(None) == b"NULL context"
    assert L.cge_set_outlet(None, 1, 1, C.c_double(1.0)) == cgevap.EINVAL
    assert L.cge_set_height_flux(None, C.c_double(1e-3), C.c_double(1.0), C.c_double(1.0),
                                 C.c_longlong(1)) == cgevap.EINVAL
    assert L.cge_set_site_threshold(None, C.c_double(0.3), C.c_double(0.0)) == cgevap.EINVAL
    L.cge_destroy(None)


def test_noalloc_observables_reject_on_the_host():
    """cge_observables_noalloc checks its parameters, pointers and the size of its static
    scratch before any device work (the pointers here are never dereferenced)."""
    L = cgevap.lib()
    fake = C.c_void_p(256)
    big = cgevap.make_params(inputs.workload("sphere3d", shape=(4, 4, 4))["params"], "fp32s")
    big.nx = big.ny = big.nz = 200           # 8e6 nodes + partials: beyond the 64 MiB
    assert L.cge_observables_noalloc(C.byref(big), fake, fake, None, None, fake) == \
        cgevap.ESCRATCH
    ok = cgevap.make_params(inputs.workload("sphere3d", shape=(4, 4, 4))["params"], "fp32s")
    ok.nx = ok.ny = ok.nz = 199              # the largest cube that fits; NULL out: EINVAL
    assert L.cge_observables_noalloc(C.byref(ok), fake, fake, None, None, None) == \
        cgevap.EINVAL
    assert L.cge_observables_noalloc(C.byref(ok), None, fake, None, None, fake) == \
        cgevap.EINVAL
    assert L.cge_observables_noalloc(C.byref(_params(tau=0.5)), fake, fake, None, None,
                                     fake) == cgevap.EINVAL
    assert L.cge_observables_noalloc(None, fake, fake, None, None, fake) == cgevap.EINVAL


def test_scratch_plan_and_caller_scratch_checks():
    """cge_scratch_bytes sizes the large per-node scratch (records only where the record form
    may run); cge_create_with_scratch refuses a missing, small or misaligned buffer before any
    device work."""
    L = cgevap.lib()
    w = inputs.workload("sphere3d", shape=(8, 8, 64))["params"]
    n = 8 * 8 * 64
    sizes = {}
    for prec in ("fp64", "fp32s", "fp16s"):
        for kernel in ("auto", "split", "twopass"):
            cp = cgevap.make_params(w, prec, kernel)
            sizes[prec, kernel] = L.cge_scratch_bytes(C.byref(cp))
            assert sizes[prec, kernel] >= n * (4 + 8), (prec, kernel)
    # the record form's 14 values per node (FP32 records, rows of 64 nodes: no padding here;
    # half records come in chunks of 128 nodes, so each 64-node row is padded to 128)
    assert sizes["fp32s", "auto"] - sizes["fp32s", "split"] == 14 * 4 * n
    assert sizes["fp64", "auto"] - sizes["fp64", "split"] == 14 * 8 * n
    assert sizes["fp16s", "auto"] - sizes["fp16s", "split"] == 14 * 2 * (8 * 8 * 128)
    assert L.cge_scratch_bytes(C.byref(_params(nx=0))) == 0
    cp = cgevap.make_params(w, "fp32s")
    need = L.cge_scratch_bytes(C.byref(cp))
    ctx = C.c_void_p()
    fake = C.c_void_p(1 << 20)
    assert L.cge_create_with_scratch(C.byref(cp), None, None, need, C.byref(ctx)) == cgevap.EINVAL
    assert L.cge_create_with_scratch(C.byref(cp), None, fake, need - 1, C.byref(ctx)) == \
        cgevap.EINVAL
    assert L.cge_create_with_scratch(C.byref(cp), None, C.c_void_p((1 << 20) + 8), need,
                                     C.byref(ctx)) == cgevap.EINVAL
    assert ctx.value is None


def test_population_bytes():
    L = cgevap.lib()
    for prec, b in (("fp64", 8), ("fp32s", 4), ("fp16s", 2)):
        p = cgevap.make_params(inputs.workload("sphere3d", shape=(4, 5, 6))["params"], prec)
        assert L.cge_population_bytes(C.byref(p)) == 2 * 19 * 120 * b


@pytest.mark.parametrize("Q", [9, 19])
def test_lattice_tables_agree_with_oracle(Q):
    a = cgevap.lattice_tables(Q)
    b = oracle_tables(Q)
    assert np.array_equal(a["c"], b["c"])
    assert np.array_equal(a["opp"], b["opp"])
    for k in ("W", "A", "B", "C"):
        assert np.allclose(a[k], b[k], rtol=0, atol=1e-16), k
    assert abs(a["zeta"] - b["zeta"]) < 1e-15
    assert cgevap.lib().cge_lattice_tables(5, None, None, None, None, None, None, None) == \
        cgevap.EINVAL


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2412_14859_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, re.M), f
                assert "cg_oracle" not in src and "libcg_oracle" not in src, f
    bench = open(os.path.join(ROOT, "bench.py")).read() if os.path.exists(
        os.path.join(ROOT, "bench.py")) else ""
    # the benchmark may use the oracle only in its CPU-baseline leg
    for line in bench.splitlines():
        if "oracle" in line and "import" in line:
            assert "cpu_baseline" in bench
