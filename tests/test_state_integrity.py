"""Integrity trailer of saved states, on the host: a snapshot sealed by the documented format
(written out here independently of the library) passes cge_verify_state, and any corruption
of the covered bytes, the trailer or the parameters is reported as CGE_ECHECKPOINT.  The GPU
side (sealing on save, the check on load) is in tests/test_gpu_state.py."""
import ctypes as C
import struct

import numpy as np
import pytest

from paper_2412_14859_amd import cgevap, inputs

MASK = (1 << 64) - 1


def splitmix64_step(z):
    z = (z + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def fnv1a(h, data):
    for b in data:
        h = ((h ^ b) * 0x100000001B3) & MASK
    return h


def layout(cp):
    L = cgevap.lib()
    pb = L.cge_population_bytes(C.byref(cp))
    cb = cp.nx * cp.ny * cp.nz * (8 if cp.site_rule == 2 else 1)
    coff = (pb + 255) // 256 * 256
    toff = (coff + cb + 255) // 256 * 256
    return pb, cb, coff, toff


def checksum(regions):
    s, i = 0, 0
    for r in regions:
        r = bytes(r) + b"\0" * (-len(r) % 8)
        for k in range(0, len(r), 8):
            w = struct.unpack_from("<Q", r, k)[0]
            s = (s + splitmix64_step(w ^ ((i * 0xD6E8FEB86659FD93) & MASK))) & MASK
            i += 1
    return s


def fingerprint(cp):
    h = 0xCBF29CE484222325
    h = fnv1a(h, struct.pack("<6i", cp.lattice, cp.nx, cp.ny, cp.nz, cp.precision, cp.site_rule))
    h = fnv1a(h, struct.pack("<2d", cp.rho_in[0], cp.rho_in[1]))
    return fnv1a(h, struct.pack("<i", 1))


def sealed(cp, rng):
    pb, cb, coff, toff = layout(cp)
    assert cgevap.lib().cge_state_bytes(C.byref(cp)) == toff + 32
    snap = bytearray(rng.integers(0, 256, toff + 32, dtype=np.uint8).tobytes())  # padding: junk
    pops, carry = bytes(snap[:pb]), bytes(snap[coff:coff + cb])
    snap[toff:toff + 32] = struct.pack("<4Q", 0x5441545356454743, fingerprint(cp), pb + cb,
                                       checksum([pops, carry]))
    return snap


def verify(cp, snap):
    a = np.frombuffer(bytes(snap), dtype=np.uint8)
    return cgevap.lib().cge_verify_state(C.byref(cp), a.ctypes.data_as(C.c_void_p))


CASES = [  # regions whose sizes are not multiples of 8 bytes, and the FP64 soft-rule carry
    ("drop2d", (1, 3, 5), "fp16s", {}),
    ("sphere3d", (3, 4, 5), "fp32s", {}),
    ("sphere3d", (2, 3, 3), "fp64", {"site_rule": "soft"}),
]


@pytest.mark.parametrize("wl,shape,precision,over", CASES)
def test_sealed_snapshot_verifies_and_corruption_is_caught(wl, shape, precision, over):
    p = dict(inputs.workload(wl, shape=shape)["params"], **over)
    cp = cgevap.make_params(p, precision)
    rng = np.random.default_rng(3)
    snap = sealed(cp, rng)
    pb, cb, coff, toff = layout(cp)
    assert verify(cp, snap) == cgevap.OK
    # the padding between the regions is not covered
    if coff > pb:
        s2 = bytearray(snap)
        s2[pb] ^= 0xFF
        assert verify(cp, s2) == cgevap.OK
    # one bit in the populations (first, middle and last byte), in the site data, in the trailer
    for pos in (0, pb // 2, pb - 1, coff, coff + cb - 1, toff, toff + 8, toff + 16, toff + 24):
        s2 = bytearray(snap)
        s2[pos] ^= 0x04
        assert verify(cp, s2) == cgevap.ECHECKPOINT, pos
    # two 8-byte words swapped
    s2 = bytearray(snap)
    s2[0:8], s2[8:16] = snap[8:16], snap[0:8]
    if snap[0:8] != snap[8:16]:
        assert verify(cp, s2) == cgevap.ECHECKPOINT
    # a snapshot of other parameters with the same layout (another density ratio)
    cp2 = cgevap.make_params(dict(p, rho_in=(1.0, 0.5)), precision)
    assert layout(cp2) == layout(cp)
    assert verify(cp2, snap) == cgevap.ECHECKPOINT
    assert cgevap.lib().cge_verify_state(C.byref(cp), None) == cgevap.EINVAL
