"""ctypes binding of the FP64 CPU oracle (oracle/cg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  Nothing on the product path imports it.

Arrays are numpy float64 in the oracle's storage order: populations [2][Q][nz][ny][nx]
(component 0 = red, the evaporating fluid), scalar fields [nz][ny][nx], vector fields
[D][nz][ny][nx].
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class OraParams(C.Structure):
    _fields_ = [("Q", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("rho_in", C.c_double * 2), ("tau", C.c_double * 2), ("sigma", C.c_double),
                ("beta", C.c_double), ("phi", C.c_double), ("sbar", C.c_double),
                ("gamma", C.c_double), ("site_rule", C.c_int), ("kappa", C.c_double),
                ("recolor_fade", C.c_double)]


class OraObs(C.Structure):
    _fields_ = [("step", C.c_longlong), ("n_sites", C.c_longlong), ("v_half", C.c_longlong),
                ("n_negative", C.c_longlong), ("site_steps", C.c_longlong),
                ("mass_r", C.c_double), ("mass_b", C.c_double), ("sink_total", C.c_double),
                ("v_mass", C.c_double), ("perim_sites", C.c_double), ("perim_grad", C.c_double),
                ("max_u", C.c_double), ("p_in", C.c_double), ("p_out", C.c_double),
                ("max_rho_r", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        src = _build.SRC
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = C.CDLL(path)
        P = C.POINTER
        dp = P(C.c_double)
        up = P(C.c_ubyte)
        L.ora_create.restype = C.c_void_p
        L.ora_create.argtypes = [P(OraParams), up, dp]
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_init_equilibrium.argtypes = [C.c_void_p, dp, dp, dp]
        L.ora_set_populations.argtypes = [C.c_void_p, dp]
        L.ora_get_populations.argtypes = [C.c_void_p, dp]
        L.ora_set_fmag.argtypes = [C.c_void_p, dp]
        L.ora_get_fmag.argtypes = [C.c_void_p, dp]
        L.ora_recompute_fmag.argtypes = [C.c_void_p]
        L.ora_set_counters.argtypes = [C.c_void_p, C.c_longlong, C.c_longlong, C.c_double]
        L.ora_step.argtypes = [C.c_void_p, C.c_longlong, up, up]
        L.ora_set_threads.argtypes = [C.c_void_p, C.c_int]
        L.ora_set_height_flux.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double,
                                          C.c_longlong]
        L.ora_get_phi_field.argtypes = [C.c_void_p, dp]
        L.ora_set_outlet.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double]
        L.ora_fields.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.ora_observables.argtypes = [C.c_void_p, P(OraObs)]
        L.ora_tables.argtypes = [C.c_int, dp, dp, dp, dp, P(C.c_int), P(C.c_int), dp]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_ubyte))


def tables(Q):
    """Lattice tables of the oracle: dict of W, A, B, C (Q,), c (Q,3) int, opp (Q,), zeta."""
    W, A, B, Cc = (np.zeros(Q) for _ in range(4))
    c = np.zeros(3 * Q, dtype=np.int32)
    opp = np.zeros(Q, dtype=np.int32)
    zeta = C.c_double()
    rc = lib().ora_tables(Q, _dp(W), _dp(A), _dp(B), _dp(Cc),
                          c.ctypes.data_as(C.POINTER(C.c_int)),
                          opp.ctypes.data_as(C.POINTER(C.c_int)), C.byref(zeta))
    if rc:
        raise ValueError(f"no lattice with Q={Q}")
    return {"W": W, "A": A, "B": B, "C": Cc, "c": c.reshape(Q, 3), "opp": opp,
            "zeta": zeta.value}


class Oracle:
    """One oracle simulation.  `params` keys: Q, shape (nz, ny, nx), rho_in, tau, sigma,
    beta, phi, sbar, gamma, site_rule ('grad', 'phase' or 'soft'), kappa (soft rule width),
    recolor_fade (optional regularisation width of cos(theta); 0, the default, is Eq. recolor)."""

    def __init__(self, params, solid=None, phi_field=None):
        Q = int(params["Q"])
        nz, ny, nx = params["shape"]
        p = OraParams()
        p.Q, p.nx, p.ny, p.nz = Q, nx, ny, nz
        p.rho_in[0], p.rho_in[1] = params.get("rho_in", (1.0, 1.0))
        p.tau[0], p.tau[1] = params.get("tau", (1.0, 1.0))
        p.sigma = params["sigma"]
        p.beta = params["beta"]
        p.phi = params.get("phi", 0.0)
        p.sbar = params.get("sbar", 3.0)
        p.gamma = params["gamma"]
        p.site_rule = {"grad": 0, "phase": 1, "soft": 2}[params.get("site_rule", "grad")]
        p.kappa = params.get("kappa", 0.01)
        p.recolor_fade = params.get("recolor_fade", 0.0)
        self.Q, self.shape, self.N = Q, (nz, ny, nx), nx * ny * nz
        self.D = 2 if Q == 9 else 3
        self._solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
        self._phi = None if phi_field is None else np.ascontiguousarray(phi_field, np.float64)
        self._ctx = lib().ora_create(C.byref(p), _up(self._solid), _dp(self._phi))
        if not self._ctx:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        if getattr(self, "_ctx", None):
            lib().ora_destroy(self._ctx)
            self._ctx = None

    def init_equilibrium(self, rho_r, rho_b, u=None):
        rr = np.ascontiguousarray(rho_r, np.float64)
        rb = np.ascontiguousarray(rho_b, np.float64)
        uu = None if u is None else np.ascontiguousarray(u, np.float64)
        lib().ora_init_equilibrium(self._ctx, _dp(rr), _dp(rb), _dp(uu))

    def populations(self):
        f = np.empty((2, self.Q) + self.shape)
        lib().ora_get_populations(self._ctx, _dp(f))
        return f

    def set_populations(self, f):
        f = np.ascontiguousarray(f, np.float64)
        assert f.size == 2 * self.Q * self.N
        lib().ora_set_populations(self._ctx, _dp(f))

    def fmag(self):
        g = np.empty(self.shape)
        lib().ora_get_fmag(self._ctx, _dp(g))
        return g

    def set_fmag(self, g):
        g = np.ascontiguousarray(g, np.float64)
        lib().ora_set_fmag(self._ctx, _dp(g))

    def recompute_fmag(self):
        lib().ora_recompute_fmag(self._ctx)

    def set_height_flux(self, phi_s, K, h_scale, every=1):
        """Height-dependent flux phi_s / (K + h / h_scale) from the column heights (Eq.
        heated), refreshed every `every` steps; every <= 0 switches it off."""
        if lib().ora_set_height_flux(self._ctx, phi_s, K, h_scale, every) != 0:
            raise ValueError("invalid height-flux parameters")

    def set_outlet(self, lo, hi, rho_out):
        """Blue pressure outlets on the end planes of the last lattice axis."""
        if lib().ora_set_outlet(self._ctx, int(bool(lo)), int(bool(hi)), rho_out) != 0:
            raise ValueError("invalid outlet parameters")

    def phi_field(self):
        out = np.empty(self.shape)
        if lib().ora_get_phi_field(self._ctx, _dp(out)) != 0:
            return None
        return out

    def set_threads(self, n):
        """OpenMP threads of the per-node loops (results do not depend on it)."""
        if lib().ora_set_threads(self._ctx, int(n)) != 0:
            raise ValueError("threads must be >= 1")

    def set_counters(self, step=0, site_steps=0, sink_total=0.0):
        lib().ora_set_counters(self._ctx, step, site_steps, sink_total)

    def step(self, n=1, log_masks=False, masks=None):
        """Advance n steps.  log_masks returns the site masks used, [n][nz][ny][nx] uint8;
        masks (same shape) replaces the site selection."""
        log = np.zeros((n,) + self.shape, np.uint8) if log_masks else None
        mi = None if masks is None else np.ascontiguousarray(masks, np.uint8)
        if mi is not None:
            assert mi.shape[0] >= n
        lib().ora_step(self._ctx, n, _up(log), _up(mi))
        return log

    def fields(self):
        rr, rb, rN, g = (np.empty(self.shape) for _ in range(4))
        u = np.empty((self.D,) + self.shape)
        lib().ora_fields(self._ctx, _dp(rr), _dp(rb), _dp(u), _dp(rN), _dp(g))
        return {"rho_r": rr, "rho_b": rb, "u": u, "rhoN": rN, "gradmag": g}

    def observables(self):
        o = OraObs()
        lib().ora_observables(self._ctx, C.byref(o))
        return o.as_dict()
