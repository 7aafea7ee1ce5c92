"""Python binding of libcgevap.so (C-ABI in include/cgevap.h): argument marshalling only.

Every step of the path runs in the HIP kernels of the library; torch provides device
memory and the stream.  Importing this module does not need a GPU; creating a simulation
does, and fails loudly when the HIP library is missing or no GPU is visible.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcgevap.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSUPPORTED, ENUMERIC = 0, -1, -2, -3, -4, -5, -6
ECHECKPOINT, ESCRATCH = -7, -8
# "fp16s64": half storage (CGE_FP16S) with FP64 arithmetic (cge_params.fp16_arith64)
PRECISIONS = {"fp64": 0, "fp32s": 1, "fp16s": 2, "fp16s64": 2}
KERNELS = {"auto": 0, "twopass": 1, "fused": 2, "split": 3, "record": 4}
SITE_RULES = {"grad": 0, "phase": 1, "soft": 2}
ELEM_BYTES = {"fp64": 8, "fp32s": 4, "fp16s": 2, "fp16s64": 2}

# every symbol the header declares
EXPORTS = ["cge_create", "cge_scratch_bytes", "cge_create_with_scratch", "cge_population_bytes", "cge_bind", "cge_init_equilibrium",
           "cge_set_populations", "cge_get_populations", "cge_state_bytes", "cge_save_state",
           "cge_load_state", "cge_verify_state", "cge_adjoint_bytes", "cge_segment_bytes", "cge_forward_ckpt", "cge_backward",
           "cge_reset_sites", "cge_set_site_threshold", "cge_set_height_flux", "cge_set_outlet",
           "cge_set_counters", "cge_set_zchunk",
           "cge_timing_kernel", "cge_step", "cge_observables", "cge_observables_noalloc", "cge_fields", "cge_set_timing", "cge_timing",
           "cge_kernel_name", "cge_lattice_tables", "cge_copy_probe", "cge_last_error",
           "cge_destroy"]


class CgeParams(C.Structure):
    _fields_ = [("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("precision", C.c_int), ("rho_in", C.c_double * 2), ("tau", C.c_double * 2),
                ("sigma", C.c_double), ("beta", C.c_double), ("phi", C.c_double),
                ("sbar", C.c_double), ("gamma", C.c_double), ("kappa", C.c_double),
                ("site_rule", C.c_int),
                ("kernel", C.c_int), ("seed", C.c_ulonglong),
                ("recolor_fade", C.c_double), ("fp16_arith64", C.c_int)]


class CgeObs(C.Structure):
    _fields_ = [("step", C.c_longlong), ("n_sites", C.c_longlong), ("v_half", C.c_longlong),
                ("n_negative", C.c_longlong), ("site_steps", C.c_longlong),
                ("mass_r", C.c_double), ("mass_b", C.c_double), ("sink_total", C.c_double),
                ("v_mass", C.c_double), ("perim_sites", C.c_double), ("perim_grad", C.c_double),
                ("max_u", C.c_double), ("p_in", C.c_double), ("p_out", C.c_double),
                ("max_rho_r", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class CgeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libcgevap status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libcgevap.so (built in-tree by __graft_entry__.build() or build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                               "python -c 'import __graft_entry__; __graft_entry__.build()'")
        L = C.CDLL(LIB_PATH)
        vp, dp, P = C.c_void_p, C.POINTER(C.c_double), C.POINTER
        L.cge_create.argtypes = [P(CgeParams), vp, P(vp)]
        L.cge_scratch_bytes.argtypes = [P(CgeParams)]
        L.cge_scratch_bytes.restype = C.c_size_t
        L.cge_create_with_scratch.argtypes = [P(CgeParams), vp, vp, C.c_size_t, P(vp)]
        L.cge_population_bytes.argtypes = [P(CgeParams)]
        L.cge_population_bytes.restype = C.c_size_t
        L.cge_bind.argtypes = [vp, vp, vp, vp, vp, vp]
        L.cge_init_equilibrium.argtypes = [vp, vp, vp, vp]
        L.cge_set_populations.argtypes = [vp, vp]
        L.cge_get_populations.argtypes = [vp, vp]
        L.cge_state_bytes.argtypes = [P(CgeParams)]
        L.cge_state_bytes.restype = C.c_size_t
        L.cge_save_state.argtypes = [vp, vp]
        L.cge_load_state.argtypes = [vp, vp]
        L.cge_verify_state.argtypes = [P(CgeParams), vp]
        L.cge_adjoint_bytes.argtypes = [P(CgeParams)]
        L.cge_adjoint_bytes.restype = C.c_size_t
        L.cge_segment_bytes.argtypes = [P(CgeParams), C.c_int]
        L.cge_segment_bytes.restype = C.c_size_t
        L.cge_forward_ckpt.argtypes = [vp, C.c_longlong, C.c_int, P(vp)]
        L.cge_backward.argtypes = [vp, C.c_longlong, C.c_int, P(vp), vp, vp, vp, vp, vp, vp, dp]
        L.cge_reset_sites.argtypes = [vp]
        L.cge_set_site_threshold.argtypes = [vp, C.c_double, C.c_double]
        L.cge_set_height_flux.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_longlong]
        L.cge_set_outlet.argtypes = [vp, C.c_int, C.c_int, C.c_double]
        L.cge_set_counters.argtypes = [vp, C.c_longlong, C.c_longlong, C.c_double]
        L.cge_set_zchunk.argtypes = [vp, C.c_int]
        L.cge_step.argtypes = [vp, C.c_longlong]
        L.cge_observables.argtypes = [vp, P(CgeObs)]
        L.cge_observables_noalloc.argtypes = [P(CgeParams), vp, vp, vp, vp, vp]
        L.cge_fields.argtypes = [vp, vp, vp, vp, vp]
        L.cge_set_timing.argtypes = [vp, C.c_int]
        L.cge_timing.argtypes = [vp, dp, P(C.c_longlong)]
        L.cge_timing_kernel.argtypes = [vp, C.c_char_p, dp, P(C.c_longlong)]
        L.cge_kernel_name.argtypes = [vp]
        L.cge_kernel_name.restype = C.c_char_p
        L.cge_lattice_tables.argtypes = [C.c_int, dp, dp, dp, dp, P(C.c_int), P(C.c_int), dp]
        L.cge_copy_probe.argtypes = [vp, vp, C.c_size_t, vp]
        L.cge_last_error.argtypes = [vp]
        L.cge_last_error.restype = C.c_char_p
        L.cge_destroy.argtypes = [vp]
        L.cge_destroy.restype = None
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype or C.c_int
        _lib = L
    return _lib


def make_params(params, precision="fp64", kernel="auto", seed=0):
    """cge_params from a workload parameter dict (keys as in inputs.workload)."""
    Q = int(params["Q"])
    nz, ny, nx = params["shape"]
    p = CgeParams()
    p.lattice, p.nx, p.ny, p.nz = Q, nx, ny, nz
    p.precision = PRECISIONS[precision]
    p.rho_in[0], p.rho_in[1] = params.get("rho_in", (1.0, 1.0))
    p.tau[0], p.tau[1] = params.get("tau", (1.0, 1.0))
    p.sigma = params["sigma"]
    p.beta = params["beta"]
    p.phi = params.get("phi", 0.0)
    p.sbar = params.get("sbar", 3.0)
    p.gamma = params["gamma"]
    p.kappa = params.get("kappa", 0.01)
    p.site_rule = SITE_RULES[params.get("site_rule", "grad")]
    p.kernel = KERNELS[kernel]
    p.seed = seed
    p.recolor_fade = params.get("recolor_fade", 0.0)
    p.fp16_arith64 = 1 if precision == "fp16s64" else 0
    return p


def lattice_tables(Q):
    W, A, B, Cc = (np.zeros(Q) for _ in range(4))
    c = np.zeros(3 * Q, np.int32)
    opp = np.zeros(Q, np.int32)
    zeta = C.c_double()
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))  # noqa: E731
    st = lib().cge_lattice_tables(Q, dp(W), dp(A), dp(B), dp(Cc), ip(c), ip(opp), C.byref(zeta))
    if st != OK:
        raise CgeError(st, f"no lattice with Q={Q}")
    return {"W": W, "A": A, "B": B, "C": Cc, "c": c.reshape(Q, 3), "opp": opp, "zeta": zeta.value}


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Simulation:
    """One simulation on one GPU.  Buffers are torch tensors on `device`; all work is
    enqueued on torch's current stream of that device at construction time."""

    def __init__(self, params, rho_r, rho_b, u=None, solid=None, phi_field=None,
                 precision="fp64", kernel="auto", seed=0, device="cuda:0"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP path needs an MI355X")
        self.torch = torch
        self.device = torch.device(device)
        self.params = dict(params)
        self.precision = precision
        self.Q = int(params["Q"])
        self.D = 2 if self.Q == 9 else 3
        self.shape = tuple(params["shape"])
        self.N = int(np.prod(self.shape))
        L = lib()
        cp = make_params(params, precision, kernel, seed)
        nbytes = L.cge_population_bytes(C.byref(cp))
        if nbytes == 0:
            raise CgeError(EINVAL, "invalid parameters")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            ctx = C.c_void_p()
            # the context's large scratch is a torch allocation (caller-owned, so torch's
            # caching allocator reuses it across simulations)
            sb = L.cge_scratch_bytes(C.byref(cp))
            self.scratch = torch.empty(sb, dtype=torch.uint8, device=self.device)
            st = L.cge_create_with_scratch(C.byref(cp), C.c_void_p(self.stream.cuda_stream),
                                           _ptr(self.scratch), C.c_size_t(sb), C.byref(ctx))
            if st != OK:
                raise CgeError(st, "cge_create failed")
            self._ctx = ctx
            dev = self.device
            self.pop = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(2)]
            soft = params.get("site_rule") == "soft"
            self.carry = torch.zeros(self.shape, dtype=torch.float64 if soft else torch.uint8,
                                     device=dev)
            self.flags = None if solid is None else torch.as_tensor(
                np.ascontiguousarray(solid, np.uint8), device=dev)
            pdt = torch.float64 if precision == "fp64" else torch.float32
            self.phi_field = None if phi_field is None else torch.as_tensor(
                np.ascontiguousarray(phi_field), device=dev).to(pdt).contiguous()
            self._check(L.cge_bind(self._ctx, _ptr(self.pop[0]), _ptr(self.pop[1]),
                                   _ptr(self.carry), _ptr(self.flags), _ptr(self.phi_field)))
            self.init_equilibrium(rho_r, rho_b, u)

    # ----------------------------------------------------------------------------- plumbing
    def _check(self, st):
        if st != OK:
            msg = lib().cge_last_error(self._ctx).decode()
            raise CgeError(st, msg)

    def _dev64(self, a):
        t = self.torch.as_tensor(np.ascontiguousarray(a, np.float64) if isinstance(a, np.ndarray)
                                 else a, device=self.device)
        return t.to(self.torch.float64).contiguous()

    def close(self):
        if getattr(self, "_ctx", None):
            self.torch.cuda.synchronize(self.device)
            lib().cge_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------------------- C-ABI calls
    def init_equilibrium(self, rho_r, rho_b, u=None):
        rr, rb = self._dev64(rho_r), self._dev64(rho_b)
        uu = None if u is None else self._dev64(u)
        self._check(lib().cge_init_equilibrium(self._ctx, _ptr(rr), _ptr(rb), _ptr(uu)))
        self.torch.cuda.current_stream(self.device).synchronize()

    def step(self, n=1):
        self._check(lib().cge_step(self._ctx, int(n)))

    def observables(self):
        o = CgeObs()
        self._check(lib().cge_observables(self._ctx, C.byref(o)))
        return o.as_dict()

    def populations(self):
        f = self.torch.empty((2, self.Q) + self.shape, dtype=self.torch.float64,
                             device=self.device)
        self._check(lib().cge_get_populations(self._ctx, _ptr(f)))
        return f

    def set_populations(self, f):
        t = self._dev64(f)
        assert t.numel() == 2 * self.Q * self.N
        self._check(lib().cge_set_populations(self._ctx, _ptr(t)))
        self.torch.cuda.current_stream(self.device).synchronize()

    def save_state(self, out=None):
        """Raw snapshot (encoded populations + site mask) as a uint8 device tensor."""
        if out is None:
            cp = make_params(self.params, self.precision)
            out = self.torch.empty(lib().cge_state_bytes(C.byref(cp)), dtype=self.torch.uint8,
                                   device=self.device)
        self._check(lib().cge_save_state(self._ctx, _ptr(out)))
        return out

    def load_state(self, snap):
        """Load a snapshot; CgeError with status ECHECKPOINT if its integrity trailer does not
        match (the state is then unchanged)."""
        self._check(lib().cge_load_state(self._ctx, _ptr(snap)))

    def reset_sites(self):
        self._check(lib().cge_reset_sites(self._ctx))

    def set_height_flux(self, phi_s, K, h_scale, every=1):
        """Flux phi_s / (K + h / h_scale) from the drop height h of each column normal to the
        substrate (the last lattice axis), refreshed from the state every `every` steps;
        every <= 0 switches it off.  Writes the bound flux field (phi_field=...)."""
        self._check(lib().cge_set_height_flux(self._ctx, float(phi_s), float(K),
                                              float(h_scale), int(every)))

    def set_outlet(self, lo, hi, rho_out=1.0):
        """Blue pressure outlets on the end planes of the last lattice axis."""
        self._check(lib().cge_set_outlet(self._ctx, int(bool(lo)), int(bool(hi)),
                                         float(rho_out)))

    def set_site_threshold(self, gamma, kappa=0.0):
        self._check(lib().cge_set_site_threshold(self._ctx, float(gamma), float(kappa)))
        self.params["gamma"] = float(gamma)
        if kappa > 0:
            self.params["kappa"] = float(kappa)

    # ----------------------------------------------------------------------------- adjoint
    def _state_bytes(self):
        return lib().cge_state_bytes(C.byref(make_params(self.params, self.precision)))

    def forward_ckpt(self, nsteps, K):
        """Advance nsteps, keeping the state at steps 0, K, 2K, ... and the final state
        (device tensors)."""
        nck = (int(nsteps) + K - 1) // K + 1
        ck = [self.torch.empty(self._state_bytes(), dtype=self.torch.uint8, device=self.device)
              for _ in range(nck)]
        arr = (C.c_void_p * nck)(*[t.data_ptr() for t in ck])
        self._check(lib().cge_forward_ckpt(self._ctx, int(nsteps), int(K), arr))
        return ck

    def backward(self, ckpt, nsteps, K, dL_drhoN=None, per_step=False, dL_drho=None):
        """Gradients of a loss given by dL/drho^N and/or dL/drho of the state after nsteps
        (from the checkpoints of forward_ckpt).  Returns grad_phi [shape] (phi held over time),
        grad_phi_t [nsteps, shape] when per_step, and grad_gamma.  The simulation is left at
        the state after nsteps."""
        t = self.torch
        nck = len(ckpt)
        assert nck == (int(nsteps) + K - 1) // K + 1
        cp = make_params(self.params, self.precision)
        seg = t.empty(lib().cge_segment_bytes(C.byref(cp), int(K)), dtype=t.uint8,
                      device=self.device)
        work = t.empty(lib().cge_adjoint_bytes(C.byref(cp)), dtype=t.uint8, device=self.device)
        g = None if dL_drhoN is None else self._dev64(dL_drhoN).reshape(self.shape).contiguous()
        gr = None if dL_drho is None else self._dev64(dL_drho).reshape(self.shape).contiguous()
        gphi = t.empty(self.shape, dtype=t.float64, device=self.device)
        gpt = (t.empty((int(nsteps),) + self.shape, dtype=t.float64, device=self.device)
               if per_step else None)
        gg = C.c_double()
        arr = (C.c_void_p * nck)(*[c.data_ptr() for c in ckpt])
        self._check(lib().cge_backward(self._ctx, int(nsteps), int(K), arr, _ptr(seg), _ptr(work),
                                       _ptr(g), _ptr(gr), _ptr(gphi), _ptr(gpt), C.byref(gg)))
        return {"grad_phi": gphi, "grad_phi_t": gpt, "grad_gamma": gg.value}

    def set_zchunk(self, planes):
        """Planes per z-chunk of the record form's z-marching pull (0: automatic)."""
        self._check(lib().cge_set_zchunk(self._ctx, int(planes)))

    def set_counters(self, step=0, site_steps=0, sink_total=0.0):
        self._check(lib().cge_set_counters(self._ctx, step, site_steps, sink_total))

    def fields(self):
        t = self.torch
        rr, rb, rn = (t.empty(self.shape, dtype=t.float64, device=self.device) for _ in range(3))
        u = t.empty((self.D,) + self.shape, dtype=t.float64, device=self.device)
        self._check(lib().cge_fields(self._ctx, _ptr(rr), _ptr(rb), _ptr(u), _ptr(rn)))
        return {"rho_r": rr, "rho_b": rb, "u": u, "rhoN": rn}

    def set_timing(self, on):
        self._check(lib().cge_set_timing(self._ctx, 1 if on else 0))

    def timing(self):
        ms, n = C.c_double(), C.c_longlong()
        self._check(lib().cge_timing(self._ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def timing_kernel(self, name):
        """(milliseconds, launches) of one pass kernel since timing was switched on."""
        ms, n = C.c_double(), C.c_longlong()
        self._check(lib().cge_timing_kernel(self._ctx, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def kernel_name(self):
        return lib().cge_kernel_name(self._ctx).decode()


def verify_state(params, precision, snapshot):
    """Integrity check of a snapshot held in host memory (bytes-like or a CPU uint8 tensor /
    numpy array): returns the status (OK or ECHECKPOINT)."""
    a = np.ascontiguousarray(np.frombuffer(bytes(snapshot), dtype=np.uint8)
                             if isinstance(snapshot, (bytes, bytearray)) else
                             np.asarray(snapshot, dtype=np.uint8))
    cp = make_params(params, precision)
    return lib().cge_verify_state(C.byref(cp), a.ctypes.data_as(C.c_void_p))


def copy_probe(dst, src, nbytes, stream):
    """Launch the library's streaming copy kernel (bandwidth reference)."""
    st = lib().cge_copy_probe(_ptr(dst), _ptr(src), int(nbytes), C.c_void_p(stream.cuda_stream))
    if st != OK:
        raise CgeError(st, "copy probe failed")


def observables_noalloc(params, precision, pop, carry, flags=None, stream=None, out=None):
    """cge_observables_noalloc on device buffers (torch tensors): the observables of the state
    in `pop` (encoded populations) and `carry`, with the library's static scratch.  Returns the
    device tensor of one cge_obs (`out` if given, else a new one) without synchronising; decode
    it with obs_from_device."""
    import torch
    if out is None:
        out = torch.empty(C.sizeof(CgeObs), dtype=torch.uint8, device=pop.device)
    cp = make_params(params, precision)
    st = lib().cge_observables_noalloc(C.byref(cp), _ptr(pop), _ptr(carry), _ptr(flags),
                                       C.c_void_p(stream.cuda_stream if stream is not None else 0),
                                       _ptr(out))
    if st != OK:
        raise CgeError(st, "cge_observables_noalloc failed")
    return out


def obs_from_device(t):
    """A cge_obs device tensor (bytes) as a dict."""
    raw = bytes(t.cpu().numpy().tobytes())
    return CgeObs.from_buffer_copy(raw).as_dict()


def _autograd_function():
    import torch

    class EvaporationRun(torch.autograd.Function):
        """rho^N after nsteps from a fixed start state, differentiable in the flux field phi(x)
        and the site threshold Gamma (hard sites held at the forward run's, or soft sites).
        The forward keeps a checkpoint every K steps; the backward recomputes each segment
        and runs the library's reverse steps.  The segments are recomputed under the flux
        field, Gamma and kappa of this forward, which the backward puts back into the
        simulation first: another run on the same simulation between forward and backward
        does not change the gradient."""

        @staticmethod
        def forward(ctx, phi_field, gamma, sim, start, nsteps, K):
            if sim.phi_field is None:
                raise ValueError("the simulation needs a flux field (phi_field=...)")
            sim.phi_field.copy_(phi_field.detach().reshape(sim.shape).to(sim.phi_field.dtype))
            sim.set_site_threshold(float(gamma))
            sim.load_state(start)
            sim.set_counters()
            ckpt = sim.forward_ckpt(nsteps, K)
            ctx.sim, ctx.ckpt, ctx.nsteps, ctx.K = sim, ckpt, nsteps, K
            ctx.phi_dtype, ctx.gamma_like = phi_field.dtype, gamma
            ctx.phi_used = sim.phi_field.clone()
            ctx.gamma_used = float(sim.params["gamma"])
            ctx.kappa_used = float(sim.params.get("kappa", 0.01))
            return sim.fields()["rhoN"]

        @staticmethod
        def backward(ctx, grad_rhoN):
            sim = ctx.sim
            sim.phi_field.copy_(ctx.phi_used)
            sim.set_site_threshold(ctx.gamma_used, ctx.kappa_used)
            r = sim.backward(ctx.ckpt, ctx.nsteps, ctx.K, grad_rhoN.contiguous())
            gphi = r["grad_phi"].to(ctx.phi_dtype)
            gg = torch.as_tensor(r["grad_gamma"], dtype=ctx.gamma_like.dtype,
                                 device=ctx.gamma_like.device)
            return gphi, gg, None, None, None, None

    return EvaporationRun


_EVAP_FN = None


def evaporate(sim, phi_field, gamma, nsteps, K, start):
    """Differentiable run: rho^N(x, nsteps) from the saved state `start` (Simulation.save_state)
    under the flux field phi_field and threshold gamma (tensors; gradients flow to both)."""
    global _EVAP_FN
    if _EVAP_FN is None:
        _EVAP_FN = _autograd_function()
    return _EVAP_FN.apply(phi_field, gamma, sim, start, int(nsteps), int(K))
