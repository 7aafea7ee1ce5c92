// C-ABI entry points of libcgevap.so (declared in include/cgevap.h): parameter validation,
// scratch management, step sequencing, timing, and the copy bandwidth probe.
#include <cmath>
#include <cstring>
#include <new>

#include <algorithm>

#include "internal.hpp"
#include "node.hpp"

namespace cge {

cge_status fail(cge_ctx* c, cge_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

cge_status check(cge_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return CGE_OK;
    return fail(c, CGE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// alpha_k of the generalized colour-gradient model (Sec. II.A): the least dense component
// takes W_0, the others 1 - (1 - W_0)/gamma_k with gamma_k = rho_k / rho_min.
static void alphas(const cge_params& p, double w0, double a[2]) {
    const double rmin = p.rho_in[0] < p.rho_in[1] ? p.rho_in[0] : p.rho_in[1];
    for (int k = 0; k < 2; ++k)
        a[k] = p.rho_in[k] == rmin ? w0 : 1.0 - (1.0 - w0) / (p.rho_in[k] / rmin);
}

template <typename M>
Phys<M> phys(const cge_ctx* c) {
    const double w0 = c->Q == 9 ? Lat<9>::w0 : Lat<19>::w0;
    double a[2];
    alphas(c->p, w0, a);
    Phys<M> P;
    P.rho_ref = M(c->p.rho_in[1]);
    P.alpha_ref = M(a[1]);
    P.alpha_r = M(a[0]);
    P.alpha_b = M(a[1]);
    P.rho_in_r = M(c->p.rho_in[0]);
    P.rho_in_b = M(c->p.rho_in[1]);
    P.omega_r = M(1.0 / c->p.tau[0]);
    P.omega_b = M(1.0 / c->p.tau[1]);
    P.sigma = M(c->p.sigma);
    P.beta = M(c->p.beta);
    P.gamma = M(c->p.gamma);
    P.phi = M(c->p.phi);
    P.inv_sbar = M(1.0 / c->p.sbar);
    P.inv_kappa = M(c->p.site_rule == CGE_SITE_SOFT ? 1.0 / c->p.kappa : 0.0);
    P.inv_fade = M(c->p.recolor_fade > 0.0 ? 1.0 / c->p.recolor_fade : 0.0);
    P.site_rule = c->p.site_rule;
    return P;
}
template Phys<float> phys<float>(const cge_ctx*);
template Phys<double> phys<double>(const cge_ctx*);

// record the next event of the pool with a label (nullptr: a step starts)
static bool timing_record(cge_ctx* c, const char* label) {
    if (c->ev_used == c->ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        c->ev.push_back(e);
        c->ev_lab.push_back(nullptr);
    }
    if (hipEventRecord(c->ev[c->ev_used], c->stream) != hipSuccess) return false;
    c->ev_lab[c->ev_used++] = label;
    return true;
}

// sum the recorded intervals: each labelled event closes an interval of that kernel
static void timing_fold(cge_ctx* c) {
    if (c->ev_used == 0) return;
    (void)hipEventSynchronize(c->ev[c->ev_used - 1]);
    for (size_t k = 1; k < c->ev_used; ++k) {
        const char* lab = c->ev_lab[k];
        if (!lab) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev[k - 1], c->ev[k]) != hipSuccess) continue;
        c->timed_ms += ms;
        auto it = c->ktime.begin();
        while (it != c->ktime.end() && it->first != lab) ++it;
        if (it == c->ktime.end()) it = c->ktime.insert(it, {std::string(lab), {0.0, 0}});
        it->second.first += ms;
        it->second.second += 1;
    }
    c->ev_used = 0;
}

void timing_begin(cge_ctx* c, const char* step_name) {
    roctxRangePushA(step_name);
    if (!c->timing) return;
    if (c->ev_used + 8 > 4096) timing_fold(c);  // a step records at most 3 events
    if (timing_record(c, nullptr)) c->timed_steps += 1;
}

void timing_pass(cge_ctx* c, const char* kernel) {
    if (c->timing && c->ev_used > 0) (void)timing_record(c, kernel);
}

void timing_end(cge_ctx* c) { roctxRangePop(); }

__global__ __launch_bounds__(256) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                              long long n16) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_zero(unsigned long long* __restrict__ p, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// zero n 8-byte words with a kernel (no memset node, so the call is safe under capture)
static hipError_t zero_words(void* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       static_cast<unsigned long long*>(p), n);
    return hipGetLastError();
}

cge_status copy_probe(void* dst, const void* src, size_t nbytes, hipStream_t s) {
    const long long n16 = (long long)(nbytes / 16);
    // four 16-byte elements per thread: the fastest of the grid sizes measured for 1 GiB
    const long long blocks = (n16 + 1023) / 1024;
    if (n16 > 0)
        hipLaunchKernelGGL(k_copy, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256),
                           0, s, static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    return hipGetLastError() == hipSuccess ? CGE_OK : CGE_EDEVICE;
}

}  // namespace cge

using namespace cge;

static bool is_fin(double v) { return std::isfinite(v); }

static const char* validate(const cge_params* p) {
    if (!p) return "params is NULL";
    if (p->lattice != CGE_D2Q9 && p->lattice != CGE_D3Q19) return "lattice must be 9 or 19";
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "nx, ny, nz must be >= 1";
    if (p->ny > 65535 || p->nz > 65535) return "ny and nz must be <= 65535";
    if (p->lattice == CGE_D2Q9 && p->nz != 1) return "D2Q9 needs nz == 1";
    if (p->precision < CGE_FP64 || p->precision > CGE_FP16S) return "unknown precision";
    for (int k = 0; k < 2; ++k) {
        if (!(is_fin(p->rho_in[k]) && p->rho_in[k] > 0.0)) return "rho_in must be > 0";
        if (!(is_fin(p->tau[k]) && p->tau[k] > 0.5)) return "tau must be > 1/2";
    }
    if (!(is_fin(p->sigma) && p->sigma >= 0.0)) return "sigma must be >= 0";
    if (!(is_fin(p->beta) && p->beta >= 0.0 && p->beta <= 1.0)) return "beta must be in [0, 1]";
    if (!is_fin(p->phi)) return "phi must be finite";
    if (!(is_fin(p->sbar) && p->sbar >= 1.0)) return "sbar must be >= 1";
    if (!is_fin(p->gamma)) return "gamma must be finite";
    if (p->site_rule != CGE_SITE_GRAD_GT && p->site_rule != CGE_SITE_PHASE_LT &&
        p->site_rule != CGE_SITE_SOFT)
        return "unknown site rule";
    if (p->site_rule == CGE_SITE_SOFT && !(is_fin(p->kappa) && p->kappa > 0.0))
        return "kappa must be > 0 for the soft site rule";
    if (p->kernel < CGE_KERNEL_AUTO || p->kernel > CGE_KERNEL_RECORD) return "unknown kernel";
    if (!(is_fin(p->recolor_fade) && p->recolor_fade >= 0.0))
        return "recolor_fade must be finite and >= 0";
    if (p->fp16_arith64 != 0 && !(p->fp16_arith64 == 1 && p->precision == CGE_FP16S))
        return "fp16_arith64 must be 0, or 1 with CGE_FP16S";
    return nullptr;
}

static size_t elem_bytes(int precision) {
    return precision == CGE_FP64 ? 8 : (precision == CGE_FP32S ? 4 : 2);
}

extern "C" {

size_t cge_population_bytes(const cge_params* p) {
    if (validate(p)) return 0;
    return 2ull * p->lattice * (size_t)p->nx * p->ny * p->nz * elem_bytes(p->precision);
}

// Large scratch of a context, carved from one block in this order (each part 256-aligned):
// the phase field (N values of the arithmetic type), the fused step's second mask (N bytes,
// D3Q19), the split step's moment record (unit tau), the record form's post-collision records
// (where the record form may run), the observables' partials and FP64 phase field, and the
// height flux's column sums.
struct ScratchPlan {
    size_t rhoN = 0, carry2 = 0, mom = 0, rec = 0, obs = 0, hf = 0, total = 0;
    bool has_rec = false;
};

static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

static ScratchPlan scratch_plan(const cge_params* p) {
    ScratchPlan s;
    const int Q = p->lattice;
    const Geo g{p->nx, p->ny, p->nz, 0, (long long)p->nx * p->ny * p->nz};
    const bool unit = p->tau[0] == 1.0 && p->tau[1] == 1.0;
    // records where the record form may run: selected, or chosen by AUTO (unit tau, D3Q19)
    const bool rec = unit && (p->kernel == CGE_KERNEL_RECORD ||
                              (p->kernel == CGE_KERNEL_AUTO && Q == 19));
    // the widest use of the field: the arithmetic type
    const size_t mbytes = (p->precision == CGE_FP16S && !p->fp16_arith64) ? 4 : 8;
    const dim3 gr = node_grid(g);
    const size_t nblk = (size_t)gr.x * gr.y * gr.z;
    size_t off = 0;
    auto take = [&](size_t& at, size_t bytes) {
        at = off;
        off += up256(bytes);
    };
    take(s.rhoN, g.N * mbytes);
    take(s.carry2, Q == 19 ? (size_t)g.N : 0);
    take(s.mom, unit ? split_scratch_bytes(p) : 0);
    take(s.rec, rec ? record_bytes(p) : 0);
    s.has_rec = rec;
    take(s.obs, (CGE_NOBS * nblk + (size_t)g.N) * sizeof(double));
    take(s.hf, height_partial_bytes(g, Q));
    s.total = off;
    return s;
}

static cge_status create_ctx(const cge_params* params, void* hip_stream, void* scratch,
                             size_t scratch_bytes, cge_ctx** out) {
    if (!out) return CGE_EINVAL;
    if (validate(params)) return CGE_EINVAL;
    const ScratchPlan plan = scratch_plan(params);
    if (scratch && scratch_bytes < plan.total) return CGE_EINVAL;
    if (scratch && ((uintptr_t)scratch & 255)) return CGE_EINVAL;
    cge_ctx* c = new (std::nothrow) cge_ctx();
    if (!c) return CGE_ENOMEM;
    c->p = *params;
    c->Q = params->lattice;
    c->g = Geo{params->nx, params->ny, params->nz, 0,
               (long long)params->nx * params->ny * params->nz};
    // non-temporal stores for each class of array a step writes that is too large to stay in
    // the 256 MB last-level cache until the next pass reads it back: populations above half
    // of it, the moment record and the post-collision records above a quarter (the pass that
    // reads them back streams the populations past them).  Measured on the D2Q9 split step:
    // a cached moment record of 21-42 MB saves 17 %, one of 84 MB costs 6 % of the finish.
    const size_t pop_bound = 128ull << 20, rec_bound = 64ull << 20;
    const size_t me = params->precision == CGE_FP64 ? 8 : 4;
    if (2ull * c->Q * (size_t)c->g.N * elem_bytes(params->precision) > pop_bound) c->g.nt |= kNtPop;
    if (5ull * (size_t)c->g.N * me > rec_bound) c->g.nt |= kNtMom;
    if (record_bytes(params) > rec_bound) c->g.nt |= kNtRec;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
            hipSuccess) {
        delete c;
        return CGE_EDEVICE;
    }
    // the fused step needs D3Q19 and no solid nodes other than plane walls (the latter is known
    // at cge_bind); the split step and the record form need unit relaxation times
    const bool unit = split_supported(c);
    const bool soft = params->site_rule == CGE_SITE_SOFT;
    if ((params->kernel == CGE_KERNEL_FUSED && (c->Q != 19 || soft)) ||
        ((params->kernel == CGE_KERNEL_SPLIT || params->kernel == CGE_KERNEL_RECORD) && !unit)) {
        delete c;
        return CGE_EUNSUPPORTED;
    }
    c->kernel = CGE_KERNEL_TWOPASS;  // resolved at cge_bind
    if (scratch) {
        c->scratch = scratch;
    } else {
        if (hipMalloc(&c->scratch, plan.total) != hipSuccess) {
            c->scratch = nullptr;
            delete c;
            return CGE_ENOMEM;
        }
        c->scratch_owned = true;
    }
    char* base = static_cast<char*>(c->scratch);
    c->rhoN = base + plan.rhoN;
    c->carry2 = c->Q == 19 ? reinterpret_cast<unsigned char*>(base + plan.carry2) : nullptr;
    // the moment record also serves the checkpointed forward run of the adjoint at unit tau
    c->mom = unit ? base + plan.mom : nullptr;
    c->rec = plan.has_rec ? base + plan.rec : nullptr;
    c->obs_part = reinterpret_cast<double*>(base + plan.obs);
    c->hf_part = base + plan.hf;
    c->acc_len = twopass_blocks(c);
    if (c->Q == 19 && fused_blocks(c) > c->acc_len) c->acc_len = fused_blocks(c);
    c->obs_blocks = twopass_blocks(c);
    // small library-owned buffers: per-block sink partials, reduction results
    bool ok = hipMalloc(&c->acc_sink, c->acc_len * sizeof(double)) == hipSuccess &&
              hipMalloc(&c->acc_sites, c->acc_len * sizeof(long long)) == hipSuccess &&
              hipMalloc(&c->obs_res, (CGE_NOBS + 2) * sizeof(double)) == hipSuccess &&
              hipMalloc(&c->ck, 32) == hipSuccess;
    if (ok && c->Q == 19)  // the fused step's z-plane table (a few bytes per plane)
        ok = hipMalloc(&c->pkind, (size_t)c->g.nz) == hipSuccess &&
             hipMalloc(&c->pcount, (size_t)c->g.nz * sizeof(unsigned)) == hipSuccess;
    if (!ok) {
        cge_destroy(c);
        return CGE_ENOMEM;
    }
    ok = zero_words(c->acc_sink, c->acc_len, c->stream) == hipSuccess &&
         zero_words(c->acc_sites, c->acc_len, c->stream) == hipSuccess;
    if (!ok) {
        cge_destroy(c);
        return CGE_EDEVICE;
    }
    *out = c;
    return CGE_OK;
}

size_t cge_scratch_bytes(const cge_params* p) { return validate(p) ? 0 : scratch_plan(p).total; }

cge_status cge_create(const cge_params* params, void* hip_stream, cge_ctx** out) {
    return create_ctx(params, hip_stream, nullptr, 0, out);
}

cge_status cge_create_with_scratch(const cge_params* params, void* hip_stream, void* scratch,
                                   size_t scratch_bytes, cge_ctx** out) {
    if (!scratch) return CGE_EINVAL;
    return create_ctx(params, hip_stream, scratch, scratch_bytes, out);
}

cge_status cge_bind(cge_ctx* c, void* pop_a, void* pop_b, unsigned char* carry,
                    const unsigned char* flags, const void* phi_field) {
    if (!c) return CGE_EINVAL;
    if (!pop_a || !pop_b || !carry) return fail(c, CGE_EINVAL, "pop_a, pop_b, carry required");
    if (pop_a == pop_b) return fail(c, CGE_EINVAL, "pop_a and pop_b must differ");
    c->pop[0] = pop_a;
    c->pop[1] = pop_b;
    c->cur = 0;
    c->carry = carry;
    c->flags = flags;
    c->phi_field = phi_field;
    c->plane_walls = false;
    if (flags && c->Q == 19 && c->p.site_rule != CGE_SITE_SOFT)
        if (cge_status s = fused_classify(c)) return s;
    if (flags && c->p.kernel == CGE_KERNEL_FUSED && !c->plane_walls)
        return fail(c, CGE_EUNSUPPORTED,
                    "the fused step supports solid nodes only as whole z-planes, none with "
                    "fluid on both sides");
    switch (c->p.kernel) {
        case CGE_KERNEL_TWOPASS: c->kernel = CGE_KERNEL_TWOPASS; break;
        case CGE_KERNEL_FUSED:
            c->kernel = fused_supported(c) ? CGE_KERNEL_FUSED : CGE_KERNEL_TWOPASS;
            break;
        case CGE_KERNEL_SPLIT: c->kernel = CGE_KERNEL_SPLIT; break;
        case CGE_KERNEL_RECORD: c->kernel = CGE_KERNEL_RECORD; break;
        default:
            // the fused step only below FP64: at FP64 its per-thread population stash takes
            // most of a CU's LDS, and it ran about three times slower than the two-pass step
            // (256 x 256 x 128 sessile drop: 4.22 against 1.47 ms per step)
            c->kernel = split_supported(c) ? (c->rec ? CGE_KERNEL_RECORD : CGE_KERNEL_SPLIT)
                        : (fused_supported(c) && c->p.precision != CGE_FP64 ? CGE_KERNEL_FUSED
                                                                             : CGE_KERNEL_TWOPASS);
    }
    c->bound = true;
    return CGE_OK;
}

static cge_status zero_counters(cge_ctx* c) {
    c->step = 0;
    c->sites_offset = 0;
    c->sink_offset = 0.0;
    if (zero_words(c->acc_sink, c->acc_len, c->stream) != hipSuccess ||
        zero_words(c->acc_sites, c->acc_len, c->stream) != hipSuccess)
        return fail(c, CGE_EDEVICE, "clearing the sink accumulators failed");
    return CGE_OK;
}

cge_status cge_init_equilibrium(cge_ctx* c, const double* rho_r, const double* rho_b,
                                const double* u) {
    TraceRange trace_("cge_init_equilibrium");
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (!rho_r || !rho_b) return fail(c, CGE_EINVAL, "rho_r and rho_b required");
    if (cge_status s = init_equilibrium(c, rho_r, rho_b, u)) return s;
    if (cge_status s = reset_sites(c)) return s;
    if (cge_status s = zero_counters(c)) return s;
    return apply_outlets(c);
}

cge_status cge_set_populations(cge_ctx* c, const double* f) {
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (!f) return fail(c, CGE_EINVAL, "f is NULL");
    if (cge_status s = set_populations(c, f)) return s;
    return apply_outlets(c);
}

cge_status cge_get_populations(cge_ctx* c, double* f) {
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (!f) return fail(c, CGE_EINVAL, "f is NULL");
    return get_populations(c, f);
}

size_t cge_state_bytes(const cge_params* p) { return validate(p) ? 0 : state_bytes(p); }

cge_status cge_save_state(cge_ctx* c, void* dst) {
    TraceRange trace_("cge_save_state");
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (!dst) return fail(c, CGE_EINVAL, "dst is NULL");
    return save_state(c, dst, true);
}

cge_status cge_load_state(cge_ctx* c, const void* src) {
    TraceRange trace_("cge_load_state");
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (!src) return fail(c, CGE_EINVAL, "src is NULL");
    return load_state(c, src, true);
}

cge_status cge_verify_state(const cge_params* p, const void* snapshot) {
    if (validate(p) || !snapshot) return CGE_EINVAL;
    return verify_state_host(p, snapshot);
}

cge_status cge_reset_sites(cge_ctx* c) {
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    return reset_sites(c);
}

cge_status cge_set_outlet(cge_ctx* c, int lo, int hi, double rho_out) {
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (lo || hi) {
        if (!is_fin(rho_out) || !(rho_out > 0.0))
            return fail(c, CGE_EINVAL, "outlet density must be finite and positive");
        if ((c->Q == 19 ? c->g.nz : c->g.ny) < 3)
            return fail(c, CGE_EINVAL, "outlets need at least 3 planes along the last axis");
    }
    c->out_lo = lo ? 1 : 0;
    c->out_hi = hi ? 1 : 0;
    c->out_rho = rho_out;
    return apply_outlets(c);
}

cge_status cge_set_height_flux(cge_ctx* c, double phi_s, double K, double h_scale,
                               long long every) {
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (every > 0) {
        if (!c->phi_field) return fail(c, CGE_ESTATE, "the height flux needs a bound flux field");
        if (!is_fin(phi_s) || !is_fin(K) || !(K > 0.0) || !is_fin(h_scale) || !(h_scale > 0.0))
            return fail(c, CGE_EINVAL, "height flux needs finite phi_s, K > 0, h_scale > 0");
        c->hf_phi = phi_s;
        c->hf_K = K;
        c->hf_hs = h_scale;
    }
    c->hf_every = every > 0 ? every : 0;
    return CGE_OK;
}

cge_status cge_set_site_threshold(cge_ctx* c, double gamma, double kappa) {
    if (!c) return CGE_EINVAL;
    if (!is_fin(gamma) || !is_fin(kappa))
        return fail(c, CGE_EINVAL, "site threshold must be finite");
    c->p.gamma = gamma;
    if (kappa > 0.0) c->p.kappa = kappa;
    return CGE_OK;
}

cge_status cge_set_zchunk(cge_ctx* c, int planes) {
    if (!c) return CGE_EINVAL;
    if (planes < 0) return fail(c, CGE_EINVAL, "planes must be >= 0");
    c->zchunk = planes;
    return CGE_OK;
}

cge_status cge_set_counters(cge_ctx* c, long long step, long long site_steps, double sink_total) {
    if (!c) return CGE_EINVAL;
    if (step < 0 || site_steps < 0 || !is_fin(sink_total))
        return fail(c, CGE_EINVAL, "counters must be non-negative and finite");
    if (cge_status s = zero_counters(c)) return s;
    c->step = step;
    c->sites_offset = site_steps;
    c->sink_offset = sink_total;
    return CGE_OK;
}

static cge_status run_steps(cge_ctx* c, long long nsteps) {
    switch (c->kernel) {
        case CGE_KERNEL_FUSED: return fused_steps(c, nsteps);
        case CGE_KERNEL_SPLIT: return split_steps(c, nsteps);
        case CGE_KERNEL_RECORD: return record_steps(c, nsteps);
        default: return twopass_steps(c, nsteps);
    }
}

cge_status cge_step(cge_ctx* c, long long nsteps) {
    TraceRange trace_("cge_step");
    if (!c) return CGE_EINVAL;
    if (nsteps < 0) return fail(c, CGE_EINVAL, "nsteps must be >= 0");
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (nsteps == 0) return CGE_OK;
    const bool outlets = c->out_lo || c->out_hi;
    if (c->hf_every <= 0 && !outlets) return run_steps(c, nsteps);
    // height flux: refresh the field before every step whose counter is a multiple of every;
    // outlets: take the outlet values after every step
    for (long long done = 0; done < nsteps;) {
        long long n = nsteps - done;
        if (c->hf_every > 0) {
            const long long phase = c->step % c->hf_every;
            if (phase == 0)
                if (cge_status s = height_flux(c)) return s;
            n = std::min(c->hf_every - phase, n);
        }
        if (outlets) n = 1;
        if (cge_status s = run_steps(c, n)) return s;
        if (outlets)
            if (cge_status s = apply_outlets(c)) return s;
        done += n;
    }
    return CGE_OK;
}

cge_status cge_observables(cge_ctx* c, cge_obs* out) {
    TraceRange trace_("cge_observables");
    if (!c) return CGE_EINVAL;
    if (!out) return fail(c, CGE_EINVAL, "out is NULL");
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (cge_status s = observables(c)) return s;
    double r[CGE_NOBS + 2];
    if (cge_status s = check(c, hipMemcpyAsync(r, c->obs_res, sizeof(r), hipMemcpyDeviceToHost,
                                               c->stream), "observable copy"))
        return s;
    if (cge_status s = check(c, hipStreamSynchronize(c->stream), "stream sync")) return s;
    // indices follow the partial layout of the observable kernels
    out->step = c->step;
    out->mass_r = r[0];
    out->mass_b = r[1];
    out->n_negative = (long long)r[2];
    out->p_in = r[4] > 0 ? r[3] / r[4] : 0.0;
    out->p_out = r[6] > 0 ? r[5] / r[6] : 0.0;
    out->n_sites = (long long)r[7];
    out->max_u = r[8];
    out->max_rho_r = r[9];
    out->perim_grad = r[10];
    out->v_half = (long long)r[11];
    out->sink_total = c->sink_offset + r[CGE_NOBS];
    out->site_steps = c->sites_offset + (long long)r[CGE_NOBS + 1];
    out->v_mass = out->mass_r / c->p.rho_in[0];
    out->perim_sites = (double)out->n_sites / c->p.sbar;
    if (!is_fin(out->mass_r) || !is_fin(out->mass_b) || !is_fin(out->max_u))
        return fail(c, CGE_ENUMERIC, "non-finite values in the state");
    return CGE_OK;
}

cge_status cge_observables_noalloc(const cge_params* p, const void* pop, const unsigned char* carry,
                                   const unsigned char* flags, void* hip_stream, cge_obs* out) {
    TraceRange trace_("cge_observables_noalloc");
    if (validate(p) || !pop || !carry || !out) return CGE_EINVAL;
    return observables_noalloc(p, pop, carry, flags, hip_stream, out);
}

cge_status cge_fields(cge_ctx* c, double* rho_r, double* rho_b, double* u, double* rhoN) {
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    return fields(c, rho_r, rho_b, u, rhoN);
}

cge_status cge_set_timing(cge_ctx* c, int on) {
    if (!c) return CGE_EINVAL;
    if (on && !c->timing) {
        c->timed_ms = 0.0;
        c->timed_steps = 0;
        c->ev_used = 0;
        c->ktime.clear();
    }
    if (!on) timing_fold(c);
    c->timing = on != 0;
    return CGE_OK;
}

cge_status cge_timing(cge_ctx* c, double* total_ms, long long* steps) {
    if (!c || !total_ms || !steps) return fail(c, CGE_EINVAL, "NULL argument");
    timing_fold(c);
    *total_ms = c->timed_ms;
    *steps = c->timed_steps;
    return CGE_OK;
}

cge_status cge_timing_kernel(cge_ctx* c, const char* kernel, double* total_ms,
                             long long* launches) {
    if (!c || !kernel || !total_ms || !launches) return fail(c, CGE_EINVAL, "NULL argument");
    timing_fold(c);
    *total_ms = 0.0;
    *launches = 0;
    for (const auto& kv : c->ktime)
        if (kv.first == kernel) {
            *total_ms = kv.second.first;
            *launches = kv.second.second;
        }
    return CGE_OK;
}

const char* cge_kernel_name(const cge_ctx* c) {
    if (!c) return "";
    switch (c->kernel) {
        case CGE_KERNEL_FUSED: return "k_fused";
        case CGE_KERNEL_SPLIT: return "k_finish";
        case CGE_KERNEL_RECORD: return "k_pull_record";
        default: return "k_collide";
    }
}

cge_status cge_lattice_tables(int lattice, double* W, double* A, double* B, double* C, int* cv,
                              int* opp, double* zeta) {
    if (lattice != 9 && lattice != 19) return CGE_EINVAL;
    for (int i = 0; i < lattice; ++i) {
        if (lattice == 9) {
            if (W) W[i] = weight<9>(i);
            if (A) A[i] = restA<9>(i);
            if (B) B[i] = restB<9>(i);
            if (C) C[i] = pertC<9>(i);
            if (cv) { cv[3 * i] = Lat<9>::cx[i]; cv[3 * i + 1] = Lat<9>::cy[i]; cv[3 * i + 2] = Lat<9>::cz[i]; }
            if (opp) opp[i] = Lat<9>::opp[i];
        } else {
            if (W) W[i] = weight<19>(i);
            if (A) A[i] = restA<19>(i);
            if (B) B[i] = restB<19>(i);
            if (C) C[i] = pertC<19>(i);
            if (cv) { cv[3 * i] = Lat<19>::cx[i]; cv[3 * i + 1] = Lat<19>::cy[i]; cv[3 * i + 2] = Lat<19>::cz[i]; }
            if (opp) opp[i] = Lat<19>::opp[i];
        }
    }
    if (zeta) *zeta = lattice == 9 ? Lat<9>::zeta : Lat<19>::zeta;
    return CGE_OK;
}

cge_status cge_copy_probe(void* dst, const void* src, size_t nbytes, void* hip_stream) {
    if (!dst || !src) return CGE_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src) & 15) return CGE_EINVAL;
    return copy_probe(dst, src, nbytes, static_cast<hipStream_t>(hip_stream));
}

const char* cge_last_error(const cge_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

void cge_destroy(cge_ctx* c) {
    if (!c) return;
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->scratch_owned) (void)hipFree(c->scratch);
    (void)hipFree(c->acc_sink);
    (void)hipFree(c->acc_sites);
    (void)hipFree(c->obs_res);
    (void)hipFree(c->ck);
    (void)hipFree(c->pkind);
    (void)hipFree(c->pcount);
    delete c;
}

}  // extern "C"
