// Host-side context and the launchers shared by the translation units of libcgevap.so.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/cgevap.h"
#include "lattice.hpp"

// Number of FP64 observables reduced per block (see observe.hip).
#define CGE_NOBS 12

struct cge_ctx {
    cge_params p{};
    int Q = 0;
    cge::Geo g{};
    hipStream_t stream = nullptr;
    int device = 0;
    int cus = 0;  // compute units of the device (launch shapes that fill the chip)
    int kernel = CGE_KERNEL_TWOPASS;  // resolved step implementation
    int zchunk = 0;                   // planes per chunk of the z-marching pull (0: automatic)
    // caller-owned buffers
    void* pop[2] = {nullptr, nullptr};
    int cur = 0;  // pop[cur] holds the current state
    unsigned char* carry = nullptr;
    const unsigned char* flags = nullptr;
    const void* phi_field = nullptr;
    bool bound = false;
    // library scratch
    void* rhoN = nullptr;           // N elements of the arithmetic type: the step forms keep
                                    // their rho^N field here at storage precision, the step-0
                                    // site data computes from it in the arithmetic type
    unsigned char* carry2 = nullptr;  // second site-mask buffer of the fused step (N bytes)
    void* mom = nullptr;              // moment record of the split step ([4][N])
    void* rec = nullptr;              // post-collision records of the record step ([14][N])
    double* acc_sink = nullptr;     // per-block cumulative sink (FP64)
    long long* acc_sites = nullptr; // per-block cumulative site count
    long long acc_len = 0;
    double* obs_part = nullptr;     // [CGE_NOBS][obs_blocks], then the FP64 phase field (N)
    long long obs_blocks = 0;
    double* obs_res = nullptr;      // [CGE_NOBS + 2] final values (device)
    unsigned char* ck = nullptr;    // 32 bytes: the checksum of a state being loaded
    // z-plane kinds of the fused step's plane walls ([nz] bytes, D3Q19), the solid-node count
    // per plane they are classified from ([nz]), and whether the bound flags are plane walls
    unsigned char* pkind = nullptr;
    unsigned* pcount = nullptr;
    bool plane_walls = false;
    // blue pressure outlets on the end planes of the last axis
    int out_lo = 0, out_hi = 0;
    double out_rho = 1.0;
    // height-dependent flux (active when hf_every > 0)
    long long hf_every = 0;
    double hf_phi = 0.0, hf_K = 1.0, hf_hs = 1.0;
    void* hf_part = nullptr;  // per-chunk column sums of the refresh (in the scratch block)
    void* scratch = nullptr;  // the block the large scratch buffers are carved from
    bool scratch_owned = false;  // allocated by cge_create (else the caller's)
    // counters
    long long step = 0;
    long long sites_offset = 0;
    double sink_offset = 0.0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;     // event pool
    std::vector<const char*> ev_lab;  // per recorded event: nullptr = a step starts, else the
                                      // kernel (pass) that ran since the previous event
    size_t ev_used = 0;
    long long timed_steps = 0;
    double timed_ms = 0.0;
    std::vector<std::pair<std::string, std::pair<double, long long>>> ktime;  // per kernel
    std::string err;
};

namespace cge {

// bytes of the carried site data: the mask byte, or ||F|| in FP64 for the soft rule
inline size_t carry_bytes(const cge_params* p) {
    return (size_t)p->nx * p->ny * p->nz * (p->site_rule == CGE_SITE_SOFT ? sizeof(double) : 1);
}

cge_status fail(cge_ctx* c, cge_status s, const std::string& msg);
cge_status check(cge_ctx* c, hipError_t e, const char* what);

// step implementations: launch `nsteps` steps, swapping c->cur
cge_status twopass_steps(cge_ctx* c, long long nsteps);
cge_status fused_steps(cge_ctx* c, long long nsteps);
cge_status split_steps(cge_ctx* c, long long nsteps);
bool split_supported(const cge_ctx* c);
size_t split_scratch_bytes(const cge_params* p);
// record form of the split step: the state between the steps of one call is kept as
// per-node post-collision records
cge_status record_steps(cge_ctx* c, long long nsteps);
size_t record_bytes(const cge_params* p);
// one split step with explicit site-data, phase-field and moment buffers
cge_status split_step_into(cge_ctx* c, const void* carry_in, void* carry_out, void* rhoN,
                           void* mom);
bool fused_supported(const cge_ctx* c);
// classify the bound solid flags for the fused step (sets plane_walls and pkind; synchronises)
cge_status fused_classify(cge_ctx* c);
long long twopass_blocks(const cge_ctx* c);
long long fused_blocks(const cge_ctx* c);

// site mask from the current state's phase field (no sink)
cge_status reset_sites(cge_ctx* c);
template <typename R>
cge_status wet_field(cge_ctx* c, R* rhoN);

// saved states (state.hip): layout, copy with or without the integrity trailer, checks
size_t state_carry_offset(const cge_params* p);
size_t state_trailer_offset(const cge_params* p);
size_t state_bytes(const cge_params* p);
cge_status save_state(cge_ctx* c, void* dst, bool seal);
cge_status load_state(cge_ctx* c, const void* src, bool verify);
cge_status verify_state_host(const cge_params* p, const void* snapshot);

// state conversion
cge_status init_equilibrium(cge_ctx* c, const double* rr, const double* rb, const double* u);
cge_status set_populations(cge_ctx* c, const double* f);
cge_status get_populations(cge_ctx* c, double* f);
cge_status fields(cge_ctx* c, double* rr, double* rb, double* u, double* rhoN);

// flux field from the column heights of the current state (flux.hip)
cge_status height_flux(cge_ctx* c);
size_t height_partial_bytes(const Geo& g, int Q);
// outlet values in the current state (outlet.hip); no-op without outlets
cge_status apply_outlets(cge_ctx* c);

// adjoint workspace size
size_t adjoint_bytes(const cge_params* p);

// observables into c->obs_res (device), then copied to host by the caller
cge_status observables(cge_ctx* c);
// the same on explicit buffers, with the scratch in the library's static device array
cge_status observables_noalloc(const cge_params* p, const void* pop, const unsigned char* carry,
                               const unsigned char* flags, void* hip_stream, cge_obs* out);

cge_status copy_probe(void* dst, const void* src, size_t nbytes, hipStream_t s);

// timing helpers around the kernel launches of one step; they also open and close a roctx range
// named after the step form (rocprofv3 --marker-trace shows the steps and their kernels).
// timing_pass after each pass's launches attributes the time since the previous mark to the
// named kernel (its helper launches, e.g. the wetting pass, included).
void timing_begin(cge_ctx* c, const char* step_name);
void timing_pass(cge_ctx* c, const char* kernel);
void timing_end(cge_ctx* c);

// roctx range over a scope (an entry point, a segment of the adjoint)
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// launch shape of the one-thread-per-node kernels: (bx, 1, 1) blocks, bx a multiple of 64
inline dim3 node_block(const Geo& g) {
    const int bx = ((g.nx + 63) / 64) * 64;
    return dim3(bx < 256 ? bx : 256, 1, 1);
}
inline dim3 node_grid(const Geo& g) {
    const dim3 b = node_block(g);
    return dim3((g.nx + b.x - 1) / b.x, g.ny, g.nz);
}

// physical constants in arithmetic type M
template <typename M>
Phys<M> phys(const cge_ctx* c);

}  // namespace cge

// Dispatch a template FN<Q, S, M, WALLS>(args...) on lattice, precision and walls.
#define CGE_DISPATCH(c, FN, ...)                                                            \
    do {                                                                                    \
        const bool w_ = (c)->flags != nullptr;                                              \
        const int key_ = (c)->Q * 10 + (c)->p.precision;                                    \
        switch (key_) {                                                                     \
            case 90:                                                                        \
                return w_ ? FN<9, double, double, true>(__VA_ARGS__)                        \
                          : FN<9, double, double, false>(__VA_ARGS__);                      \
            case 91:                                                                        \
                return w_ ? FN<9, float, double, true>(__VA_ARGS__)                          \
                          : FN<9, float, double, false>(__VA_ARGS__);                        \
            case 92:                                                                        \
                if ((c)->p.fp16_arith64)                                                    \
                    return w_ ? FN<9, _Float16, double, true>(__VA_ARGS__)                   \
                              : FN<9, _Float16, double, false>(__VA_ARGS__);                 \
                return w_ ? FN<9, _Float16, float, true>(__VA_ARGS__)                        \
                          : FN<9, _Float16, float, false>(__VA_ARGS__);                      \
            case 190:                                                                       \
                return w_ ? FN<19, double, double, true>(__VA_ARGS__)                       \
                          : FN<19, double, double, false>(__VA_ARGS__);                     \
            case 191:                                                                       \
                return w_ ? FN<19, float, double, true>(__VA_ARGS__)                         \
                          : FN<19, float, double, false>(__VA_ARGS__);                       \
            case 192:                                                                       \
                if ((c)->p.fp16_arith64)                                                    \
                    return w_ ? FN<19, _Float16, double, true>(__VA_ARGS__)                  \
                              : FN<19, _Float16, double, false>(__VA_ARGS__);                \
                return w_ ? FN<19, _Float16, float, true>(__VA_ARGS__)                       \
                          : FN<19, _Float16, float, false>(__VA_ARGS__);                     \
            default:                                                                        \
                return cge::fail((c), CGE_EUNSUPPORTED, "unsupported lattice/precision");   \
        }                                                                                   \
    } while (0)
