// Observables of the current state, reduced in FP64 in a fixed order:
//   pass A (per node): masses, negative-population count, max |u|, EOS pressure sums over
//          the two bulk phases (Eq. EOS), max rho_r, site count; rho^N into scratch
//   wetting of solid nodes
//   pass B (per node): (1/2)||grad rho^N|| (interface measure), after max rho_r is known:
//          count of rho_r > max/2 (interface position rule of Sec. III)
//   final: one block sums the per-block partials and the per-block sink accumulators.
#include <mutex>

#include "internal.hpp"
#include "node.hpp"

namespace cge {

enum {
    O_MASS_R = 0,
    O_MASS_B,
    O_NNEG,
    O_PIN,
    O_NIN,
    O_POUT,
    O_NOUT,
    O_NSITES,
    O_MAXU,
    O_MAXRR,
    O_PERIM,
    O_VHALF
};
static_assert(O_VHALF + 1 == CGE_NOBS, "observable count");

template <int Q, typename S, bool WALLS>
__device__ __forceinline__ void decode_node(const S* __restrict__ src, const uint8_t* __restrict__ flags,
                                            const Geo& g, int x, int y, int z, long long n,
                                            const Phys<double>& P, double& rr, double& rb,
                                            double (&j)[3], int& nneg) {
    const Nb b = wrap(g, x, y, z);
    double ft[Q], dd[Q];
    pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
    rr = rb = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    nneg = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double full = ft[i] + P.rho_ref * (restA<Q>(i) + restB<Q>(i) * P.alpha_ref);
        const double a = 0.5 * (full + dd[i]), c = 0.5 * (full - dd[i]);
        rr += a;
        rb += c;
        // negative beyond rounding noise: below -1e-6 of the bulk equilibrium value
        nneg += (a < -1e-6 * P.rho_in_r * (restA<Q>(i) + restB<Q>(i) * P.alpha_r)) +
                (c < -1e-6 * P.rho_in_b * (restA<Q>(i) + restB<Q>(i) * P.alpha_b));
        j[0] += Lat<Q>::cx[i] * (a + c);
        j[1] += Lat<Q>::cy[i] * (a + c);
        j[2] += Lat<Q>::cz[i] * (a + c);
    }
}

__device__ __forceinline__ long long block_id() {
    return blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
}

template <int Q, typename S, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_obs_a(const S* __restrict__ src,
                                                 const uint8_t* __restrict__ flags,
                                                 const void* __restrict__ carry,
                                                 double* __restrict__ rhoN,
                                                 double* __restrict__ part, long long nblk, Geo g,
                                                 Phys<double> P, double zeta) {
    int x, y, z;
    long long n;
    const bool valid = node_xyz(g, x, y, z, n);
    double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (valid && !(WALLS && flags[n])) {
        double rr, rb, j[3];
        int nneg;
        decode_node<Q, S, WALLS>(src, flags, g, x, y, z, n, P, rr, rb, j, nneg);
        const double rho = rr + rb;
        const double rN = (rr - rb) / rho;
        rhoN[n] = rN;
        const double p = rr * zeta * (1.0 - P.alpha_r) + rb * zeta * (1.0 - P.alpha_b);
        v[O_MASS_R] = rr;
        v[O_MASS_B] = rb;
        v[O_NNEG] = nneg;
        if (rN > 0.9) { v[O_PIN] = p; v[O_NIN] = 1.0; }
        if (rN < -0.9) { v[O_POUT] = p; v[O_NOUT] = 1.0; }
        const bool site = is_site(site_weight<double>(P, carry, n, rho, rr - rb));
        v[O_NSITES] = site ? 1.0 : 0.0;
        v[O_MAXU] = sqrt(j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / rho;
        v[O_MAXRR] = rr;
    }
    const bool is_max[10] = {false, false, false, false, false, false, false, false, true, true};
    double out[10];
    block_reduce<10>(v, is_max, threadIdx.x, blockDim.x, out);
    if (threadIdx.x == 0) {
        const long long bid = block_id();
        for (int k = 0; k < 10; ++k) part[k * nblk + bid] = out[k];
    }
}

template <int Q, typename S, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_obs_b(const S* __restrict__ src,
                                                 const uint8_t* __restrict__ flags,
                                                 const double* __restrict__ rhoN,
                                                 const double* __restrict__ res,
                                                 double* __restrict__ part, long long nblk, Geo g,
                                                 Phys<double> P) {
    int x, y, z;
    long long n;
    const bool valid = node_xyz(g, x, y, z, n);
    double v[2] = {0.0, 0.0};
    if (valid && !(WALLS && flags[n])) {
        const Nb b = wrap(g, x, y, z);
        double F[3];
        gradient<Q>(rhoN, g, b, x, y, z, F);
        v[0] = 0.5 * sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
        double rr, rb, j[3];
        int nneg;
        decode_node<Q, S, WALLS>(src, flags, g, x, y, z, n, P, rr, rb, j, nneg);
        v[1] = rr > 0.5 * res[O_MAXRR] ? 1.0 : 0.0;
    }
    const bool is_max[2] = {false, false};
    double out[2];
    block_reduce<2>(v, is_max, threadIdx.x, blockDim.x, out);
    if (threadIdx.x == 0) {
        const long long bid = block_id();
        part[O_PERIM * nblk + bid] = out[0];
        part[O_VHALF * nblk + bid] = out[1];
    }
}

// Sum (max) of the per-block partials k0..k1-1 in block order; one block of 256 threads.
// res[CGE_NOBS] and res[CGE_NOBS+1] receive the sink and site accumulators.
__global__ __launch_bounds__(256) void k_obs_final(const double* __restrict__ part, long long nblk,
                                                   int k0, int k1, const double* __restrict__ acc_sink,
                                                   const long long* __restrict__ acc_sites,
                                                   long long nacc, double* __restrict__ res) {
    __shared__ double sh[256];
    for (int k = k0; k < k1; ++k) {
        const bool is_max = (k == O_MAXU || k == O_MAXRR);
        double s = is_max ? 0.0 : 0.0;
        for (long long b = threadIdx.x; b < nblk; b += blockDim.x) {
            const double v = part[k * nblk + b];
            s = is_max ? fmax(s, v) : s + v;
        }
        sh[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = sh[0];
            for (int i = 1; i < (int)blockDim.x; ++i) t = is_max ? fmax(t, sh[i]) : t + sh[i];
            res[k] = t;
        }
        __syncthreads();
    }
    if (acc_sink) {
        double s = 0.0, c = 0.0;
        for (long long b = threadIdx.x; b < nacc; b += blockDim.x) {
            s += acc_sink[b];
            c += static_cast<double>(acc_sites[b]);
        }
        sh[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < (int)blockDim.x; ++i) t += sh[i];
            res[CGE_NOBS] = t;
        }
        __syncthreads();
        sh[threadIdx.x] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < (int)blockDim.x; ++i) t += sh[i];
            res[CGE_NOBS + 1] = t;
        }
    }
}

// Scratch of one reduction: CGE_NOBS per-block partials, then the FP64 phase field (N values).
static long long obs_blocks_of(const Geo& g) {
    const dim3 gr = node_grid(g);
    return (long long)gr.x * gr.y * gr.z;
}
static size_t obs_scratch_bytes(const Geo& g) {
    return ((size_t)CGE_NOBS * obs_blocks_of(g) + (size_t)g.N) * sizeof(double);
}

// The reduction's launches on explicit buffers: part (obs_scratch_bytes), res (CGE_NOBS + 2
// doubles; the last two take the sink accumulators when acc_sink is given).
template <int Q, typename S, bool WALLS>
static hipError_t obs_launch(const S* pop, const uint8_t* flags, const void* carry, double* part,
                             double* res, const double* acc_sink, const long long* acc_sites,
                             long long nacc, const Geo& g, const Phys<double>& P,
                             hipStream_t stream) {
    const dim3 gr = node_grid(g), bl = node_block(g);
    const long long nblk = obs_blocks_of(g);
    double* rhoN = part + (long long)CGE_NOBS * nblk;  // N doubles after the partials
    hipLaunchKernelGGL((k_obs_a<Q, S, WALLS>), gr, bl, 0, stream, pop, flags, carry, rhoN, part,
                       nblk, g, P, Lat<Q>::zeta);
    if (WALLS)  // neutral wetting of the solid nodes, for the gradient of pass B
        hipLaunchKernelGGL((k_wet<Q, double>), gr, bl, 0, stream, flags, rhoN, g);
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, stream, part, nblk, 0, 10,
                       (const double*)nullptr, (const long long*)nullptr, 0LL, res);
    hipLaunchKernelGGL((k_obs_b<Q, S, WALLS>), gr, bl, 0, stream, pop, flags, rhoN, res, part,
                       nblk, g, P);
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(256), 0, stream, part, nblk, O_PERIM, CGE_NOBS,
                       acc_sink, acc_sites, nacc, res);
    return hipGetLastError();
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status obs_impl(cge_ctx* c) {
    return check(c,
                 obs_launch<Q, S, WALLS>(static_cast<const S*>(c->pop[c->cur]), c->flags,
                                         c->carry, c->obs_part, c->obs_res, c->acc_sink,
                                         c->acc_sites, c->acc_len, c->g, phys<double>(c),
                                         c->stream),
                 "observable kernels");
}

cge_status observables(cge_ctx* c) { CGE_DISPATCH(c, obs_impl, c); }

// ------------------------------------------------------------ allocation-free observables
//
// cge_observables_noalloc keeps the reduction's scratch in this file-scope array instead of a
// context's.  Each device holds its own copy from the moment the library's code is loaded on
// it until the process ends.  Host code never passes the array's name to a kernel (that is a
// host-side stand-in): the device address is looked up once per device and kept below.
constexpr size_t kNoallocScratch = 64ull << 20;  // bytes
constexpr size_t kNoallocRes = 256;             // bytes reserved for res and the result
static __device__ __align__(256) unsigned char scratch[kNoallocScratch];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first call there)
static hipError_t scratch_on_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// res (sums and counts of the reduction) -> the cge_obs fields a state determines
__global__ void k_obs_noalloc_out(const double* __restrict__ r, double rho_in_r, double sbar,
                                  cge_obs* __restrict__ out) {
    if (threadIdx.x != 0) return;
    cge_obs o;
    o.step = 0;
    o.site_steps = 0;
    o.sink_total = 0.0;
    o.mass_r = r[O_MASS_R];
    o.mass_b = r[O_MASS_B];
    o.n_negative = (long long)r[O_NNEG];
    o.p_in = r[O_NIN] > 0 ? r[O_PIN] / r[O_NIN] : 0.0;
    o.p_out = r[O_NOUT] > 0 ? r[O_POUT] / r[O_NOUT] : 0.0;
    o.n_sites = (long long)r[O_NSITES];
    o.max_u = r[O_MAXU];
    o.max_rho_r = r[O_MAXRR];
    o.perim_grad = r[O_PERIM];
    o.v_half = (long long)r[O_VHALF];
    o.v_mass = o.mass_r / rho_in_r;
    o.perim_sites = (double)o.n_sites / sbar;
    *out = o;
}

template <int Q, typename S, bool WALLS>
static hipError_t noalloc_impl(const cge_params* p, const void* pop, const uint8_t* flags,
                               const void* carry, unsigned char* base, hipStream_t stream,
                               cge_obs* out) {
    cge_ctx tmp;  // host-side constants only: phys() reads the parameters and lattice
    tmp.p = *p;
    tmp.Q = Q;
    const Geo g{p->nx, p->ny, p->nz, 0, (long long)p->nx * p->ny * p->nz};
    double* res = reinterpret_cast<double*>(base);
    double* part = reinterpret_cast<double*>(base + kNoallocRes);
    hipError_t e = obs_launch<Q, S, WALLS>(static_cast<const S*>(pop), flags, carry, part, res,
                                           nullptr, nullptr, 0, g, phys<double>(&tmp), stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_obs_noalloc_out, dim3(1), dim3(64), 0, stream, res, p->rho_in[0],
                       p->sbar, out);
    return hipGetLastError();
}

size_t noalloc_limit_bytes() { return kNoallocScratch - kNoallocRes; }
size_t noalloc_need_bytes(const cge_params* p) {
    const Geo g{p->nx, p->ny, p->nz, 0, (long long)p->nx * p->ny * p->nz};
    return obs_scratch_bytes(g);
}

cge_status observables_noalloc(const cge_params* p, const void* pop, const unsigned char* carry,
                               const unsigned char* flags, void* hip_stream, cge_obs* out) {
    if (noalloc_need_bytes(p) > noalloc_limit_bytes()) return CGE_ESCRATCH;
    void* base = nullptr;
    if (scratch_on_current_device(&base) != hipSuccess) return CGE_EDEVICE;
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    unsigned char* b = static_cast<unsigned char*>(base);
    const int key = p->lattice * 10 + p->precision;
    const bool w = flags != nullptr;
    hipError_t e;
    switch (key) {
        case 90: e = w ? noalloc_impl<9, double, true>(p, pop, flags, carry, b, st, out)
                       : noalloc_impl<9, double, false>(p, pop, flags, carry, b, st, out); break;
        case 91: e = w ? noalloc_impl<9, float, true>(p, pop, flags, carry, b, st, out)
                       : noalloc_impl<9, float, false>(p, pop, flags, carry, b, st, out); break;
        case 92: e = w ? noalloc_impl<9, _Float16, true>(p, pop, flags, carry, b, st, out)
                       : noalloc_impl<9, _Float16, false>(p, pop, flags, carry, b, st, out); break;
        case 190: e = w ? noalloc_impl<19, double, true>(p, pop, flags, carry, b, st, out)
                        : noalloc_impl<19, double, false>(p, pop, flags, carry, b, st, out); break;
        case 191: e = w ? noalloc_impl<19, float, true>(p, pop, flags, carry, b, st, out)
                        : noalloc_impl<19, float, false>(p, pop, flags, carry, b, st, out); break;
        case 192: e = w ? noalloc_impl<19, _Float16, true>(p, pop, flags, carry, b, st, out)
                        : noalloc_impl<19, _Float16, false>(p, pop, flags, carry, b, st, out); break;
        default: return CGE_EUNSUPPORTED;
    }
    return e == hipSuccess ? CGE_OK : CGE_EDEVICE;
}

}  // namespace cge
