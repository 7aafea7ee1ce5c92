// Two-pass step: k_phase writes the post-sink phase field rho^N of every fluid node,
// k_wet fills solid nodes with the neutral-wetting value, k_collide pulls again, applies
// the sink, takes rho^N and the colour gradient from the rho^N field, collides, perturbs,
// recolours, stores, and writes the next step's site mask.  One thread per node; works for
// any domain and any solid geometry.  The rho^N field is stored like the populations (float
// next to FP32 or FP16 populations, double next to FP64 ones).
#include "internal.hpp"
#include "node.hpp"

namespace cge {


// Pass 1: post-sink rho^N of fluid nodes (apply_sink = 0: pre-sink, for the step-0 mask),
// stored in type R.
template <int Q, typename S, typename M, bool WALLS, typename R>
__global__ __launch_bounds__(kTPBX) void k_phase(const S* __restrict__ src,
                                                 const uint8_t* __restrict__ flags,
                                                 const void* __restrict__ carry,
                                                 const void* __restrict__ phi_field,
                                                 R* __restrict__ rhoN, Geo g, Phys<M> P,
                                                 int apply_sink) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (WALLS && flags[n]) return;
    const Nb b = wrap(g, x, y, z);
    M ft[Q], dd[Q], j[3], drho, dsum;
    pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
    moments<Q>(ft, dd, drho, dsum, j);
    const M rho = P.rho_ref + drho;
    if (apply_sink) dsum -= M(2) * site_sink<S>(P, carry, phi_field, n, rho, dsum);
    rhoN[n] = static_cast<R>(dsum / rho);
}

// Site data (mask byte, or ||F|| for the soft rule) from the rho^N field, without
// collision; solid nodes get 0.
template <int Q, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_carry(const uint8_t* __restrict__ flags,
                                                 const M* __restrict__ rhoN,
                                                 void* __restrict__ carry, Geo g, Phys<M> P) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (WALLS && flags[n]) {
        carry_store<M>(P, carry, n, M(0));
        return;
    }
    const Nb b = wrap(g, x, y, z);
    M F[3];
    gradient<Q>(rhoN, g, b, x, y, z, F);
    carry_store<M>(P, carry, n, sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]));
}

// Pass 2: the full step at one node.
template <int Q, typename S, typename M, bool WALLS, bool NTS>
__global__ __launch_bounds__(kTPBX) void k_collide(const S* __restrict__ src, S* __restrict__ dst,
                                                   const uint8_t* __restrict__ flags,
                                                   void* __restrict__ carry,
                                                   const void* __restrict__ phi_field,
                                                   const MomT<S>* __restrict__ rhoN,
                                                   double* __restrict__ acc_sink,
                                                   long long* __restrict__ acc_sites, Geo g,
                                                   Phys<M> P, uint64_t salt) {
    int x, y, z;
    long long n;
    const bool valid = node_xyz(g, x, y, z, n);
    double v[2] = {0.0, 0.0};
    if (valid && !(WALLS && flags[n])) {
        const Nb b = wrap(g, x, y, z);
        M ft[Q], dd[Q], j[3], drho, dsum;
        pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
        moments<Q>(ft, dd, drho, dsum, j);
        const M rho = P.rho_ref + drho;
        M w;
        const M s = site_sink<S>(P, carry, phi_field, n, rho, dsum, w);
        dd[0] -= M(2) * s;
        dsum -= M(2) * s;
        v[0] = static_cast<double>(s);
        v[1] = is_site(w) ? 1.0 : 0.0;
        const M inv_rho = M(1) / rho;
        const M u[3] = {j[0] * inv_rho, j[1] * inv_rho, j[2] * inv_rho};
        const M rN = static_cast<M>(rhoN[n]);  // as stored by the first pass
        M F[3];
        gradient<Q>(rhoN, g, b, x, y, z, F);
        const M Fn = collide<Q>([&](int i) { return ft[i]; }, drho, rho, rN, u, F, P,
                                [&](int i, M a, M d) {
                                    st_nt<NTS>(dst + (long long)i * g.N + n, a, sr_bits(salt, g.N, n, 2 * i));
                                    st_nt<NTS>(dst + (long long)(Q + i) * g.N + n, d,
                                          sr_bits(salt, g.N, n, 2 * i + 1));
                                });
        carry_store<M>(P, carry, n, Fn);
    }
    const bool is_max[2] = {false, false};
    double out[2];
    block_reduce<2>(v, is_max, threadIdx.x, blockDim.x, out);
    if (threadIdx.x == 0) {
        const long long bid = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
        acc_sink[bid] += out[0];
        acc_sites[bid] += static_cast<long long>(out[1]);
    }
}

long long twopass_blocks(const cge_ctx* c) {
    const dim3 gr = node_grid(c->g);
    return (long long)gr.x * gr.y * gr.z;
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status twopass_impl(cge_ctx* c, long long nsteps) {
    const Phys<M> P = phys<M>(c);
    const dim3 gr = node_grid(c->g), bl = node_block(c->g);
    MomT<S>* rhoN = static_cast<MomT<S>*>(c->rhoN);  // stored like the populations
    const uint64_t seedmix = mix64(c->p.seed);
    for (long long t = 0; t < nsteps; ++t) {
        const S* src = static_cast<const S*>(c->pop[c->cur]);
        S* dst = static_cast<S*>(c->pop[1 - c->cur]);
        const uint64_t salt = mix64(seedmix + (uint64_t)c->step) * 0x100000001B3ull;
        timing_begin(c, "two-pass step");
        hipLaunchKernelGGL((k_phase<Q, S, M, WALLS, MomT<S>>), gr, bl, 0, c->stream, src,
                           c->flags, c->carry, c->phi_field, rhoN, c->g, P, 1);
        if (WALLS)
            hipLaunchKernelGGL((k_wet<Q, MomT<S>>), gr, bl, 0, c->stream, c->flags, rhoN, c->g);
        timing_pass(c, "k_phase");
        by_policy(c->g.nt, kNtPop, [&](auto nts) {
            hipLaunchKernelGGL((k_collide<Q, S, M, WALLS, decltype(nts)::value>), gr, bl, 0,
                               c->stream, src, dst, c->flags, c->carry, c->phi_field, rhoN,
                               c->acc_sink, c->acc_sites, c->g, P, salt);
        });
        timing_pass(c, "k_collide");
        timing_end(c);
        if (cge_status s = check(c, hipGetLastError(), "step kernel launch")) return s;
        c->cur = 1 - c->cur;
        c->step += 1;
    }
    return CGE_OK;
}

cge_status twopass_steps(cge_ctx* c, long long nsteps) { CGE_DISPATCH(c, twopass_impl, c, nsteps); }

template <int Q, typename S, typename M, bool WALLS>
static cge_status reset_impl(cge_ctx* c) {
    const Phys<M> P = phys<M>(c);
    const dim3 gr = node_grid(c->g), bl = node_block(c->g);
    M* rhoN = static_cast<M*>(c->rhoN);
    hipLaunchKernelGGL((k_phase<Q, S, M, WALLS, M>), gr, bl, 0, c->stream,
                       static_cast<const S*>(c->pop[c->cur]), c->flags, c->carry, c->phi_field,
                       rhoN, c->g, P, 0);
    if (WALLS) hipLaunchKernelGGL((k_wet<Q, M>), gr, bl, 0, c->stream, c->flags, rhoN, c->g);
    hipLaunchKernelGGL((k_carry<Q, M, WALLS>), gr, bl, 0, c->stream, c->flags, rhoN, c->carry,
                       c->g, P);
    return check(c, hipGetLastError(), "site-mask kernels");
}

cge_status reset_sites(cge_ctx* c) { CGE_DISPATCH(c, reset_impl, c); }

// Wetting values of solid nodes in any rho^N field (used by the field export).
template <typename R>
cge_status wet_field(cge_ctx* c, R* rhoN) {
    const dim3 gr = node_grid(c->g), bl = node_block(c->g);
    if (c->Q == 9) hipLaunchKernelGGL((k_wet<9, R>), gr, bl, 0, c->stream, c->flags, rhoN, c->g);
    else hipLaunchKernelGGL((k_wet<19, R>), gr, bl, 0, c->stream, c->flags, rhoN, c->g);
    return check(c, hipGetLastError(), "wetting kernel");
}
template cge_status wet_field<float>(cge_ctx*, float*);
template cge_status wet_field<double>(cge_ctx*, double*);

}  // namespace cge
