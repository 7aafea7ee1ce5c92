// Split step for unit relaxation times (tau_r = tau_b = 1): two passes, populations read once.
//
// With 1/tau = 1 at every node, BGK relaxation returns the equilibrium (Eq. collision), so
// the post-collision populations depend on the pulled ones only through the post-sink
// moments: rho (via drho = sum ft_i), rho^N and j.  The first pass pulls, applies the sink
// and writes those moments (rho^N, drho and j in the storage type's width: FP64 next to FP64
// populations, FP32 otherwise, like the populations themselves); the second pass reads them back,
// takes the colour gradient from the rho^N field, and runs equilibrium, perturbation and
// recolouring (Eqs. feq, perturb, recolor) without touching the old populations.
//
// Per node: 2Q reads + 2Q writes of populations, plus the moment record written and read
// once (20 B at FP32 storage) and the neighbours' rho^N (cache hits).  Both kernels are one
// thread per node with no synchronisation, so many waves hide memory latency.
#include "internal.hpp"
#include "node.hpp"

namespace cge {

// Pass 1: pull, sink, moments; FP64 sink bookkeeping per block.
template <int Q, typename S, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_moments(const S* __restrict__ src,
                                                   const uint8_t* __restrict__ flags,
                                                   const void* __restrict__ carry,
                                                   const void* __restrict__ phi_field,
                                                   MomT<S>* __restrict__ rhoN,
                                                   MomT<S>* __restrict__ mom,
                                                   double* __restrict__ acc_sink,
                                                   long long* __restrict__ acc_sites, Geo g,
                                                   Phys<M> P) {
    int x, y, z;
    long long n;
    const bool valid = node_xyz(g, x, y, z, n);
    const RowOff r = row_offsets<S>(g, x < g.nx ? x : 0);
    double v[2] = {0.0, 0.0};
    if (valid && !(WALLS && flags[n])) {
        M j[3] = {M(0), M(0), M(0)}, drho = M(0), dsum = M(0);
        if constexpr (WALLS) {
            const Nb b = wrap(g, x, y, z);
            M ft[Q], dd[Q];
            pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
            moments<Q>(ft, dd, drho, dsum, j);
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) {  // pull (Eq. Stream): from x - c_i
                const long long rowz = r.yrow[1 - Lat<Q>::cy[i]] + r.zpl[1 - Lat<Q>::cz[i]];
                const uint32_t xo = r.xo[1 - Lat<Q>::cx[i]];
                const M a = static_cast<M>(ld_at(src + (long long)i * g.N + rowz, xo));
                drho += a;
                dsum += static_cast<M>(ld_at(src + (long long)(Q + i) * g.N + rowz, xo));
                if (Lat<Q>::cx[i]) j[0] += Lat<Q>::cx[i] * a;
                if (Lat<Q>::cy[i]) j[1] += Lat<Q>::cy[i] * a;
                if (Lat<Q>::cz[i]) j[2] += Lat<Q>::cz[i] * a;
            }
        }
        const M rho = P.rho_ref + drho;
        M wgt;
        const M s = site_sink<S>(P, carry, phi_field, n, rho, dsum, wgt);
        dsum -= M(2) * s;
        v[0] = static_cast<double>(s);
        v[1] = is_site(wgt) ? 1.0 : 0.0;
        rhoN[n] = static_cast<MomT<S>>(dsum / rho);
        mom[n] = static_cast<MomT<S>>(drho);
        mom[g.N + n] = static_cast<MomT<S>>(j[0]);
        mom[2 * g.N + n] = static_cast<MomT<S>>(j[1]);
        mom[3 * g.N + n] = static_cast<MomT<S>>(j[2]);
    }
    const bool is_max[2] = {false, false};
    double out[2];
    block_reduce<2>(v, is_max, threadIdx.x, blockDim.x, out);
    if (threadIdx.x == 0) {
        const long long bid =
            blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
        acc_sink[bid] += out[0];
        acc_sites[bid] += static_cast<long long>(out[1]);
    }
}

// Pass 2: gradient, equilibrium, perturbation, recolouring, store, next site mask.
// At least 5 waves per SIMD (the register budget allows it without spills): more stores in
// flight.
template <int Q, typename S, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_finish(S* __restrict__ dst,
                                                  const uint8_t* __restrict__ flags,
                                                  void* __restrict__ carry,
                                                  const MomT<S>* __restrict__ rhoN,
                                                  const MomT<S>* __restrict__ mom, Geo g,
                                                  Phys<M> P, uint64_t salt) {
    int x, y, z;
    long long n;
    const bool valid = node_xyz(g, x, y, z, n);
    const RowOff r = row_offsets<MomT<S>>(g, x < g.nx ? x : 0);  // x offsets into rho^N
    if (!valid) return;
    if (WALLS && flags[n]) return;
    const M drho = static_cast<M>(mom[n]);
    const M rho = P.rho_ref + drho;
    const M inv_rho = M(1) / rho;
    const M u[3] = {static_cast<M>(mom[g.N + n]) * inv_rho,
                    static_cast<M>(mom[2 * g.N + n]) * inv_rho,
                    static_cast<M>(mom[3 * g.N + n]) * inv_rho};
    M F[3];
    if constexpr (WALLS) {
        const Nb b = wrap(g, x, y, z);
        gradient<Q>(rhoN, g, b, x, y, z, F);
    } else {  // F = 3 sum_i W_i rho^N(x + c_i) c_i
        F[0] = F[1] = F[2] = M(0);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const long long rowz = r.yrow[1 + Lat<Q>::cy[i]] + r.zpl[1 + Lat<Q>::cz[i]];
            const M v = M(weight<Q>(i)) * static_cast<M>(ld_at(rhoN + rowz, r.xo[1 + Lat<Q>::cx[i]]));
            if (Lat<Q>::cx[i]) F[0] += Lat<Q>::cx[i] * v;
            if (Lat<Q>::cy[i]) F[1] += Lat<Q>::cy[i] * v;
            if (Lat<Q>::cz[i]) F[2] += Lat<Q>::cz[i] * v;
        }
        F[0] *= M(3);
        F[1] *= M(3);
        F[2] *= M(3);
    }
    // stores at the node itself: the row base is uniform, x is the lane offset
    const long long row = r.yrow[1] + r.zpl[1];
    const uint32_t xb = (uint32_t)x * (uint32_t)sizeof(S);
    const M Fn = collide<Q, M, true>([](int) { return M(0); }, drho, rho, static_cast<M>(rhoN[n]), u, F, P,
                                     [&](int i, M a, M d) {
                                         const uint64_t key = salt + (uint64_t)(2 * i) * (uint64_t)g.N +
                                                              (uint64_t)n;
                                         S* pa = dst + (long long)i * g.N + row;
                                         S* pd = dst + (long long)(Q + i) * g.N + row;
                                         st_nt(reinterpret_cast<S*>(reinterpret_cast<char*>(pa) + xb), a, key);
                                         st_nt(reinterpret_cast<S*>(reinterpret_cast<char*>(pd) + xb), d,
                                               key + (uint64_t)g.N);
                                     });
    carry_store(P, carry, n, Fn);
}

// Pass 2 for D3Q19 without solid nodes in FP64 storage, one 64 x 4 tile of nodes per block:
// rho^N of the 3 planes x 6 rows x 66 columns around the tile is staged in LDS once, so the
// stencil reads about 4.6 values from memory per node instead of 18.  The arithmetic and its
// order are k_finish's, so the results are bit-identical.  A tile row is 64 nodes, so every
// output array is written in runs of 64 elements: 512 B in FP64, where the tile is 5 %
// faster than k_finish, but 256 B in FP32 and 128 B in FP16, where the shorter runs cost
// what the stencil saves (FP32 no gain, FP16 15 % slower), so those keep k_finish's rows
// of 256 nodes.
constexpr int kTileX = 64, kTileY = 4;

__device__ __forceinline__ int wrapm(int v, int n) { return ((v % n) + n) % n; }

template <typename S, typename M>
__global__ __launch_bounds__(kTileX* kTileY) __attribute__((amdgpu_waves_per_eu(5, 8))) void
k_finish_tile(S* __restrict__ dst, void* __restrict__ carry, const MomT<S>* __restrict__ rhoN,
              const MomT<S>* __restrict__ mom, Geo g, Phys<M> P, uint64_t salt) {
    constexpr int Q = 19, W = kTileX + 2, H = kTileY + 2, NT = kTileX * kTileY;
    __shared__ M tile[3][H][W];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + kTileX * ty;
    const int x0 = blockIdx.x * kTileX, y0 = blockIdx.y * kTileY, z = blockIdx.z;
    const long long plane = (long long)g.nx * g.ny;
    for (int e = tid; e < 3 * H * W; e += NT) {
        const int pz = e / (H * W), ry = (e / W) % H, cx = e % W;
        const int gx = wrapm(x0 - 1 + cx, g.nx), gy = wrapm(y0 - 1 + ry, g.ny);
        const int gz = wrapc(z - 1 + pz, g.nz);
        tile[pz][ry][cx] = rhoN[gx + (long long)g.nx * gy + plane * gz];
    }
    __syncthreads();
    const int x = x0 + tx, y = y0 + ty;
    if (x >= g.nx || y >= g.ny) return;
    M F[3] = {M(0), M(0), M(0)};  // F = 3 sum_i W_i rho^N(x + c_i) c_i
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const M v = M(weight<Q>(i)) *
                    tile[1 + Lat<Q>::cz[i]][1 + ty + Lat<Q>::cy[i]][1 + tx + Lat<Q>::cx[i]];
        if (Lat<Q>::cx[i]) F[0] += Lat<Q>::cx[i] * v;
        if (Lat<Q>::cy[i]) F[1] += Lat<Q>::cy[i] * v;
        if (Lat<Q>::cz[i]) F[2] += Lat<Q>::cz[i] * v;
    }
    F[0] *= M(3);
    F[1] *= M(3);
    F[2] *= M(3);
    const long long n = x + (long long)g.nx * y + plane * z;
    const M drho = static_cast<M>(mom[n]);
    const M rho = P.rho_ref + drho;
    const M inv_rho = M(1) / rho;
    const M u[3] = {static_cast<M>(mom[g.N + n]) * inv_rho,
                    static_cast<M>(mom[2 * g.N + n]) * inv_rho,
                    static_cast<M>(mom[3 * g.N + n]) * inv_rho};
    const M Fn = collide<Q, M, true>([](int) { return M(0); }, drho, rho, tile[1][1 + ty][1 + tx],
                                     u, F, P, [&](int i, M a, M d) {
                                         const uint64_t key =
                                             salt + (uint64_t)(2 * i) * (uint64_t)g.N + (uint64_t)n;
                                         st_nt(dst + (long long)i * g.N + n, a, key);
                                         st_nt(dst + (long long)(Q + i) * g.N + n, d,
                                               key + (uint64_t)g.N);
                                     });
    carry_store(P, carry, n, Fn);
}

bool split_supported(const cge_ctx* c) { return c->p.tau[0] == 1.0 && c->p.tau[1] == 1.0; }

size_t split_scratch_bytes(const cge_params* p) {
    const size_t e = p->precision == CGE_FP64 ? 8 : 4;
    return 4 * e * (size_t)p->nx * p->ny * p->nz;
}

// One step from the current population buffer with explicit site-data and moment buffers:
// the sink reads carry_in, the next step's site data goes to carry_out (the same buffer in a
// plain run), rho^N and the moments to rhoN / mom (kept by the adjoint's recomputation).
template <int Q, typename S, typename M, bool WALLS>
static cge_status split_one(cge_ctx* c, const void* carry_in, void* carry_out, void* rhoN_out,
                            void* mom_out) {
    const Phys<M> P = phys<M>(c);
    const dim3 gr = node_grid(c->g), bl = node_block(c->g);
    MomT<S>* rhoN = static_cast<MomT<S>*>(rhoN_out);  // stored like the moment record
    MomT<S>* mom = static_cast<MomT<S>*>(mom_out);
    const S* src = static_cast<const S*>(c->pop[c->cur]);
    S* dst = static_cast<S*>(c->pop[1 - c->cur]);
    const uint64_t salt = mix64(mix64(c->p.seed) + (uint64_t)c->step) * 0x100000001B3ull;
    timing_begin(c);
    hipLaunchKernelGGL((k_moments<Q, S, M, WALLS>), gr, bl, 0, c->stream, src, c->flags,
                       carry_in, c->phi_field, rhoN, mom, c->acc_sink, c->acc_sites, c->g, P);
    if (WALLS) hipLaunchKernelGGL((k_wet<Q, MomT<S>>), gr, bl, 0, c->stream, c->flags, rhoN, c->g);
    if constexpr (Q == 19 && !WALLS && std::is_same<S, double>::value) {
        const dim3 tb(kTileX, kTileY, 1);
        const dim3 tg((c->g.nx + kTileX - 1) / kTileX, (c->g.ny + kTileY - 1) / kTileY, c->g.nz);
        hipLaunchKernelGGL((k_finish_tile<S, M>), tg, tb, 0, c->stream, dst, carry_out, rhoN, mom,
                           c->g, P, salt);
    } else {
        hipLaunchKernelGGL((k_finish<Q, S, M, WALLS>), gr, bl, 0, c->stream, dst, c->flags,
                           carry_out, rhoN, mom, c->g, P, salt);
    }
    timing_end(c);
    if (cge_status s = check(c, hipGetLastError(), "split step launch")) return s;
    c->cur = 1 - c->cur;
    c->step += 1;
    return CGE_OK;
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status split_impl(cge_ctx* c, long long nsteps) {
    if (!split_supported(c)) return fail(c, CGE_EUNSUPPORTED, "split step needs tau = 1");
    if (!c->mom) return fail(c, CGE_ESTATE, "moment scratch missing");
    for (long long t = 0; t < nsteps; ++t)
        if (cge_status s = split_one<Q, S, M, WALLS>(c, c->carry, c->carry, c->rhoN, c->mom))
            return s;
    return CGE_OK;
}

cge_status split_steps(cge_ctx* c, long long nsteps) { CGE_DISPATCH(c, split_impl, c, nsteps); }

cge_status split_step_into(cge_ctx* c, const void* carry_in, void* carry_out, void* rhoN,
                           void* mom) {
    if (!split_supported(c)) return fail(c, CGE_EUNSUPPORTED, "split step needs tau = 1");
    CGE_DISPATCH(c, split_one, c, carry_in, carry_out, rhoN, mom);
}

}  // namespace cge
