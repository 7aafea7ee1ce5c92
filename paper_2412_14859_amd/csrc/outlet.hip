// Pressure outlet (Zou and He) for the blue component on the end planes of the last lattice
// axis a (z for D3Q19, y for D2Q9), as used with density contrast in Sec. III.
//
// The populations entering the domain through an outlet plane (c_i . n = -1, n the outward
// normal) are unknown after streaming.  With the blue density held at rho_out and no
// tangential velocity they are
//     u_n = (sum_{c.n=0} f + 2 sum_{c.n=1} f) / rho_out - 1,
//     f_i = f_opp(i) - 6 W_i rho_out u_n - sum_{t != a} c_it N_t,  N_t = (1/2) sum_{c.n=0} f_j c_jt
// (the odd part of the equilibrium, 6 W_i rho c_i.u, does not depend on alpha; N_t removes the
// tangential momentum).  No red fluid enters: its unknown populations are 0.
//
// The steps stream by pulling, and with periodic wrap an outlet node pulls its unknown
// populations from slots on the opposite plane that no other node reads.  So the outlet is a
// fix-up after each step (and when a state is set): per outlet node, read the known pulled
// populations, and write the unknowns into the slots the next pull reads them from.  A node
// reads only slots of its own and its inner neighbour plane and writes only slots on the
// opposite end plane, so the nodes of both planes never touch each other's data.
#include "internal.hpp"
#include "node.hpp"

namespace cge {

template <int Q, typename S, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_outlet(S* __restrict__ pop,
                                                  const uint8_t* __restrict__ flags, Geo g,
                                                  Phys<double> P, int lo, int hi, double rho_out,
                                                  uint64_t salt) {
    constexpr int a = Lat<Q>::D == 3 ? 2 : 1;  // lattice axis of the outlet normal
    const int side = (int)blockIdx.z;            // 0: plane at index 0, 1: last index
    if (side == 0 ? !lo : !hi) return;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const int last = (a == 2 ? g.nz : g.ny) - 1;
    const int y = a == 2 ? (int)blockIdx.y : (side ? last : 0);
    const int z = a == 2 ? (side ? last : 0) : 0;
    const long long n = lin(g, x, y, z);
    if (WALLS && flags[n]) return;
    const int sgn = side ? 1 : -1;
    const Nb b = wrap(g, x, y, z);
    double ft[Q], dd[Q];
    pull<Q, WALLS>(pop, flags, g, b, x, y, z, n, ft, dd);
    double fb[Q];
    double s0 = 0.0, s1 = 0.0, N[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int c[3] = {Lat<Q>::cx[i], Lat<Q>::cy[i], Lat<Q>::cz[i]};
        const double tref = P.rho_ref * (restA<Q>(i) + restB<Q>(i) * P.alpha_ref);
        fb[i] = 0.5 * (ft[i] + tref - dd[i]);
        const int cn = sgn * c[a];
        if (cn == 0) {
            s0 += fb[i];
#pragma unroll
            for (int t = 0; t < 3; ++t)
                if (t != a && c[t]) N[t] += 0.5 * c[t] * fb[i];
        } else if (cn == 1) {
            s1 += fb[i];
        }
    }
    const double un = (s0 + 2.0 * s1) / rho_out - 1.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int c[3] = {Lat<Q>::cx[i], Lat<Q>::cy[i], Lat<Q>::cz[i]};
        if (sgn * c[a] != -1) continue;
        double f = fb[Lat<Q>::opp[i]] - 6.0 * weight<Q>(i) * rho_out * un;
#pragma unroll
        for (int t = 0; t < 3; ++t)
            if (t != a && c[t]) f -= c[t] * N[t];
        // the slot this node pulls direction i from (as in pull: bounce-back from a solid)
        long long sn = shifted<Q, -1>(g, b, x, y, z, i);
        int di = i;
        if (WALLS && flags[sn]) {
            sn = n;
            di = Lat<Q>::opp[i];
        }
        const double tref = P.rho_ref * (restA<Q>(di) + restB<Q>(di) * P.alpha_ref);
        st(pop + (long long)di * g.N + sn, static_cast<M>(f - tref),
           sr_bits(salt, g.N, sn, 2 * di));  // f^r = 0
        st(pop + (long long)(Q + di) * g.N + sn, static_cast<M>(-f), sr_bits(salt, g.N, sn, 2 * di + 1));
    }
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status outlet_impl(cge_ctx* c) {
    const dim3 bl = node_block(c->g);
    const dim3 gr((c->g.nx + bl.x - 1) / bl.x, Lat<Q>::D == 3 ? c->g.ny : 1, 2);
    const uint64_t salt =
        mix64(mix64(c->p.seed) ^ 0xD1B54A32D192ED03ull ^ (uint64_t)c->step) * 0x100000001B3ull;
    hipLaunchKernelGGL((k_outlet<Q, S, M, WALLS>), gr, bl, 0, c->stream,
                       static_cast<S*>(c->pop[c->cur]), c->flags, c->g, phys<double>(c),
                       c->out_lo, c->out_hi, c->out_rho, salt);
    return check(c, hipGetLastError(), "outlet launch");
}

cge_status apply_outlets(cge_ctx* c) {
    if (!c->out_lo && !c->out_hi) return CGE_OK;
    CGE_DISPATCH(c, outlet_impl, c);
}

}  // namespace cge
