// Height-dependent flux (Sec. III, space- and time-varying flux; Eq. heated): the flux of a
// drop on a substrate is Phi = phi_S / (K + h / h_s), where h is the local drop height.
//
// The substrate normal is the last lattice axis (z for D3Q19, y for D2Q9).  The height of a
// column of nodes along it is the column's red thickness, the sum over its fluid nodes of the
// red fraction (1 + rho^N)/2 of the current (pre-sink) state, and every node of the column
// gets the column's flux.  The field depends on the current state only, so it is refreshed
// from the state before a step (every `every` steps) and a run resumed from a saved state
// takes the same fluxes as an uninterrupted one.
//
// One thread per column; a block covers consecutive x at one y, so the loop along the column
// reads each population slot with unit stride across the lanes.  The read is a pass over the
// whole state (2Q values per node) plus one flux value written per node.
#include "internal.hpp"
#include "node.hpp"

namespace cge {

template <int Q, typename S, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_height_flux(const S* __restrict__ src,
                                                       const uint8_t* __restrict__ flags,
                                                       PhiT<S>* __restrict__ phi, Geo g,
                                                       Phys<M> P, double phi_s, double K,
                                                       double h_scale) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const bool three = Lat<Q>::D == 3;
    const int len = three ? g.nz : g.ny;  // nodes along the column
    double h = 0.0;
    for (int k = 0; k < len; ++k) {
        const int y = three ? (int)blockIdx.y : k;
        const int z = three ? k : 0;
        const long long n = lin(g, x, y, z);
        if (WALLS && flags[n]) continue;
        const Nb b = wrap(g, x, y, z);
        M ft[Q], dd[Q], j[3], drho, dsum;
        pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
        moments<Q>(ft, dd, drho, dsum, j);
        h += 0.5 * (1.0 + static_cast<double>(dsum) / static_cast<double>(P.rho_ref + drho));
    }
    const PhiT<S> f = static_cast<PhiT<S>>(phi_s / (K + h / h_scale));
    for (int k = 0; k < len; ++k) {
        const int y = three ? (int)blockIdx.y : k;
        const int z = three ? k : 0;
        phi[lin(g, x, y, z)] = f;
    }
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status height_flux_impl(cge_ctx* c) {
    const dim3 bl = node_block(c->g);
    const dim3 gr((c->g.nx + bl.x - 1) / bl.x, Lat<Q>::D == 3 ? c->g.ny : 1, 1);
    hipLaunchKernelGGL((k_height_flux<Q, S, M, WALLS>), gr, bl, 0, c->stream,
                       static_cast<const S*>(c->pop[c->cur]), c->flags,
                       static_cast<PhiT<S>*>(const_cast<void*>(c->phi_field)), c->g, phys<M>(c),
                       c->hf_phi, c->hf_K, c->hf_hs);
    return check(c, hipGetLastError(), "height flux launch");
}

cge_status height_flux(cge_ctx* c) { CGE_DISPATCH(c, height_flux_impl, c); }

}  // namespace cge
