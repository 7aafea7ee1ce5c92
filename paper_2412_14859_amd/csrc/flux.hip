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
// Two passes, both one thread per chunk of kChunk consecutive nodes of a column: the first
// pulls every node of its chunk and writes the chunk's red thickness (FP64), the second sums
// the column's chunk values in order and writes the flux of its chunk's nodes.  A block
// covers consecutive x, so every access has unit stride across the lanes.  The read is one
// pass over the whole state (2Q values per node), plus one flux value written per node.
#include "internal.hpp"
#include "node.hpp"

namespace cge {

constexpr int kChunk = 8;

template <int Q>
__device__ __forceinline__ void chunk_coords(const Geo& g, int& y, int& z0, int& len, int& c) {
    const bool three = Lat<Q>::D == 3;
    len = three ? g.nz : g.ny;  // nodes along the column
    c = three ? (int)blockIdx.z : (int)blockIdx.y;
    y = three ? (int)blockIdx.y : 0;
    z0 = c * kChunk;
}

template <int Q, typename S, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_height_partial(const S* __restrict__ src,
                                                          const uint8_t* __restrict__ flags,
                                                          double* __restrict__ part, Geo g,
                                                          Phys<M> P) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    int yb, k0, len, c;
    chunk_coords<Q>(g, yb, k0, len, c);
    const bool three = Lat<Q>::D == 3;
    double h = 0.0;
    for (int k = k0; k < k0 + kChunk && k < len; ++k) {
        const int y = three ? yb : k;
        const int z = three ? k : 0;
        const long long n = lin(g, x, y, z);
        if (WALLS && flags[n]) continue;
        const Nb b = wrap(g, x, y, z);
        M ft[Q], dd[Q], j[3], drho, dsum;
        pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
        moments<Q>(ft, dd, drho, dsum, j);
        h += 0.5 * (1.0 + static_cast<double>(dsum) / static_cast<double>(P.rho_ref + drho));
    }
    // part[c][yb][x]
    part[((long long)c * (three ? g.ny : 1) + yb) * g.nx + x] = h;
}

template <int Q, typename S>
__global__ __launch_bounds__(kTPBX) void k_height_write(const double* __restrict__ part,
                                                        PhiT<S>* __restrict__ phi, Geo g,
                                                        double phi_s, double K, double h_scale) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    int yb, k0, len, c;
    chunk_coords<Q>(g, yb, k0, len, c);
    const bool three = Lat<Q>::D == 3;
    const int nch = (len + kChunk - 1) / kChunk;
    const long long stride = (long long)(three ? g.ny : 1) * g.nx;
    double h = 0.0;
    for (int q = 0; q < nch; ++q) h += part[q * stride + (long long)yb * g.nx + x];
    const PhiT<S> f = static_cast<PhiT<S>>(phi_s / (K + h / h_scale));
    for (int k = k0; k < k0 + kChunk && k < len; ++k) {
        const int y = three ? yb : k;
        const int z = three ? k : 0;
        phi[lin(g, x, y, z)] = f;
    }
}

size_t height_partial_bytes(const Geo& g, int Q) {
    const int len = Q == 19 ? g.nz : g.ny;
    const long long other = Q == 19 ? g.ny : 1;
    return sizeof(double) * (size_t)g.nx * other * ((len + kChunk - 1) / kChunk);
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status height_flux_impl(cge_ctx* c) {
    if (!c->hf_part) return fail(c, CGE_ESTATE, "height flux scratch missing");
    const dim3 bl = node_block(c->g);
    const bool three = Lat<Q>::D == 3;
    const int len = three ? c->g.nz : c->g.ny;
    const int nch = (len + kChunk - 1) / kChunk;
    const dim3 gr((c->g.nx + bl.x - 1) / bl.x, three ? c->g.ny : nch, three ? nch : 1);
    double* part = static_cast<double*>(c->hf_part);
    hipLaunchKernelGGL((k_height_partial<Q, S, M, WALLS>), gr, bl, 0, c->stream,
                       static_cast<const S*>(c->pop[c->cur]), c->flags, part, c->g, phys<M>(c));
    hipLaunchKernelGGL((k_height_write<Q, S>), gr, bl, 0, c->stream, part,
                       static_cast<PhiT<S>*>(const_cast<void*>(c->phi_field)), c->g, c->hf_phi,
                       c->hf_K, c->hf_hs);
    return check(c, hipGetLastError(), "height flux launch");
}

cge_status height_flux(cge_ctx* c) { CGE_DISPATCH(c, height_flux_impl, c); }

}  // namespace cge
