// State conversion between plain FP64 populations (post-streaming, f^r and f^b) and the
// library's encoded post-collision pull layout, plus equilibrium initialisation and the
// per-node FP64 field export.
#include "internal.hpp"
#include "node.hpp"

namespace cge {

// Rounding of an imported FP64 value to the storage type.  Half storage rounds
// stochastically, as the step does: a uniform initial state rounded to nearest would give every
// bulk node the same rounding error, which adds up to a mass offset over the domain.
template <typename S>
__device__ __forceinline__ S enc_import(double v, uint32_t bits) {
    if constexpr (std::is_same<S, _Float16>::value)
        return enc<_Float16, float>(static_cast<float>(v), bits);
    else
        return static_cast<S>(v);
}

// Store the post-streaming pair (fr, fb) of direction i at node n into the slot the next
// pull reads it from: (i, n - c_i), or (opp(i), n) when n - c_i is solid.
template <int Q, typename S, bool WALLS>
__device__ __forceinline__ void store_prestream(S* __restrict__ dst, const uint8_t* __restrict__ flags,
                                                const Geo& g, const Nb& b, int x, int y, int z,
                                                long long n, int i, double fr, double fb,
                                                double rho_ref, double alpha_ref, uint64_t salt) {
    long long sn = shifted<Q, -1>(g, b, x, y, z, i);
    int di = i;
    if (WALLS && i != 0 && flags[sn]) {
        sn = n;
        di = Lat<Q>::opp[i];
    }
    // the shift and encoding depend on the direction the value is stored under; the
    // bounce-back pair (i, opp(i)) shares the same rest weight, so either index gives it
    const double tref = rho_ref * (restA<Q>(i) + restB<Q>(i) * alpha_ref);
    dst[(long long)di * g.N + sn] = enc_import<S>(fr + fb - tref, sr_bits(salt, g.N, sn, 2 * di));
    dst[(long long)(Q + di) * g.N + sn] = enc_import<S>(fr - fb, sr_bits(salt, g.N, sn, 2 * di + 1));
}

template <int Q, typename S, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_init(S* __restrict__ dst, const uint8_t* __restrict__ flags,
                                                const double* __restrict__ rr,
                                                const double* __restrict__ rb,
                                                const double* __restrict__ u, Geo g,
                                                Phys<double> P, uint64_t salt) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (WALLS && flags[n]) return;
    const Nb b = wrap(g, x, y, z);
    double uv[3] = {0.0, 0.0, 0.0};
    if (u)
        for (int a = 0; a < Lat<Q>::D; ++a) uv[a] = u[(long long)a * g.N + n];
    const double uu = uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = Lat<Q>::cx[i] * uv[0] + Lat<Q>::cy[i] * uv[1] + Lat<Q>::cz[i] * uv[2];
        const double vel = weight<Q>(i) * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        const double fr = rr[n] * (restA<Q>(i) + restB<Q>(i) * P.alpha_r + vel);
        const double fb = rb[n] * (restA<Q>(i) + restB<Q>(i) * P.alpha_b + vel);
        store_prestream<Q, S, WALLS>(dst, flags, g, b, x, y, z, n, i, fr, fb, P.rho_ref,
                                     P.alpha_ref, salt);
    }
}

template <int Q, typename S, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_import(S* __restrict__ dst, const uint8_t* __restrict__ flags,
                                                  const double* __restrict__ f, Geo g,
                                                  Phys<double> P, uint64_t salt) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (WALLS && flags[n]) return;
    const Nb b = wrap(g, x, y, z);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        store_prestream<Q, S, WALLS>(dst, flags, g, b, x, y, z, n, i, f[(long long)i * g.N + n],
                                     f[(long long)(Q + i) * g.N + n], P.rho_ref, P.alpha_ref,
                                     salt);
}

template <int Q, typename S, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_export(const S* __restrict__ src,
                                                  const uint8_t* __restrict__ flags,
                                                  double* __restrict__ f, Geo g, Phys<double> P) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (WALLS && flags[n]) {
        for (int i = 0; i < 2 * Q; ++i) f[(long long)i * g.N + n] = 0.0;
        return;
    }
    const Nb b = wrap(g, x, y, z);
    double ft[Q], dd[Q];
    pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double full = ft[i] + P.rho_ref * (restA<Q>(i) + restB<Q>(i) * P.alpha_ref);
        f[(long long)i * g.N + n] = 0.5 * (full + dd[i]);
        f[(long long)(Q + i) * g.N + n] = 0.5 * (full - dd[i]);
    }
}

template <int Q, typename S, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_fields(const S* __restrict__ src,
                                                  const uint8_t* __restrict__ flags,
                                                  double* __restrict__ rr, double* __restrict__ rb,
                                                  double* __restrict__ u, double* __restrict__ rhoN,
                                                  Geo g, Phys<double> P) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    double r = 0.0, bl = 0.0, j[3] = {0.0, 0.0, 0.0};
    if (!(WALLS && flags[n])) {
        const Nb b = wrap(g, x, y, z);
        double ft[Q], dd[Q];
        pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double full = ft[i] + P.rho_ref * (restA<Q>(i) + restB<Q>(i) * P.alpha_ref);
            const double a = 0.5 * (full + dd[i]), c = 0.5 * (full - dd[i]);
            r += a;
            bl += c;
            j[0] += Lat<Q>::cx[i] * (a + c);
            j[1] += Lat<Q>::cy[i] * (a + c);
            j[2] += Lat<Q>::cz[i] * (a + c);
        }
    }
    const double rho = r + bl;
    if (rr) rr[n] = r;
    if (rb) rb[n] = bl;
    if (u)
        for (int a = 0; a < Lat<Q>::D; ++a) u[(long long)a * g.N + n] = rho > 0.0 ? j[a] / rho : 0.0;
    if (rhoN) rhoN[n] = rho > 0.0 ? (r - bl) / rho : 0.0;
}

// rounding keys of imported states: a stream of their own, apart from the steps' keys
static uint64_t import_salt(const cge_ctx* c) {
    return mix64(mix64(c->p.seed) ^ 0x9E3779B97F4A7C15ull) * 0x100000001B3ull;
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status init_impl(cge_ctx* c, const double* rr, const double* rb, const double* u) {
    hipLaunchKernelGGL((k_init<Q, S, WALLS>), node_grid(c->g), node_block(c->g), 0, c->stream,
                       static_cast<S*>(c->pop[c->cur]), c->flags, rr, rb, u, c->g, phys<double>(c),
                       import_salt(c));
    return check(c, hipGetLastError(), "init kernel");
}
cge_status init_equilibrium(cge_ctx* c, const double* rr, const double* rb, const double* u) {
    CGE_DISPATCH(c, init_impl, c, rr, rb, u);
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status import_impl(cge_ctx* c, const double* f) {
    hipLaunchKernelGGL((k_import<Q, S, WALLS>), node_grid(c->g), node_block(c->g), 0, c->stream,
                       static_cast<S*>(c->pop[c->cur]), c->flags, f, c->g, phys<double>(c),
                       import_salt(c));
    return check(c, hipGetLastError(), "import kernel");
}
cge_status set_populations(cge_ctx* c, const double* f) { CGE_DISPATCH(c, import_impl, c, f); }

template <int Q, typename S, typename M, bool WALLS>
static cge_status export_impl(cge_ctx* c, double* f) {
    hipLaunchKernelGGL((k_export<Q, S, WALLS>), node_grid(c->g), node_block(c->g), 0, c->stream,
                       static_cast<const S*>(c->pop[c->cur]), c->flags, f, c->g, phys<double>(c));
    return check(c, hipGetLastError(), "export kernel");
}
cge_status get_populations(cge_ctx* c, double* f) { CGE_DISPATCH(c, export_impl, c, f); }

template <int Q, typename S, typename M, bool WALLS>
static cge_status fields_impl(cge_ctx* c, double* rr, double* rb, double* u, double* rhoN) {
    hipLaunchKernelGGL((k_fields<Q, S, WALLS>), node_grid(c->g), node_block(c->g), 0, c->stream,
                       static_cast<const S*>(c->pop[c->cur]), c->flags, rr, rb, u, rhoN, c->g,
                       phys<double>(c));
    if (cge_status s = check(c, hipGetLastError(), "field kernel")) return s;
    if (WALLS && rhoN) return wet_field<double>(c, rhoN);
    return CGE_OK;
}
cge_status fields(cge_ctx* c, double* rr, double* rb, double* u, double* rhoN) {
    CGE_DISPATCH(c, fields_impl, c, rr, rb, u, rhoN);
}

}  // namespace cge
