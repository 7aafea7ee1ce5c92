// Per-node device arithmetic of the colour-gradient step (HIP path).
//
// Population encoding (all precisions): per direction i the library stores
//   ft_i = f_i^r + f_i^b - rho_ref t_i(alpha_ref)   (colour-blind deviation)
//   dd_i = f_i^r - f_i^b                             (colour difference)
// of the post-collision values; streaming is a pull.  Streaming is linear, so (ft, dd)
// stream exactly as (f^r, f^b).  The sink (Eq. exchange) leaves ft untouched and lowers
// dd_0 by 2s; rho = rho_ref + sum ft, rho_r - rho_b = sum dd.  Collision and perturbation
// act on the colour-blind population only; recolouring (Eq. recolor) then gives
//   dd_i* = rho^N f_i'' + 2 beta (rho_r rho_b / rho^2) cos(theta_i) rho t_i(abar),
// with rho_r/rho = (1 + rho^N)/2 and rho_r rho_b / rho^2 = (1 - rho^N^2)/4.
#pragma once

#include <type_traits>

#include "lattice.hpp"

namespace cge {

template <typename M, typename S>
__device__ __forceinline__ M ld(const S* p) {
    return static_cast<M>(*p);
}

// splitmix64 finaliser (Steele, Lea, Flood 2014): counter-based random bits
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Round v to half precision stochastically: the neighbour above |v| is taken with
// probability proportional to the distance from the one below, so the rounding is
// unbiased in expectation (needed for per-step sinks far below one half-precision ulp).
// Where half has a spacing coarser than float's (|v| >= 2^-24), the float bits below the
// half spacing are dropped after adding that many random bits: a carry out of them (to the
// next half number, possibly across a power of two) happens with probability equal to
// their value over the spacing, so the expectation is exact.  Below 2^-24 the result is 0
// or 2^-24, up with probability |v| 2^24 on a 2^-24 grid (bias at most 2^-48).  At and
// above the largest half (65504), and for inf and nan, it is rounded to nearest.
__device__ __forceinline__ _Float16 sr_half(float v, uint32_t r) {
    const uint32_t u = __builtin_bit_cast(uint32_t, v);
    const uint32_t a = u & 0x7FFFFFFFu;
    if (!(a < 0x477FE000u)) return static_cast<_Float16>(v);  // |v| >= 65504, inf, nan
    const int e = static_cast<int>(a >> 23);                  // biased float exponent
    uint32_t t;
    if (e >= 103) {
        // bits of the float fraction below the half spacing: 13 for normal halves, up to 23
        // in the subnormal range where the spacing stays 2^-24
        const int drop = e < 113 ? 126 - e : 13;
        const uint32_t mask = (1u << drop) - 1u;
        t = (a + (r & mask)) & ~mask;
    } else {
        const float p = __builtin_bit_cast(float, a) * 16777216.0f;             // |v| 2^24
        const float q = static_cast<float>(r >> 8) * 5.9604644775390625e-8f;   // k 2^-24
        t = q < p ? 0x33800000u : 0u;                                           // 2^-24 or 0
    }
    // t is a half number, so this conversion is exact
    return static_cast<_Float16>(__builtin_bit_cast(float, t | (u & 0x80000000u)));
}

// 32-bit finaliser of MurmurHash3 (Appleby): a bijection with full avalanche, used to turn a
// node's rounding key into random bits.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    return h ^ (h >> 16);
}

// Random bits for the stochastic rounding of stored value `slot` (0 .. 2Q - 1: ft_i in slot
// 2i, dd_i in slot 2i + 1) of node n in the step whose salt is `salt`: the finaliser of the key
// salt + slot N + n.  Within one step the keys of all stored values differ in their low 32
// bits while 2 Q N < 2^32 (above that, values far apart share random bits, which leaves each
// rounding unbiased), and the per-step salt randomises those bits.  Every value has bits of
// its own: deriving a node's values from one hash (a Weyl sequence over the slots) ties their
// low bits to one random offset, and the population error of the 128^2 drop after 2000 steps
// at frozen site sets grew from 3.1e-3 to 5.9e-3.
__device__ __forceinline__ uint32_t sr_bits(uint64_t salt, long long N, long long n, int slot) {
    return fmix32(static_cast<uint32_t>(salt + static_cast<uint64_t>(slot) * static_cast<uint64_t>(N) +
                                        static_cast<uint64_t>(n)));
}

// rounding to the storage type: nearest for double/float, stochastic for half (bits from
// sr_bits)
template <typename S, typename M>
__device__ __forceinline__ S enc(M v, uint32_t bits) {
    return static_cast<S>(v);
}
template <>
__device__ __forceinline__ _Float16 enc<_Float16, float>(float v, uint32_t bits) {
    return sr_half(v, bits);
}
// FP64 arithmetic into half storage: to FP32 by nearest (13 bits finer than half), then
// stochastically to half
template <>
__device__ __forceinline__ _Float16 enc<_Float16, double>(double v, uint32_t bits) {
    return sr_half(static_cast<float>(v), bits);
}
template <typename S, typename M>
__device__ __forceinline__ void st(S* p, M v, uint32_t bits) {
    *p = enc<S, M>(v, bits);
}
// The same with a streaming (non-temporal) hint where NT: the value is not read again in
// this step.  The policy is a template argument: with a run-time flag the compiler merges
// the two stores of the branch into one and drops the hint.
template <bool NT, typename S, typename M>
__device__ __forceinline__ void st_nt(S* p, M v, uint32_t bits) {
    if constexpr (NT)
        __builtin_nontemporal_store(enc<S, M>(v, bits), p);
    else
        *p = enc<S, M>(v, bits);
}
// a value stored with the streaming hint where NT
template <bool NT, typename T>
__device__ __forceinline__ void st_pol(T* p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// neighbour coordinates with periodic wrap
struct Nb {
    int xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Nb wrap(const Geo& g, int x, int y, int z) {
    Nb b;
    b.xm = x == 0 ? g.nx - 1 : x - 1;
    b.xp = x == g.nx - 1 ? 0 : x + 1;
    b.ym = y == 0 ? g.ny - 1 : y - 1;
    b.yp = y == g.ny - 1 ? 0 : y + 1;
    b.zm = z == 0 ? g.nz - 1 : z - 1;
    b.zp = z == g.nz - 1 ? 0 : z + 1;
    return b;
}

__device__ __forceinline__ long long lin(const Geo& g, int x, int y, int z) {
    return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

// one thread per node on a (ceil(nx/bx), ny, nz) grid of (bx, 1, 1) blocks
constexpr int kTPBX = 256;

__device__ __forceinline__ bool node_xyz(const Geo& g, int& x, int& y, int& z, long long& n) {
    x = blockIdx.x * blockDim.x + threadIdx.x;
    y = blockIdx.y;
    z = blockIdx.z;
    n = lin(g, x, y, z);
    return x < g.nx;
}

// node at x + s*c_i (s = +1 or -1)
template <int Q, int SGN>
__device__ __forceinline__ long long shifted(const Geo& g, const Nb& b, int x, int y, int z, int i) {
    const int cx = SGN * Lat<Q>::cx[i], cy = SGN * Lat<Q>::cy[i], cz = SGN * Lat<Q>::cz[i];
    const int sx = cx == 1 ? b.xp : (cx == -1 ? b.xm : x);
    const int sy = cy == 1 ? b.yp : (cy == -1 ? b.ym : y);
    const int sz = cz == 1 ? b.zp : (cz == -1 ? b.zm : z);
    return lin(g, sx, sy, sz);
}

// Periodic addressing of one block (one x-row segment at fixed y = blockIdx.y, z =
// blockIdx.z): the y and z parts of every neighbour index are the same for all lanes, so each
// (slot, row, plane) base is a scalar pointer and only the x offset (3 values per lane) varies.
struct RowOff {
    long long yrow[3], zpl[3];  // element offsets of rows y-1, y, y+1 and planes z-1, z, z+1
    uint32_t xo[3];             // byte offsets of x-1, x, x+1 (times the element size)
};

__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Call at kernel entry, before any lane-dependent branch.
template <typename T>
__device__ __forceinline__ RowOff row_offsets(const Geo& g, int x) {
    RowOff r;
    const int y = (int)blockIdx.y, z = (int)blockIdx.z;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // readfirstlane keeps the uniform offsets in scalar registers (they fit in 31 bits)
        const int yo = __builtin_amdgcn_readfirstlane(wrapc(y - 1 + d, g.ny) * g.nx);
        const int zo = __builtin_amdgcn_readfirstlane(wrapc(z - 1 + d, g.nz));
        r.yrow[d] = yo;
        r.zpl[d] = (long long)zo * ((long long)g.nx * g.ny);
        r.xo[d] = (uint32_t)wrapc(x - 1 + d, g.nx) * (uint32_t)sizeof(T);
    }
    return r;
}

// XCD-aware placement of the one-thread-per-node blocks.  Workgroups are dealt to the 8 XCDs
// round-robin by linear block id, and each XCD has its own L2.  Kernels whose nodes read
// their neighbours' rows (a stencil with reuse) renumber the blocks: rows are taken in bands
// of kBandY consecutive y, each band walking z (all x-blocks of a row, then the band's rows
// of a plane, then the next plane), and XCD k takes a contiguous run of that order.  The rows
// an XCD works on at one time then form a patch of kBandY rows by a few planes, whose
// neighbours (the patch plus one row and one plane around it) stay in its L2.  The map is a
// bijection of [0, blocks).
constexpr int kXcds = 8, kBandY = 16;
struct RowPos {
    int bx, y, z;  // x-block, row and plane of this block (uniform)
};
__device__ __forceinline__ RowPos xcd_row(const Geo& g) {
    const unsigned gx = gridDim.x, ny = gridDim.y, nz = gridDim.z;
    const unsigned nb = gx * ny * nz;
    const unsigned b = blockIdx.x + gx * (blockIdx.y + ny * blockIdx.z);
    const unsigned q = nb / kXcds, rem = nb % kXcds, k = b % kXcds, l = b / kXcds;
    const unsigned r = k * q + (k < rem ? k : rem) + l;  // position in band order
    const unsigned band_blocks = kBandY * nz * gx;       // blocks of one full band
    const unsigned band = r / band_blocks;
    const unsigned h = ny - band * kBandY < (unsigned)kBandY ? ny - band * kBandY : kBandY;
    const unsigned t = r - band * band_blocks;           // within the band
    RowPos p;
    p.bx = __builtin_amdgcn_readfirstlane((int)(t % gx));
    const unsigned yz = t / gx;
    p.y = __builtin_amdgcn_readfirstlane((int)(band * kBandY + yz % h));
    p.z = __builtin_amdgcn_readfirstlane((int)(yz / h));
    return p;
}
__device__ __forceinline__ bool node_xyz_at(const Geo& g, const RowPos& p, int& x, int& y, int& z,
                                            long long& n) {
    x = p.bx * blockDim.x + threadIdx.x;
    y = p.y;
    z = p.z;
    n = lin(g, x, y, z);
    return x < g.nx;
}
template <typename T>
__device__ __forceinline__ RowOff row_offsets_at(const Geo& g, const RowPos& p, int x) {
    RowOff r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int yo = __builtin_amdgcn_readfirstlane(wrapc(p.y - 1 + d, g.ny) * g.nx);
        const int zo = __builtin_amdgcn_readfirstlane(wrapc(p.z - 1 + d, g.nz));
        r.yrow[d] = yo;
        r.zpl[d] = (long long)zo * ((long long)g.nx * g.ny);
        r.xo[d] = (uint32_t)wrapc(x - 1 + d, g.nx) * (uint32_t)sizeof(T);
    }
    return r;
}

// A pointer known to be the same in every lane, kept in scalar registers: the address of an
// access through it plus a 32-bit lane offset is then the scalar-base form of the instruction
// (no 64-bit vector address arithmetic per access).
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return reinterpret_cast<T*>((static_cast<uint64_t>(hi) << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Streaming as a pull (Eq. Stream): f_i(x) = f_i*(x - c_i); from a solid x - c_i the
// halfway bounce-back returns f_opp(i)*(x).
template <int Q, bool WALLS, typename S, typename M>
__device__ __forceinline__ void pull(const S* __restrict__ src, const uint8_t* __restrict__ flags,
                                     const Geo& g, const Nb& b, int x, int y, int z, long long n,
                                     M (&ft)[Q], M (&dd)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        long long sn = shifted<Q, -1>(g, b, x, y, z, i);
        int di = i;
        if (WALLS && i != 0 && flags[sn]) {
            sn = n;
            di = Lat<Q>::opp[i];
        }
        ft[i] = ld<M>(src + (long long)di * g.N + sn);
        dd[i] = ld<M>(src + (long long)(Q + di) * g.N + sn);
    }
}

template <int Q, typename M>
__device__ __forceinline__ void moments(const M (&ft)[Q], const M (&dd)[Q], M& drho, M& dsum,
                                        M (&j)[3]) {
    drho = M(0);
    dsum = M(0);
    j[0] = j[1] = j[2] = M(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += ft[i];
        dsum += dd[i];
        if (Lat<Q>::cx[i]) j[0] += Lat<Q>::cx[i] * ft[i];
        if (Lat<Q>::cy[i]) j[1] += Lat<Q>::cy[i] * ft[i];
        if (Lat<Q>::cz[i]) j[2] += Lat<Q>::cz[i] * ft[i];
    }
}

// Site weight m(x) of the sink (site criterion of Sec. II.B) from the carried site data:
//   rule 0: the carried mask byte (||F_{n-1}|| > Gamma, set by the previous step);
//   rule 1: |rho^N_pre| < Gamma from the current pre-sink phase field (dsum / rho);
//   rule 2: the logistic function of (||F_{n-1}|| - Gamma) / kappa with the carried gradient
//           magnitude (double): a differentiable stand-in for the threshold.
template <typename M>
__device__ __forceinline__ M site_weight(const Phys<M>& P, const void* __restrict__ carry,
                                         long long n, M rho, M dsum) {
    if (P.site_rule == 2) {
        const M fprev = static_cast<M>(static_cast<const double*>(carry)[n]);
        return M(1) / (M(1) + exp(-(fprev - P.gamma) * P.inv_kappa));
    }
    if (P.site_rule == 0) return static_cast<const uint8_t*>(carry)[n] ? M(1) : M(0);
    return fabs(dsum / rho) < P.gamma ? M(1) : M(0);
}

// A node counts as a site when its weight exceeds 1/2 (exactly the sharp rules' sites).
template <typename M>
__device__ __forceinline__ bool is_site(M w) {
    return w > M(0.5);
}

// Carry of the next step: the mask byte, or ||F_n|| for the soft rule.
template <typename M>
__device__ __forceinline__ void carry_store(const Phys<M>& P, void* __restrict__ carry, long long n,
                                            M Fn) {
    if (P.site_rule == 2) static_cast<double*>(carry)[n] = static_cast<double>(Fn);
    else static_cast<uint8_t*>(carry)[n] = Fn > P.gamma ? 1 : 0;
}

// Node flux phi(x): the bound field (double next to FP64 populations, float otherwise) or the
// uniform value.
// Moment record of the split step (drho, j): FP64 next to FP64 populations, FP32 otherwise.
template <typename S>
using MomT = typename std::conditional<std::is_same<S, double>::value, double, float>::type;

template <typename S>
using PhiT = typename std::conditional<std::is_same<S, double>::value, double, float>::type;

// Post-collision record of the record form: stored like the populations (double, float or
// half), rebuilt in the arithmetic type RecE (float for a half record).
template <typename S>
using RecT = typename std::conditional<std::is_same<S, float>::value, float, S>::type;
template <typename R>
using RecE = typename std::conditional<std::is_same<R, _Float16>::value, float, R>::type;

template <typename S, typename M>
__device__ __forceinline__ M node_phi(const Phys<M>& P, const void* __restrict__ phi_field,
                                      long long n) {
    return phi_field ? static_cast<M>(static_cast<const PhiT<S>*>(phi_field)[n]) : P.phi;
}

// Sink s = m phi / Sbar of one node (Eqs. relation, exchange); w receives the weight m.
// dsum is pre-sink.
template <typename S, typename M>
__device__ __forceinline__ M site_sink(const Phys<M>& P, const void* __restrict__ carry,
                                       const void* __restrict__ phi_field, long long n, M rho,
                                       M dsum, M& w) {
    w = site_weight<M>(P, carry, n, rho, dsum);
    if (w == M(0)) return M(0);
    return w * (node_phi<S, M>(P, phi_field, n) * P.inv_sbar);
}
template <typename S, typename M>
__device__ __forceinline__ M site_sink(const Phys<M>& P, const void* __restrict__ carry,
                                       const void* __restrict__ phi_field, long long n, M rho,
                                       M dsum) {
    M w;
    return site_sink<S, M>(P, carry, phi_field, n, rho, dsum, w);
}

// The same decision from values fetched ahead of the populations: the carried mask byte and
// the node's flux (P.phi when no field is bound).
template <typename M>
__device__ __forceinline__ M site_sink_pre(const Phys<M>& P, uint8_t carry_byte, M phi, M rho,
                                           M dsum) {
    const bool m = P.site_rule == 0 ? carry_byte != 0 : fabs(dsum / rho) < P.gamma;
    return m ? phi * P.inv_sbar : M(0);
}

// Colour gradient by the compact isotropic stencil: F = (1/c_s^2) sum_i W_i rho^N(x+c_i) c_i
template <int Q, typename M, typename R>
__device__ __forceinline__ void gradient(const R* __restrict__ rhoN, const Geo& g, const Nb& b,
                                         int x, int y, int z, M (&F)[3]) {
    F[0] = F[1] = F[2] = M(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const M v = M(weight<Q>(i)) * static_cast<M>(rhoN[shifted<Q, 1>(g, b, x, y, z, i)]);
        if (Lat<Q>::cx[i]) F[0] += Lat<Q>::cx[i] * v;
        if (Lat<Q>::cy[i]) F[1] += Lat<Q>::cy[i] * v;
        if (Lat<Q>::cz[i]) F[2] += Lat<Q>::cz[i] * v;
    }
    F[0] *= M(3);
    F[1] *= M(3);
    F[2] *= M(3);
}

// BGK collision with harmonic tau and alpha-equilibrium (Eqs. collision, feq), perturbation
// (Eq. perturb) and recolouring (Eq. recolor), direction by direction.  Inputs are post-sink
// moments: drho = rho - rho_ref = sum_i ft_i, rhoN, u; F is the colour gradient.  The new
// populations depend on the old ones only through ft_i and these moments, so each direction
// is read with load(i) -> ft_i and written with store(i, ft_i*, dd_i*) at once, which keeps
// few values live.  With UNIT (both relaxation times 1, so 1/tau = 1 at every node) BGK
// relaxation returns the equilibrium and load() is not called.  Returns ||F||.
//
// Everything that depends on the direction only through its weight class (rest, axis,
// diagonal) is formed once per node:
//   feq_i = base_k + W_k rho (c_i.u) (3 + 4.5 c_i.u),   base_k = A_k drho + B_k dB - 1.5 W_k rho u.u
//   pert_i = (9/4)(sigma/tau) [W_k (F.c_i)^2 / |F| - C_k |F|]
//   dd_i = rho^N full_i + [2 beta (rho_r rho_b / rho) / (|F| |c_i|) t_k(abar)] (F.c_i)
// (cos(theta) and the perturbation taken as 0 where F.F <= kF2Cut; the optional fade of
// cos(theta) multiplies the bracket)
template <int Q, typename M, bool UNIT = false, typename Load, typename Store>
__device__ __forceinline__ M collide(Load&& load, M drho, M rho, M rhoN, const M (&u)[3],
                                     const M (&F)[3], const Phys<M>& P, Store&& store) {
    const M pr = M(0.5) * (M(1) + rhoN);  // rho_r / rho
    const M pb = M(0.5) * (M(1) - rhoN);  // rho_b / rho
    const M omega = pr * P.omega_r + pb * P.omega_b;
    const M abar = pr * P.alpha_r + pb * P.alpha_b;
    // rho t_i(abar) - rho_ref t_i(alpha_ref) = A_i drho + B_i (rho abar - rho_ref alpha_ref)
    const M dB = rho * (abar - P.alpha_ref) + drho * P.alpha_ref;
    const M uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const M F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    const M Fn = F2 > M(0) ? sqrt(F2) : M(0);  // carried to the next step's site decision
    const bool hg = F2 > M(kF2Cut);
    const M Fp = hg ? Fn : M(0);               // ||F|| in the perturbation
    const M invFn = hg ? M(1) / Fn : M(0);
    const M kp = M(2.25) * P.sigma * omega;                         // (9/4) sigma / tau
    const M sep = M(0.5) * P.beta * (M(1) - rhoN * rhoN) * rho;      // 2 beta rho_r rho_b / rho
    // cos(theta_i) = F.c_i / (|F| |c_i|) (Eq. recolor), times the optional fade
    const M cosw = invFn * recolor_fade(Fn, P.inv_fade);
    // per weight class k: 0 rest, 1 axis (|c| = 1), 2 diagonal (|c| = sqrt 2)
    constexpr int i1 = 1, i2 = Q == 9 ? 5 : 7;  // first direction of classes 1 and 2
    M base[3], wr[3], pf[3], kc[3], tref[3], gs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = k == 0 ? 0 : (k == 1 ? i1 : i2);
        const M A = M(restA<Q>(i)), B = M(restB<Q>(i)), W = M(weight<Q>(i));
        wr[k] = W * rho;
        base[k] = A * drho + B * dB - M(1.5) * wr[k] * uu;
        pf[k] = kp * W * invFn;
        kc[k] = kp * M(pertC<Q>(i)) * Fp;
        tref[k] = P.rho_ref * (A + B * P.alpha_ref);
        gs[k] = sep * cosw * M(inv_len<Q>(i)) * (A + B * abar);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int k = norm2<Q>(i);  // 0, 1, 2 = weight class
        const M cu = M(Lat<Q>::cx[i]) * u[0] + M(Lat<Q>::cy[i]) * u[1] + M(Lat<Q>::cz[i]) * u[2];
        const M Fc = M(Lat<Q>::cx[i]) * F[0] + M(Lat<Q>::cy[i]) * F[1] + M(Lat<Q>::cz[i]) * F[2];
        const M feq = base[k] + wr[k] * cu * (M(3) + M(4.5) * cu);
        M f1;
        if (UNIT) {
            f1 = feq;
        } else {
            const M fti = load(i);
            f1 = fti - omega * (fti - feq);
        }
        f1 += pf[k] * Fc * Fc - kc[k];
        const M full = f1 + tref[k];
        store(i, f1, rhoN * full + gs[k] * Fc);
    }
    return Fn;
}

// Post-collision record of a node at unit relaxation times (omega_r = omega_b = 1).  BGK
// relaxation then returns the equilibrium, so collide()'s populations of the node are, per
// weight class k and direction i of that class (h_k = W_k / W_1), with n = F / |F| the unit
// normal (0 where F.F <= kF2Cut):
//   ft_i* = b_k + h_k A (c_i.u)(1 + 1.5 c_i.u) + h_k P (n.c_i)^2
//   dd_i* = rho^N (ft_i* + t_ref,k) + g_k (n.c_i)
// with A = 3 W_1 rho, P = W_1 kp |F| (so that h_k P (n.c_i)^2 is the perturbation's
// W_k kp (F.c_i)^2 / |F|), b_k = base_k - kc_k and g_k = |F| gs_k (so that g_k (n.c_i) is the
// recolouring term gs_k (F.c_i)), where base_k, kc_k and gs_k are formed as in collide and
// t_ref,k = rho_ref t_k(alpha_ref).  The record is b_0, b_1, b_2, A, P, u, n, rho^N, g_1, g_2:
// 14 values instead of 2Q populations, each bounded by the state (a record holding F and
// kp / |F| instead would overflow half precision where F is tiny).  Returns ||F||.
constexpr int kRec = 14;
enum RecSlot { kB0 = 0, kB1, kB2, kA3, kP1, kUx, kUy, kUz, kNx, kNy, kNz, kRhoN, kG1, kG2 };

template <int Q, typename M>
__device__ __forceinline__ M record_values(M drho, M rho, M rhoN, const M (&u)[3],
                                          const M (&F)[3], const Phys<M>& P, M (&r)[kRec]) {
    const M pr = M(0.5) * (M(1) + rhoN);
    const M pb = M(0.5) * (M(1) - rhoN);
    const M omega = pr * P.omega_r + pb * P.omega_b;
    const M abar = pr * P.alpha_r + pb * P.alpha_b;
    const M dB = rho * (abar - P.alpha_ref) + drho * P.alpha_ref;
    const M uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const M F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    const M Fn = F2 > M(0) ? sqrt(F2) : M(0);
    const bool hg = F2 > M(kF2Cut);
    const M Fp = hg ? Fn : M(0);
    const M invFn = hg ? M(1) / Fn : M(0);
    const M kp = M(2.25) * P.sigma * omega;
    const M sep = M(0.5) * P.beta * (M(1) - rhoN * rhoN) * rho;
    // |F| cos(theta) / (F.c_i / |c_i|) = 1, times the optional fade, where F.F > kF2Cut
    const M fade = hg ? recolor_fade(Fn, P.inv_fade) : M(0);
    constexpr int i1 = 1, i2 = Q == 9 ? 5 : 7;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = k == 0 ? 0 : (k == 1 ? i1 : i2);
        const M A = M(restA<Q>(i)), B = M(restB<Q>(i)), W = M(weight<Q>(i));
        const M base = A * drho + B * dB - M(1.5) * (W * rho) * uu;
        r[kB0 + k] = base - kp * M(pertC<Q>(i)) * Fp;
        if (k > 0) r[kG1 + k - 1] = sep * fade * M(inv_len<Q>(i)) * (A + B * abar);
    }
    const M W1 = M(weight<Q>(i1));
    r[kA3] = M(3) * W1 * rho;
    r[kP1] = W1 * (kp * Fp);
    r[kUx] = u[0];
    r[kUy] = u[1];
    r[kUz] = u[2];
    r[kNx] = F[0] * invFn;
    r[kNy] = F[1] * invFn;
    r[kNz] = F[2] * invFn;
    r[kRhoN] = rhoN;
    return Fn;
}

// ft_i* and the colour difference of direction i (sgn = -1: of the opposite direction, for
// the bounce-back) from the record, in the record's arithmetic type E; L(slot) loads one
// record value of the source node as E.  dd_i* is returned in two parts, dd_i* = dp + rn
// t_ref,k: dp = rho^N ft_i* + g_k (n.c_i) and the source's rn = rho^N.  The caller adds rn
// t_ref,k in its arithmetic type: formed in E, the rounding of t_ref,k would repeat at every
// node and step and move red mass steadily between the bulks.  Only the values direction i
// needs are loaded.
template <int Q, typename E, typename Load>
__device__ __forceinline__ void record_dir(int i, E sgn, Load&& L, E& a, E& dp, E& rn) {
    const int k = norm2<Q>(i);
    rn = L(kRhoN);
    if (k == 0) {
        a = L(kB0);
        dp = rn * a;
        return;
    }
    // c.u and n.c from the non-zero components of c_i only (a sum started at zero costs an
    // add per direction: 0 + x is not x for x = -0)
    E cu = E(0), nc = E(0);
    bool any = false;
    auto term = [&](int c, int su, int sn) {
        if (c == 0) return;
        const E tu = c > 0 ? L(su) : -L(su), tn = c > 0 ? L(sn) : -L(sn);
        cu = any ? cu + tu : tu;
        nc = any ? nc + tn : tn;
        any = true;
    };
    term(Lat<Q>::cx[i], kUx, kNx);
    term(Lat<Q>::cy[i], kUy, kNy);
    term(Lat<Q>::cz[i], kUz, kNz);
    cu *= sgn;
    nc *= sgn;
    constexpr double h = weight<Q>(Q == 9 ? 5 : 7) / weight<Q>(1);  // W_2 / W_1
    const E hk = k == 1 ? E(1) : E(h);
    a = L(k == 1 ? kB1 : kB2) + L(kA3) * (cu * (hk + E(1.5) * hk * cu));
    a += (hk * L(kP1)) * (nc * nc);
    dp = rn * a + L(k == 1 ? kG1 : kG2) * nc;
}

// The record slots record_dir reads for direction i (bit sl set), for callers that load them
// ahead of the call.
template <int Q>
__host__ __device__ constexpr uint32_t dir_slots(int i) {
    const int k = norm2<Q>(i);
    if (k == 0) return (1u << kRhoN) | (1u << kB0);
    uint32_t m = (1u << kRhoN) | (1u << (k == 1 ? kB1 : kB2)) | (1u << kA3) | (1u << kP1) |
                 (1u << (k == 1 ? kG1 : kG2));
    if (Lat<Q>::cx[i]) m |= (1u << kUx) | (1u << kNx);
    if (Lat<Q>::cy[i]) m |= (1u << kUy) | (1u << kNy);
    if (Lat<Q>::cz[i]) m |= (1u << kUz) | (1u << kNz);
    return m;
}

// Neutral wetting: a solid node takes the W-weighted mean of rho^N over its fluid neighbours.
template <int Q, typename R>
__global__ __launch_bounds__(kTPBX) void k_wet(const uint8_t* __restrict__ flags,
                                               R* __restrict__ rhoN, Geo g) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (!flags[n]) return;
    const Nb b = wrap(g, x, y, z);
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const long long m = shifted<Q, 1>(g, b, x, y, z, i);
        if (flags[m]) continue;
        num += weight<Q>(i) * static_cast<double>(rhoN[m]);
        den += weight<Q>(i);
    }
    rhoN[n] = static_cast<R>(den > 0.0 ? num / den : 0.0);
}

// ---------------------------------------------------------------- block reductions (FP64)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum (or max for the flagged entries) of NV values over the block, fixed order; result in
// out[] of thread 0.  tid = linear thread index, nthreads = block size (multiple of 64).
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const bool (&is_max)[NV], int tid,
                                             int nthreads, double (&out)[NV]) {
    __shared__ double sh[NV][16];
    const int lane = tid & 63, wave = tid >> 6, nw = nthreads >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double r = is_max[k] ? wave_max(v[k]) : wave_sum(v[k]);
        if (lane == 0) sh[k][wave] = r;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = sh[k][0];
            for (int w = 1; w < nw; ++w) s = is_max[k] ? fmax(s, sh[k][w]) : s + sh[k][w];
            out[k] = s;
        }
    }
}

}  // namespace cge
