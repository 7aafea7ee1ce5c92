// Single-pass fused step for D3Q19 on periodic domains (no solid nodes).
//
// The colour gradient at a node needs the post-sink phase field rho^N of its 18 neighbours,
// which exists only after those neighbours have pulled their populations.  Instead of
// writing rho^N to memory and reading the populations a second time (two-pass form), each
// workgroup owns a TX x TY tile of the x-y plane and marches along a chunk of z:
//   for plane p = z0-1 .. z1:
//     pull the populations of the tile's nodes at plane p, apply the sink, reduce them to
//     what the collision needs (colour-blind populations and FP64 moments) and keep that in
//     registers; compute rho^N of the tile and of its one-node ring (the ring nodes' pulls
//     read data that neighbouring tiles read as their own, mostly from L2);
//     put rho^N(p) into a three-plane LDS ring;
//     finish plane p-1: gradient from LDS planes p-2, p-1, p, collision, perturbation,
//     recolouring, store, next site mask.
// Every population is read once from HBM and written once; the extra reads are the ring
// and the two end planes of each z-chunk.
//
// Memory access goes through buffer resources: each thread computes the byte offsets of its
// nine (x, y) neighbours once (periodic wrap included); the population slot and the z plane
// enter as a scalar offset, so a load costs no vector address arithmetic.
//
// The site mask is double-buffered (read cin, write cout): a ring node's mask is read by the
// neighbouring tile while its owner writes the next one.
//
// With both relaxation times equal to 1, BGK relaxation returns the equilibrium, and the
// pulled populations enter the collision only through their moments: the plane waiting to be
// finished is then held as six FP64 moments per node instead of 19 populations.
//
// Tile -> workgroup mapping: consecutive workgroups go to different XCDs, so workgroup b
// takes tile (b % 8) * (nb / 8) + b / 8 when nb % 8 == 0: each XCD gets a contiguous range
// of tiles (x fastest, then y, then z-chunk), and tiles that share ring data share an L2.
#include "internal.hpp"
#include "node.hpp"

namespace cge {

constexpr int kFTX = 64;  // tile width in x: one wavefront per row
constexpr int kFTY = 4;   // tile rows per workgroup

struct FusedShape {
    int ntx, nty, nzc, zlen;
    long long nb;
};

static FusedShape fused_shape(const Geo& g) {
    FusedShape s;
    s.ntx = (g.nx + kFTX - 1) / kFTX;
    s.nty = (g.ny + kFTY - 1) / kFTY;
    const long long tiles = (long long)s.ntx * s.nty;
    // enough workgroups to fill the chip several times over, z-chunks of >= 16 planes
    long long want = (2048 + tiles - 1) / tiles;
    const long long maxc = (g.nz + 15) / 16;
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    s.zlen = (int)((g.nz + want - 1) / want);
    s.nzc = (g.nz + s.zlen - 1) / s.zlen;
    s.nb = tiles * s.nzc;
    return s;
}

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Loads and stores of one storage element through a buffer resource at byte offset
// voff (per lane) + soff (uniform).
template <typename S>
struct Buf;
template <>
struct Buf<float> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
    }
    static __device__ __forceinline__ void st(float x, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                              uint32_t s) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, v, s, 0);
    }
};
template <>
struct Buf<double> {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
    }
    static __device__ __forceinline__ void st(double x, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                              uint32_t s) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, v, s, 0);
    }
};
template <>
struct Buf<_Float16> {
    static __device__ __forceinline__ _Float16 ld(__amdgpu_buffer_rsrc_t r, uint32_t v,
                                                  uint32_t s) {
        return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
    }
    static __device__ __forceinline__ void st(_Float16 x, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                              uint32_t s) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, x), r, v, s, 0);
    }
};

// Byte offsets within one z plane of the nine nodes (x + dx, y + dy), dx, dy in {-1, 0, 1},
// periodic: o[1 + dy][1 + dx].
template <typename S>
struct Plane9 {
    uint32_t o[3][3];
};

template <typename S>
__device__ __forceinline__ Plane9<S> plane9(const Geo& g, int x, int y) {
    Plane9<S> p;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
        const uint32_t row = (uint32_t)wrap1(y - 1 + dy, g.ny) * (uint32_t)g.nx;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
            p.o[dy][dx] = (row + (uint32_t)wrap1(x - 1 + dx, g.nx)) * (uint32_t)sizeof(S);
    }
    return p;
}

// What the finishing half of the step needs of a pulled node: the colour-blind populations
// ft_i (the colour differences enter only through their sum) and the post-sink moments.
// With unit relaxation times the collision needs the moments only.
template <int Q, typename S, typename M, bool UNIT>
struct Pulled {
    S ft[UNIT ? 1 : Q];
    M drho, dsum, j[3], s;  // dsum is post-sink; s is the sink applied
};

// Pull (Eq. Stream) of the node whose plane offsets are `pl`, at plane z: direction i comes
// from (x, y, z) - c_i.  zoff[1 + d] is the byte offset of plane z + d (wrapped).  Returns
// the post-sink rho^N (rounded to the storage precision, as the other step forms store it);
// with FULL, also fills the reduced node for the collision.
template <int Q, typename S, typename M, bool FULL, bool UNIT>
__device__ __forceinline__ M pull_node(__amdgpu_buffer_rsrc_t rft, __amdgpu_buffer_rsrc_t rdd,
                                       const Plane9<S>& pl, const uint32_t (&zoff)[3],
                                       uint32_t slot_bytes, const Phys<M>& P,
                                       const uint8_t* __restrict__ cin,
                                       const void* __restrict__ phi_field, uint32_t n,
                                       Pulled<Q, S, M, UNIT>& pn) {
    // the site byte and flux do not depend on the populations: fetch them first
    const uint8_t cb = cin[n];
    const M phi = phi_field ? static_cast<M>(static_cast<const PhiT<S>*>(phi_field)[n]) : P.phi;
    M drho = M(0), dsum = M(0), j[3] = {M(0), M(0), M(0)};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t vo = pl.o[1 - Lat<Q>::cy[i]][1 - Lat<Q>::cx[i]];
        const uint32_t so = (uint32_t)i * slot_bytes + zoff[1 - Lat<Q>::cz[i]];
        const S a = Buf<S>::ld(rft, vo, so);
        if (FULL && !UNIT) pn.ft[i] = a;
        const M am = static_cast<M>(a);
        drho += am;
        dsum += static_cast<M>(Buf<S>::ld(rdd, vo, so));
        if (FULL) {
            if (Lat<Q>::cx[i]) j[0] += Lat<Q>::cx[i] * am;
            if (Lat<Q>::cy[i]) j[1] += Lat<Q>::cy[i] * am;
            if (Lat<Q>::cz[i]) j[2] += Lat<Q>::cz[i] * am;
        }
    }
    const M rho = P.rho_ref + drho;
    const M s = site_sink_pre<M>(P, cb, phi, rho, dsum);
    const M dpost = dsum - M(2) * s;
    if (FULL) {
        pn.drho = drho;
        pn.dsum = dpost;
        pn.j[0] = j[0];
        pn.j[1] = j[1];
        pn.j[2] = j[2];
        pn.s = s;
    }
    // rho^N as a stored field holds it: float next to FP32 or FP16 populations
    return static_cast<M>(static_cast<MomT<S>>(dpost / rho));
}

template <int Q, typename S, typename M, bool UNIT>
__global__ __launch_bounds__(kFTX* kFTY) void k_fused(
    const S* __restrict__ src, S* __restrict__ dst, const uint8_t* __restrict__ cin,
    uint8_t* __restrict__ cout, const void* __restrict__ phi_field, double* __restrict__ acc_sink,
    long long* __restrict__ acc_sites, Geo g, Phys<M> P, uint64_t salt, FusedShape fs) {
    static_assert(Q == 19, "the fused step is written for D3Q19");
    __shared__ M rn[3][kFTY + 2][kFTX + 2];

    const int tid = threadIdx.x;
    const int lx = tid % kFTX, ly = tid / kFTX;
    long long b = blockIdx.x;
    if (fs.nb % 8 == 0) b = (b % 8) * (fs.nb / 8) + b / 8;
    const int tx = (int)(b % fs.ntx);
    const int ty = (int)((b / fs.ntx) % fs.nty);
    const int zc = (int)(b / ((long long)fs.ntx * fs.nty));
    const int x0 = tx * kFTX, y0 = ty * kFTY;
    const int w = min(kFTX, g.nx - x0), h = min(kFTY, g.ny - y0);
    const int z0 = zc * fs.zlen, z1 = min(z0 + fs.zlen, g.nz);
    const bool own = lx < w && ly < h;
    const int x = own ? x0 + lx : x0, y = own ? y0 + ly : y0;

    // Ring nodes in order: top row, bottom row, left column, right column.  Each wave takes a
    // contiguous quarter of the list (rows stay coalesced, waves stay balanced).
    int rx = 0, ry = 0;
    bool ring;
    {
        const int row = w + 2, nring = 2 * row + 2 * h;
        const int per = (nring + kFTY - 1) / kFTY;  // kFTY waves of 64 lanes each
        const int lane = tid % 64, wave = tid / 64;
        int t = wave * per + lane;
        ring = lane < per && t < nring;
        if (t < row) {
            rx = t - 1;
            ry = -1;
        } else if ((t -= row) < row) {
            rx = t - 1;
            ry = h;
        } else if ((t -= row) < h) {
            rx = -1;
            ry = t;
        } else {
            t -= h;
            rx = w;
            ry = t;
        }
    }
    const int gx = wrap1(x0 + rx, g.nx), gy = wrap1(y0 + ry, g.ny);

    const uint32_t E = sizeof(S);
    const uint32_t slot_bytes = (uint32_t)g.N * E;
    const uint32_t plane_bytes = (uint32_t)g.nx * (uint32_t)g.ny * E;
    const int range = (int)((uint32_t)Q * slot_bytes);
    const long long QN = (long long)Q * g.N;
    const __amdgpu_buffer_rsrc_t sft =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(src), 0, range, 0x00020000);
    const __amdgpu_buffer_rsrc_t sdd =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(src + QN), 0, range, 0x00020000);
    const __amdgpu_buffer_rsrc_t dft = __builtin_amdgcn_make_buffer_rsrc(dst, 0, range, 0x00020000);
    const __amdgpu_buffer_rsrc_t ddd =
        __builtin_amdgcn_make_buffer_rsrc(dst + QN, 0, range, 0x00020000);

    const Plane9<S> po = plane9<S>(g, x, y);    // own node's neighbourhood
    const Plane9<S> pr = plane9<S>(g, gx, gy);  // ring node's neighbourhood
    const uint32_t own_xy = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y;
    const uint32_t ring_xy = (uint32_t)gx + (uint32_t)g.nx * (uint32_t)gy;
    const uint32_t nplane = (uint32_t)g.nx * (uint32_t)g.ny;

    Pulled<Q, S, M, UNIT> cur, nxt;  // plane waiting to be finished, plane being pulled
    cur.s = M(0);
    double acc_s = 0.0, acc_n = 0.0;

    for (int p = z0 - 1; p <= z1; ++p) {
        const int pz = wrap1(p, g.nz);
        const uint32_t zoff[3] = {(uint32_t)wrap1(pz - 1, g.nz) * plane_bytes,
                                  (uint32_t)pz * plane_bytes,
                                  (uint32_t)wrap1(pz + 1, g.nz) * plane_bytes};
        const int slot = (p - z0 + 1) % 3;
        M r_ring = M(0), r_own = M(0);
        if (ring)
            r_ring = pull_node<Q, S, M, false, UNIT>(sft, sdd, pr, zoff, slot_bytes, P, cin,
                                                     phi_field, ring_xy + (uint32_t)pz * nplane, nxt);
        if (own)
            r_own = pull_node<Q, S, M, true, UNIT>(sft, sdd, po, zoff, slot_bytes, P, cin,
                                                   phi_field, own_xy + (uint32_t)pz * nplane, nxt);
        __syncthreads();  // every thread is done reading the slot about to be overwritten
        if (own) rn[slot][ly + 1][lx + 1] = r_own;
        if (ring) rn[slot][ry + 1][rx + 1] = r_ring;
        __syncthreads();

        const int pc = p - 1;  // plane to finish
        if (pc >= z0 && own) {
            const uint32_t n = own_xy + (uint32_t)pc * nplane;
            if (cur.s != M(0)) {
                acc_s += static_cast<double>(cur.s);
                acc_n += 1.0;
            }
            const M rho = P.rho_ref + cur.drho;
            const M inv_rho = M(1) / rho;
            const M u[3] = {cur.j[0] * inv_rho, cur.j[1] * inv_rho, cur.j[2] * inv_rho};
            const M rN = static_cast<M>(static_cast<MomT<S>>(cur.dsum / rho));  // as in the ring
            // gradient from the LDS ring: planes pc-1, pc, pc+1 are slots of p-2, p-1, p
            const int sl[3] = {(p - z0 + 2) % 3, (p - z0) % 3, slot};  // cz = -1, 0, +1
            M F[3] = {M(0), M(0), M(0)};
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int cx = Lat<Q>::cx[i], cy = Lat<Q>::cy[i], cz = Lat<Q>::cz[i];
                const M v = M(weight<Q>(i)) * rn[sl[cz + 1]][ly + 1 + cy][lx + 1 + cx];
                if (cx) F[0] += cx * v;
                if (cy) F[1] += cy * v;
                if (cz) F[2] += cz * v;
            }
            F[0] *= M(3);
            F[1] *= M(3);
            F[2] *= M(3);
            const uint32_t vo = po.o[1][1];
            const uint32_t zo = (uint32_t)pc * plane_bytes;
            const M Fn = collide<Q, M, UNIT>(
                [&](int i) { return static_cast<M>(cur.ft[UNIT ? 0 : i]); }, cur.drho, rho, rN, u,
                F, P,
                [&](int i, M a, M d) {
                    const uint64_t key = salt + (uint64_t)(2 * i) * (uint64_t)g.N + (uint64_t)n;
                    const uint32_t so = (uint32_t)i * slot_bytes + zo;
                    Buf<S>::st(enc<S, M>(a, key), dft, vo, so);
                    Buf<S>::st(enc<S, M>(d, key + (uint64_t)g.N), ddd, vo, so);
                });
            cout[n] = Fn > P.gamma ? 1 : 0;
        }
        if (own && p < z1) cur = nxt;
    }

    double v[2] = {acc_s, acc_n};
    const bool is_max[2] = {false, false};
    double out[2];
    block_reduce<2>(v, is_max, tid, kFTX * kFTY, out);
    if (tid == 0) {
        acc_sink[b] += out[0];
        acc_sites[b] += static_cast<long long>(out[1]);
    }
}

__global__ __launch_bounds__(256) void k_copy_bytes(const uint8_t* __restrict__ src,
                                                    uint8_t* __restrict__ dst, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// The Q slots of one component must fit a buffer resource's signed 32-bit byte range.
bool fused_supported(const cge_ctx* c) {
    const long long elem = c->p.precision == CGE_FP64 ? 8 : (c->p.precision == CGE_FP32S ? 4 : 2);
    return c->Q == 19 && c->flags == nullptr && c->p.site_rule != CGE_SITE_SOFT &&
           19ll * c->g.N * elem < (1ll << 31);
}

long long fused_blocks(const cge_ctx* c) { return fused_shape(c->g).nb; }

template <int Q, typename S, typename M, bool WALLS>
static cge_status fused_impl(cge_ctx* c, long long nsteps) {
    if constexpr (Q != 19 || WALLS) {
        return fail(c, CGE_EUNSUPPORTED, "fused step needs D3Q19 without solid nodes");
    } else {
        const Phys<M> P = phys<M>(c);
        const FusedShape fs = fused_shape(c->g);
        if (fs.nb > c->acc_len) return fail(c, CGE_ESTATE, "accumulator too small");
        const uint64_t seedmix = mix64(c->p.seed);
        const bool unit = c->p.tau[0] == 1.0 && c->p.tau[1] == 1.0;
        uint8_t* mask[2] = {c->carry, c->carry2};
        int m = 0;
        for (long long t = 0; t < nsteps; ++t) {
            const S* src = static_cast<const S*>(c->pop[c->cur]);
            S* dst = static_cast<S*>(c->pop[1 - c->cur]);
            const uint64_t salt = mix64(seedmix + (uint64_t)c->step) * 0x100000001B3ull;
            timing_begin(c, "fused step");
            if (unit)
                hipLaunchKernelGGL((k_fused<Q, S, M, true>), dim3((unsigned)fs.nb),
                                   dim3(kFTX * kFTY), 0, c->stream, src, dst, mask[m],
                                   mask[1 - m], c->phi_field, c->acc_sink, c->acc_sites, c->g, P,
                                   salt, fs);
            else
                hipLaunchKernelGGL((k_fused<Q, S, M, false>), dim3((unsigned)fs.nb),
                                   dim3(kFTX * kFTY), 0, c->stream, src, dst, mask[m],
                                   mask[1 - m], c->phi_field, c->acc_sink, c->acc_sites, c->g, P,
                                   salt, fs);
            timing_pass(c, "k_fused");
            timing_end(c);
            if (cge_status s = check(c, hipGetLastError(), "fused step launch")) return s;
            m = 1 - m;
            c->cur = 1 - c->cur;
            c->step += 1;
        }
        if (m == 1) {  // the current mask is in the library's buffer: hand it back
            hipLaunchKernelGGL(k_copy_bytes, dim3((unsigned)((c->g.N + 255) / 256)), dim3(256), 0,
                               c->stream, c->carry2, c->carry, c->g.N);
            if (cge_status s = check(c, hipGetLastError(), "mask copy launch")) return s;
        }
        return CGE_OK;
    }
}

cge_status fused_steps(cge_ctx* c, long long nsteps) { CGE_DISPATCH(c, fused_impl, c, nsteps); }

}  // namespace cge
