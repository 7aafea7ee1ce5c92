// Single-pass fused step for D3Q19: periodic domains, and solid walls that fill whole z-planes.
//
// The colour gradient at a node needs the post-sink phase field rho^N of its 18 neighbours,
// which exists only after those neighbours have pulled their populations.  Instead of
// writing rho^N to memory and reading the populations a second time (two-pass form), each
// workgroup owns a 64 x kFTY tile of the x-y plane and marches along a chunk of z:
//   for plane p:
//     pull the populations of the tile's nodes at plane p, apply the sink, reduce them to
//     what the collision needs (colour-blind populations and FP64 moments) and keep that in
//     registers; compute rho^N of the tile and of its one-node ring (the ring nodes' pulls
//     read data that neighbouring tiles read as their own, mostly from L2);
//     put rho^N(p) into a three-plane LDS ring;
//     finish plane p-1: gradient from LDS planes p-2, p-1, p, collision, perturbation,
//     recolouring, store, next site mask.
// Every population is read once from HBM and written once; the extra reads are the ring
// and the end planes of each z-chunk.
//
// Walls (halfway bounce-back, neutral wetting) are served when every z-plane is wholly solid
// or wholly fluid and no solid plane has fluid on both sides: the floors, lids and slabs of
// the wall-bounded workloads.  A pulled direction then bounces back exactly when its source
// plane is solid, a test on the plane alone.  A solid plane's rho^N is the wetting value of
// its nodes, the W-weighted mean over their fluid neighbours (as k_wet forms it), all of
// which lie in its one fluid neighbour plane: a lid (fluid below) takes it from the plane
// pulled before it, a floor (fluid above) from the plane pulled after it, one plane before
// the floor is needed as a neighbour.  The wetting values of the ring's nodes need rho^N one
// node further out, so a fluid plane next to a wall also pulls a second ring (rho^N only).
//
// Memory access goes through buffer resources, one per component spanning its Q slots (an
// unsigned 32-bit byte range, up to 4 GiB): each thread computes the byte offsets of its nine
// (x, y) neighbours once (periodic wrap included); the population slot and the z plane enter
// as a scalar offset, so a load costs no vector address arithmetic.
//
// The site mask is double-buffered (read cin, write cout): a ring node's mask is read by the
// neighbouring tile while its owner writes the next one.
//
// With both relaxation times equal to 1, BGK relaxation returns the equilibrium, and the
// pulled populations enter the collision only through their moments: the plane waiting to be
// finished is then held as six FP64 moments per node instead of 19 populations.
//
// Tile -> workgroup mapping: workgroups are dealt to the XCDs round-robin by id, so XCD k
// takes a contiguous run of tiles (x fastest, then y, then z-chunk), and tiles that share
// ring data share an L2.
#include "internal.hpp"
#include "node.hpp"

namespace cge {

constexpr int kFTX = 64;  // tile width in x: one wavefront per row
// Tile rows per workgroup.  At general relaxation times a thread holds one pulled node's
// moments and the 38 loads of a pull in flight, and the FP64 collision: 167 registers at FP32
// storage with plane walls, three waves per SIMD (three workgroups per CU by their LDS).  The
// 384 x 384 x 192 sessile drop runs in 2.52 ms per step.  Six rows, whose halo ring adds
// 38 % instead of 55 % to the pulls, ran in 3.10 ms (two workgroups per CU by their LDS) and
// eight rows slower still; issuing a plane's own pull one plane ahead of the previous plane's
// collision ran in 2.77 ms (the loads held across the collision take two waves per SIMD).
constexpr int kFTY = 4;

// Kinds of the z-planes under plane walls.
enum : uint8_t {
    kPlaneSolid = 1,       // the plane is solid
    kPlaneFluidBelow = 2,  // a solid plane whose plane z - 1 is fluid (a lid)
    kPlaneFluidAbove = 4,  // a solid plane whose plane z + 1 is fluid (a floor)
    kPlaneNearWall = 8,    // a fluid plane next to a solid one
};

struct FusedShape {
    int ntx, nty, nzc, zlen;
    long long nb;
};

// zchunk > 0: planes per z-chunk (cge_set_zchunk), else chosen here
static FusedShape fused_shape(const Geo& g, int zchunk) {
    FusedShape s;
    s.ntx = (g.nx + kFTX - 1) / kFTX;
    s.nty = (g.ny + kFTY - 1) / kFTY;
    const long long tiles = (long long)s.ntx * s.nty;
    // enough workgroups to fill the chip several times over, z-chunks of >= 16 planes
    long long want = (2048 + tiles - 1) / tiles;
    const long long maxc = (g.nz + 15) / 16;
    if (want > maxc) want = maxc;
    if (want < 1) want = 1;
    s.zlen = zchunk > 0 ? (zchunk < g.nz ? zchunk : g.nz) : (int)((g.nz + want - 1) / want);
    s.nzc = (g.nz + s.zlen - 1) / s.zlen;
    s.nb = tiles * s.nzc;
    return s;
}

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int wrapf(int v, int n) { return ((v % n) + n) % n; }

// Loads and stores of one storage element through a buffer resource at byte offset
// voff (per lane) + soff (uniform).  Stores of populations too large to stay in the
// last-level cache (Geo::nt kNtPop) are non-temporal (cache policy bit 1, as
// __builtin_nontemporal_store gives the other step forms): they are read only by the next
// step, long after a plane's lines would have left L2, and left to allocate normally they
// evict the ring rows that neighbouring tiles are about to re-read (the 384 x 384 x 192
// sessile drop: 2.54 -> 2.42 ms per step).
constexpr int kStoreNT = 2;
template <typename S>
struct Buf;
template <>
struct Buf<float> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
    }
    static __device__ __forceinline__ void st(float x, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                              uint32_t s, bool nt) {
        if (nt)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, v, s, kStoreNT);
        else
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
                                              uint32_t s, bool nt) {
        if (nt)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, v, s, kStoreNT);
        else
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
                                              uint32_t s, bool nt) {
        if (nt)
            __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, x), r, v, s, kStoreNT);
        else
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

// What the finishing half of the step needs of a pulled node: the post-sink moments (in
// registers) and, unless both relaxation times are 1, the colour-blind populations ft_i (the
// colour differences enter only through their sum), which the pull leaves in the thread's
// own LDS slots (ftl below).
template <int Q, typename S, typename M, bool UNIT>
struct Pulled {
    M drho, dsum, j[3], s;  // dsum is post-sink; s is the sink applied
};

// Pull (Eq. Stream) of the node whose plane offsets are `pl`, at plane z: direction i comes
// from (x, y, z) - c_i, or, where the plane of the source is solid (bit 1 + c_z of bb, plane
// walls), from the node itself in the opposite direction (halfway bounce-back).  zoff[1 + d]
// is the byte offset of plane z + d (wrapped).  Returns the post-sink rho^N (rounded to the
// storage precision, as the other step forms store it); with FULL, also fills the reduced
// node for the collision.
template <int Q, typename S, typename M, bool FULL, bool UNIT, bool PW>
__device__ __forceinline__ M pull_node(__amdgpu_buffer_rsrc_t rft, __amdgpu_buffer_rsrc_t rdd,
                                       const Plane9<S>& pl, const uint32_t (&zoff)[3],
                                       uint32_t slot_bytes, uint32_t bb, const Phys<M>& P,
                                       const uint8_t* __restrict__ cin,
                                       __amdgpu_buffer_rsrc_t rphi, bool has_phi, uint32_t n,
                                       Pulled<Q, S, M, UNIT>& pn, S* __restrict__ ft_out,
                                       int ft_stride) {
    // The site byte and flux do not depend on the populations: fetch them first, and convert
    // the flux only after the population loads are issued, so no wait for it comes first (a
    // wait for one load is a wait for every earlier load and store of the wave).  The flux
    // goes through a buffer resource with no records when no field is bound (the load then
    // returns 0 and touches no memory), so the load needs no branch and stays up front.
    const uint8_t cb = cin[n];
    const PhiT<S> phi_raw = Buf<PhiT<S>>::ld(rphi, n * (uint32_t)sizeof(PhiT<S>), 0);
    M drho = M(0), dsum = M(0), j[3] = {M(0), M(0), M(0)};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        uint32_t vo = pl.o[1 - Lat<Q>::cy[i]][1 - Lat<Q>::cx[i]];
        uint32_t so = (uint32_t)i * slot_bytes + zoff[1 - Lat<Q>::cz[i]];
        if (PW && i != 0 && ((bb >> (1 + Lat<Q>::cz[i])) & 1u)) {
            vo = pl.o[1][1];
            so = (uint32_t)Lat<Q>::opp[i] * slot_bytes + zoff[1];
        }
        const S a = Buf<S>::ld(rft, vo, so);
        if (FULL && !UNIT) ft_out[i * ft_stride] = a;
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
    const M phi = has_phi ? static_cast<M>(phi_raw) : P.phi;
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

// Position t of the ring at distance d around a w x h tile (tile coordinates): its top row,
// bottom row, left column, right column.
__device__ __forceinline__ void ring_at(int t, int d, int w, int h, int& rx, int& ry) {
    const int row = w + 2 * d, col = h + 2 * d - 2;
    if (t < row) {
        rx = t - d;
        ry = -d;
    } else if ((t -= row) < row) {
        rx = t - d;
        ry = h - 1 + d;
    } else if ((t -= row) < col) {
        rx = -d;
        ry = t - d + 1;
    } else {
        t -= col;
        rx = w - 1 + d;
        ry = t - d + 1;
    }
}

// PW: the solid flags are plane walls, described per plane by pkind.
template <int Q, typename S, typename M, bool UNIT, bool PW, bool NTS>
__global__ __launch_bounds__(kFTX* kFTY) void k_fused(
    const S* __restrict__ src, S* __restrict__ dst, const uint8_t* __restrict__ cin,
    uint8_t* __restrict__ cout, const void* __restrict__ phi_field,
    const uint8_t* __restrict__ pkind, double* __restrict__ acc_sink,
    long long* __restrict__ acc_sites, Geo g, Phys<M> P, uint64_t salt, FusedShape fs) {
    static_assert(Q == 19, "the fused step is written for D3Q19");
    constexpr int R = PW ? 2 : 1;  // rings of rho^N held around the tile
    constexpr int NW = kFTY;       // waves per workgroup
    __shared__ M rn[3][kFTY + 2 * R][kFTX + 2 * R];
    // the colour-blind populations of the pulled own nodes, by plane parity: thread t keeps
    // direction i of its node at ftl[p & 1][i][t] (written by its pull of plane p, read by its
    // finish of plane p one plane later; no other thread touches the slot)
    __shared__ S ftl[UNIT ? 1 : 2][UNIT ? 1 : Q][kFTX * kFTY];
    // plane kinds of the chunk (plane walls): fused_kinds_bytes(zlen) bytes of dynamic LDS
    extern __shared__ uint8_t kinds[];

    const int tid = threadIdx.x;
    const int lx = tid % kFTX, ly = tid / kFTX;
    constexpr bool nt = NTS;
    const unsigned nb = gridDim.x, bid = blockIdx.x;
    const unsigned xq = nb / kXcds, xrem = nb % kXcds, xk = bid % kXcds;
    const long long b = (long long)(xk * xq + (xk < xrem ? xk : xrem) + bid / kXcds);
    const int tx = (int)(b % fs.ntx);
    const int ty = (int)((b / fs.ntx) % fs.nty);
    const int zc = (int)(b / ((long long)fs.ntx * fs.nty));
    const int x0 = tx * kFTX, y0 = ty * kFTY;
    const int w = min(kFTX, g.nx - x0), h = min(kFTY, g.ny - y0);
    const int z0 = zc * fs.zlen, z1 = min(z0 + fs.zlen, g.nz);
    const bool own = lx < w && ly < h;
    const int x = own ? x0 + lx : x0, y = own ? y0 + ly : y0;

    // Ring nodes: each wave takes a contiguous share of each ring's list (rows stay
    // coalesced, waves stay balanced).
    const int lane = tid % 64, wave = tid / 64;
    int rx = 0, ry = 0, r2x = 0, r2y = 0;
    bool ring, ring2 = false;
    {
        const int n1 = 2 * w + 2 * h + 4, per = (n1 + NW - 1) / NW;
        const int t = wave * per + lane;
        ring = lane < per && t < n1;
        if (ring) ring_at(t, 1, w, h, rx, ry);
        if (PW) {
            const int n2 = 2 * w + 2 * h + 12, per2 = (n2 + NW - 1) / NW;
            const int t2 = wave * per2 + lane;
            ring2 = lane < per2 && t2 < n2;
            if (ring2) ring_at(t2, 2, w, h, r2x, r2y);
        }
    }
    const int gx = wrapf(x0 + rx, g.nx), gy = wrapf(y0 + ry, g.ny);

    const uint32_t E = sizeof(S);
    const uint32_t slot_bytes = (uint32_t)g.N * E;
    const uint32_t plane_bytes = (uint32_t)g.nx * (uint32_t)g.ny * E;
    // the record count of a raw buffer is an unsigned 32-bit byte count (fused_supported
    // keeps Q slots below 2^32 bytes)
    const int range = (int)((uint32_t)Q * slot_bytes);
    const long long QN = (long long)Q * g.N;
    const __amdgpu_buffer_rsrc_t sft =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(src), 0, range, 0x00020000);
    const __amdgpu_buffer_rsrc_t sdd =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(src + QN), 0, range, 0x00020000);
    const __amdgpu_buffer_rsrc_t dft = __builtin_amdgcn_make_buffer_rsrc(dst, 0, range, 0x00020000);
    const __amdgpu_buffer_rsrc_t ddd =
        __builtin_amdgcn_make_buffer_rsrc(dst + QN, 0, range, 0x00020000);
    const bool has_phi = phi_field != nullptr;
    const __amdgpu_buffer_rsrc_t rphi = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void*>(phi_field), 0, has_phi ? (int)((uint32_t)g.N * (uint32_t)sizeof(PhiT<S>)) : 0,
        0x00020000);

    const Plane9<S> po = plane9<S>(g, x, y);    // own node's neighbourhood
    const Plane9<S> pr = plane9<S>(g, gx, gy);  // ring node's neighbourhood
    const uint32_t own_xy = (uint32_t)x + (uint32_t)g.nx * (uint32_t)y;
    const uint32_t ring_xy = (uint32_t)gx + (uint32_t)g.nx * (uint32_t)gy;
    const uint32_t nplane = (uint32_t)g.nx * (uint32_t)g.ny;

    // Kinds of the planes z0 - 3 .. z1 + 1 (every plane the chunk asks about), copied once into
    // LDS: read from global memory in the loop, each would cost a wait for all of the wave's
    // loads and stores in flight.
    const int z0k = z0 - 3;
    if (PW) {
        for (int t = tid; t < z1 - z0 + 5; t += kFTX * kFTY) kinds[t] = pkind[wrapf(z0k + t, g.nz)];
        __syncthreads();
    }
    auto kind = [&](int zp) -> uint32_t {
        return PW ? (uint32_t)__builtin_amdgcn_readfirstlane(kinds[zp - z0k]) : 0u;
    };
    // wetting value of the solid node at LDS position (yy, xx) of a plane from the fluid
    // plane in LDS slot sf on the side dz (the neighbours x + c_i with c_z = dz), summed in
    // the order of k_wet and rounded as a stored rho^N field holds it
    auto wet_at = [&](int sf, int dz, int yy, int xx) -> M {
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (Lat<Q>::cz[i] != dz) continue;
            num += weight<Q>(i) *
                   static_cast<double>(rn[sf][yy + Lat<Q>::cy[i]][xx + Lat<Q>::cx[i]]);
            den += weight<Q>(i);
        }
        return static_cast<M>(static_cast<MomT<S>>(den > 0.0 ? num / den : 0.0));
    };
    auto put_wet = [&](int slot, int sf, int dz) {
        if (own) rn[slot][ly + R][lx + R] = wet_at(sf, dz, ly + R, lx + R);
        if (ring) rn[slot][ry + R][rx + R] = wet_at(sf, dz, ry + R, rx + R);
    };

    Pulled<Q, S, M, UNIT> cur, nxt;  // plane waiting to be finished, plane being pulled
    cur.s = M(0);
    double acc_s = 0.0, acc_n = 0.0;

    // a lid just below the chunk takes its wetting values from the plane below it
    const int ps = (PW && (kind(z0 - 1) & kPlaneFluidBelow)) ? z0 - 2 : z0 - 1;
    auto slot_of = [&](int zp) { return (zp - ps + 3) % 3; };
    for (int p = ps; p <= z1; ++p) {
        const int pz = wrapf(p, g.nz);
        const uint32_t kp = kind(p);
        const int slot = slot_of(p);
        if (!(kp & kPlaneSolid)) {
            const uint32_t zoff[3] = {(uint32_t)wrap1(pz - 1, g.nz) * plane_bytes,
                                      (uint32_t)pz * plane_bytes,
                                      (uint32_t)wrap1(pz + 1, g.nz) * plane_bytes};
            // bounce-back where the source plane is solid: c_z = -1 from plane p + 1 (bit 0),
            // c_z = +1 from plane p - 1 (bit 2)
            const uint32_t bb = PW ? (((kind(p + 1) & kPlaneSolid) ? 1u : 0u) |
                                      ((kind(p - 1) & kPlaneSolid) ? 4u : 0u))
                                   : 0u;
            M r_ring = M(0), r_own = M(0), r_ring2 = M(0);
            if (ring)
                r_ring = pull_node<Q, S, M, false, UNIT, PW>(sft, sdd, pr, zoff, slot_bytes, bb, P,
                                                             cin, rphi, has_phi,
                                                             ring_xy + (uint32_t)pz * nplane, nxt,
                                                             nullptr, 0);
            if (own)
                r_own = pull_node<Q, S, M, true, UNIT, PW>(sft, sdd, po, zoff, slot_bytes, bb, P,
                                                           cin, rphi, has_phi,
                                                           own_xy + (uint32_t)pz * nplane, nxt,
                                                           &ftl[UNIT ? 0 : (p & 1)][0][tid],
                                                           kFTX * kFTY);
            const bool far = PW && (kp & kPlaneNearWall) && ring2;
            if (far) {  // the second ring, for the wetting values of the wall next to plane p
                const int g2x = wrapf(x0 + r2x, g.nx), g2y = wrapf(y0 + r2y, g.ny);
                const Plane9<S> p2 = plane9<S>(g, g2x, g2y);
                r_ring2 = pull_node<Q, S, M, false, UNIT, PW>(
                    sft, sdd, p2, zoff, slot_bytes, bb, P, cin, rphi, has_phi,
                    (uint32_t)g2x + (uint32_t)g.nx * (uint32_t)g2y + (uint32_t)pz * nplane, nxt,
                    nullptr, 0);
            }
            __syncthreads();  // every thread is done reading the slot about to be overwritten
            if (own) rn[slot][ly + R][lx + R] = r_own;
            if (ring) rn[slot][ry + R][rx + R] = r_ring;
            if (far) rn[slot][r2y + R][r2x + R] = r_ring2;
        } else {
            __syncthreads();
            if (kp & kPlaneFluidBelow)  // a lid: wetting values from the plane below
                put_wet(slot, slot_of(p - 1), -1);
            else if (!(kp & kPlaneFluidAbove)) {  // no fluid neighbour: the wetting value 0
                if (own) rn[slot][ly + R][lx + R] = M(0);
                if (ring) rn[slot][ry + R][rx + R] = M(0);
            }  // a floor waits for the plane above it
        }
        __syncthreads();
        if (PW && p - 1 >= ps) {  // a floor below plane p: its wetting values from plane p
            const uint32_t km = kind(p - 1);
            if ((km & kPlaneSolid) && (km & kPlaneFluidAbove)) {
                put_wet(slot_of(p - 1), slot, 1);
                __syncthreads();
            }
        }

        const int pc = p - 1;  // plane to finish
        if (pc >= z0 && own) {
            const uint32_t n = own_xy + (uint32_t)pc * nplane;
            if (PW && (kind(pc) & kPlaneSolid)) {
                cout[n] = 0;  // solid nodes carry no site
            } else {
                if (cur.s != M(0)) {
                    acc_s += static_cast<double>(cur.s);
                    acc_n += 1.0;
                }
                const M rho = P.rho_ref + cur.drho;
                const M inv_rho = M(1) / rho;
                const M u[3] = {cur.j[0] * inv_rho, cur.j[1] * inv_rho, cur.j[2] * inv_rho};
                const M rN = static_cast<M>(static_cast<MomT<S>>(cur.dsum / rho));  // as in the ring
                // gradient from the LDS ring: planes pc-1, pc, pc+1
                const int sl[3] = {slot_of(pc - 1), slot_of(pc), slot};  // cz = -1, 0, +1
                M F[3] = {M(0), M(0), M(0)};
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const int cx = Lat<Q>::cx[i], cy = Lat<Q>::cy[i], cz = Lat<Q>::cz[i];
                    const M v = M(weight<Q>(i)) * rn[sl[cz + 1]][ly + R + cy][lx + R + cx];
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
                    [&](int i) {
                        return UNIT ? M(0) : static_cast<M>(ftl[UNIT ? 0 : (pc & 1)][UNIT ? 0 : i][tid]);
                    },
                    cur.drho, rho,
                    rN, u, F, P,
                    [&](int i, M a, M d) {
                        const uint32_t so = (uint32_t)i * slot_bytes + zo;
                        Buf<S>::st(enc<S, M>(a, sr_bits(salt, g.N, n, 2 * i)), dft, vo, so, nt);
                        Buf<S>::st(enc<S, M>(d, sr_bits(salt, g.N, n, 2 * i + 1)), ddd, vo, so, nt);
                    });
                cout[n] = Fn > P.gamma ? 1 : 0;
            }
        }
        if (own && p < z1 && !(kp & kPlaneSolid)) cur = nxt;
    }

    double v[2] = {acc_s, acc_n};
    const bool is_max[2] = {false, false};
    double out[2];
    block_reduce<2>(v, is_max, tid, kFTX * kFTY, out);
    if (tid == 0) {
        acc_sink[bid] += out[0];
        acc_sites[bid] += static_cast<long long>(out[1]);
    }
}

__global__ __launch_bounds__(256) void k_copy_bytes(const uint8_t* __restrict__ src,
                                                    uint8_t* __restrict__ dst, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Solid nodes per z-plane: blocks blockIdx.y, blockIdx.y + gridDim.y, ... take planes; each
// block adds its count of a plane once.
__global__ __launch_bounds__(256) void k_plane_count(const uint8_t* __restrict__ flags,
                                                     long long plane, int nz,
                                                     unsigned* __restrict__ cnt) {
    __shared__ unsigned sh[4];
    for (int z = blockIdx.y; z < nz; z += gridDim.y) {
        const uint8_t* f = flags + (long long)z * plane;
        unsigned c = 0;
        for (long long i = blockIdx.x * 256ll + threadIdx.x; i < plane;
             i += (long long)gridDim.x * 256)
            c += f[i] != 0 ? 1u : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(cnt + z, sh[0] + sh[1] + sh[2] + sh[3]);
        __syncthreads();
    }
}

__global__ void k_zero_u32(unsigned* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

cge_status fused_classify(cge_ctx* c) {
    c->plane_walls = false;
    if (!c->flags || !c->pkind || !c->pcount) return CGE_OK;
    const int nz = c->g.nz;
    const long long plane = (long long)c->g.nx * c->g.ny;
    hipLaunchKernelGGL(k_zero_u32, dim3((nz + 255) / 256), dim3(256), 0, c->stream, c->pcount, nz);
    const long long bx = (plane + 255) / 256;
    hipLaunchKernelGGL(k_plane_count, dim3((unsigned)(bx < 64 ? bx : 64), (unsigned)(nz < 4096 ? nz : 4096)),
                       dim3(256), 0, c->stream, c->flags, plane, nz, c->pcount);
    if (cge_status s = check(c, hipGetLastError(), "plane classification launch")) return s;
    std::vector<unsigned> cnt((size_t)nz);
    if (cge_status s = check(c, hipMemcpyAsync(cnt.data(), c->pcount, nz * sizeof(unsigned),
                                               hipMemcpyDeviceToHost, c->stream),
                             "plane classification"))
        return s;
    if (cge_status s = check(c, hipStreamSynchronize(c->stream), "plane classification"))
        return s;
    std::vector<unsigned char> kind((size_t)nz, 0);
    auto solid = [&](int z) { return cnt[(size_t)((z % nz + nz) % nz)] == (unsigned)plane; };
    for (int z = 0; z < nz; ++z) {
        if (cnt[z] != 0 && cnt[z] != (unsigned)plane) return CGE_OK;  // a mixed plane
        if (solid(z)) {
            const bool below = !solid(z - 1), above = !solid(z + 1);
            if (below && above) return CGE_OK;  // fluid on both sides (or nz < 3)
            kind[z] = kPlaneSolid | (below ? kPlaneFluidBelow : 0) | (above ? kPlaneFluidAbove : 0);
        } else if (solid(z - 1) || solid(z + 1)) {
            kind[z] = kPlaneNearWall;
        }
    }
    if (cge_status s = check(c, hipMemcpyAsync(c->pkind, kind.data(), (size_t)nz,
                                               hipMemcpyHostToDevice, c->stream),
                             "plane classification"))
        return s;
    if (cge_status s = check(c, hipStreamSynchronize(c->stream), "plane classification"))
        return s;
    c->plane_walls = true;
    return CGE_OK;
}

// The Q slots of one component must fit a raw buffer's unsigned 32-bit byte range; solid
// nodes only as plane walls.
bool fused_supported(const cge_ctx* c) {
    const long long elem = c->p.precision == CGE_FP64 ? 8 : (c->p.precision == CGE_FP32S ? 4 : 2);
    return c->Q == 19 && (c->flags == nullptr || c->plane_walls) &&
           c->p.site_rule != CGE_SITE_SOFT && 19ll * c->g.N * elem < (1ll << 32);
}

// dynamic LDS of a workgroup: the kinds of the planes z0 - 3 .. z1 + 1 of its chunk
static size_t fused_kinds_bytes(int zlen) { return ((size_t)zlen + 5 + 3) & ~(size_t)3; }

// workgroups of the fused step at one plane per chunk, the most any chunk length gives
long long fused_blocks(const cge_ctx* c) { return fused_shape(c->g, 1).nb; }

template <int Q, typename S, typename M, bool WALLS>
static cge_status fused_impl(cge_ctx* c, long long nsteps) {
    if constexpr (Q != 19) {
        return fail(c, CGE_EUNSUPPORTED, "fused step needs D3Q19");
    } else {
        if (WALLS && !c->plane_walls)
            return fail(c, CGE_EUNSUPPORTED, "fused step: solid nodes other than plane walls");
        const Phys<M> P = phys<M>(c);
        const FusedShape fs = fused_shape(c->g, c->zchunk);
        if (fs.nb > c->acc_len) return fail(c, CGE_ESTATE, "accumulator too small");
        const uint64_t seedmix = mix64(c->p.seed);
        const bool unit = c->p.tau[0] == 1.0 && c->p.tau[1] == 1.0;
        uint8_t* mask[2] = {c->carry, c->carry2};
        const uint8_t* pk = WALLS ? c->pkind : nullptr;
        const size_t kbytes = WALLS ? fused_kinds_bytes(fs.zlen) : 0;
        int m = 0;
        for (long long t = 0; t < nsteps; ++t) {
            const S* src = static_cast<const S*>(c->pop[c->cur]);
            S* dst = static_cast<S*>(c->pop[1 - c->cur]);
            const uint64_t salt = mix64(seedmix + (uint64_t)c->step) * 0x100000001B3ull;
            timing_begin(c, "fused step");
            by_policy(c->g.nt, kNtPop, [&](auto nts) {
                constexpr bool NTS = decltype(nts)::value;
                if (unit)
                    hipLaunchKernelGGL((k_fused<Q, S, M, true, WALLS, NTS>), dim3((unsigned)fs.nb),
                                       dim3(kFTX * kFTY), kbytes, c->stream, src, dst, mask[m],
                                       mask[1 - m], c->phi_field, pk, c->acc_sink, c->acc_sites,
                                       c->g, P, salt, fs);
                else
                    hipLaunchKernelGGL((k_fused<Q, S, M, false, WALLS, NTS>), dim3((unsigned)fs.nb),
                                       dim3(kFTX * kFTY), kbytes, c->stream, src, dst, mask[m],
                                       mask[1 - m], c->phi_field, pk, c->acc_sink, c->acc_sites,
                                       c->g, P, salt, fs);
            });
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
