// Split step for unit relaxation times (tau_r = tau_b = 1): two passes, populations read once,
// and its record form, which keeps a per-node post-collision record between the steps of
// one call instead of the populations.
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

// The moment record of node n between the two passes: rho^N and (delta rho, j), stored at
// the record's precision T.  Where the record is too large to stay in the last-level cache
// (Geo::nt kNtMom) the stores are non-temporal: the next pass reads them after the rest of
// this pass's traffic, and allocated normally they only displace the data this pass
// re-reads (measured: the FP32 finish from records 0.304 -> 0.285 ms at 256^3).  A record
// that fits stays cached for the next pass (non-temporal, the 1024^2 D2Q9 split step ran
// 20 % slower).
template <bool NTS, typename T, typename V, typename W>
__device__ __forceinline__ void store_moments(T* __restrict__ rhoN, T* __restrict__ mom,
                                              const Geo& g, long long n, V rn, W drho,
                                              const W (&j)[3]) {
    const long long N = g.N;
    st_pol<NTS>(rhoN + n, static_cast<T>(rn));
    st_pol<NTS>(mom + n, static_cast<T>(drho));
    st_pol<NTS>(mom + N + n, static_cast<T>(j[0]));
    st_pol<NTS>(mom + 2 * N + n, static_cast<T>(j[1]));
    st_pol<NTS>(mom + 3 * N + n, static_cast<T>(j[2]));
}

// Pass 1: pull, sink, moments; FP64 sink bookkeeping per block.
template <int Q, typename S, typename M, bool WALLS, bool NTS>
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
        store_moments<NTS>(rhoN, mom, g, n, dsum / rho, drho, j);
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
template <int Q, typename S, typename M, bool WALLS, bool NTS>
__global__ __launch_bounds__(kTPBX) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_finish(S* __restrict__ dst,
                                                  const uint8_t* __restrict__ flags,
                                                  void* __restrict__ carry,
                                                  const MomT<S>* __restrict__ rhoN,
                                                  const MomT<S>* __restrict__ mom, Geo g,
                                                  Phys<M> P, uint64_t salt) {
    int x, y, z;
    long long n;
    // banded block order: the rho^N rows around a block stay in one L2 (FP32 storage 14 %
    // faster); at FP16 storage the pass is bound by the stochastic rounding and the plain
    // order measured faster
    constexpr bool banded = !std::is_same<S, _Float16>::value;
    const RowPos pos = banded ? xcd_row(g) : RowPos{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
    const bool valid = node_xyz_at(g, pos, x, y, z, n);
    const RowOff r = row_offsets_at<MomT<S>>(g, pos, x < g.nx ? x : 0);  // offsets into rho^N
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
                                         S* pa = uniform_ptr(dst + (long long)i * g.N + row);
                                         S* pd = uniform_ptr(dst + (long long)(Q + i) * g.N + row);
                                         st_nt<NTS>(reinterpret_cast<S*>(reinterpret_cast<char*>(pa) + xb), a,
                                               sr_bits(salt, g.N, n, 2 * i));
                                         st_nt<NTS>(reinterpret_cast<S*>(reinterpret_cast<char*>(pd) + xb), d,
                                               sr_bits(salt, g.N, n, 2 * i + 1));
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

template <typename S, typename M, bool NTS>
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
                                         st_nt<NTS>(dst + (long long)i * g.N + n, a, sr_bits(salt, g.N, n, 2 * i));
                                         st_nt<NTS>(dst + (long long)(Q + i) * g.N + n, d,
                                               sr_bits(salt, g.N, n, 2 * i + 1));
                                     });
    carry_store(P, carry, n, Fn);
}

// ---------------------------------------------------------------- record form
//
// Between the steps of one call the state is the post-collision record of every node
// (record_values) instead of its 2Q populations: k_finish_record stores the 14 record
// values where k_finish stores the populations, and k_pull_record rebuilds each pulled
// population from the source node's record (record_dir) where k_moments loads it.  The
// first step of a call pulls populations and the last stores them, so callers only see
// populations.  Per node and step: 14 values read and 14 written (FP32 next to FP32 or FP16
// populations, FP64 next to FP64) instead of 2Q and 2Q.  A pulled population is rebuilt in
// the record's precision (a few operations per direction, record_dir) and summed into the
// moments in the arithmetic type.

// Record layout: rows of nodes (y, z) one after the other; within a row, chunks of W
// nodes (256 B of one value), and within a chunk the 14 values one after the other.  A
// node's values are then at one offset plus the value index times 256 B, which the load
// instruction takes as its immediate offset, and the rows around a node are 9 scalar bases.
template <typename R>
struct RecLayout {
    static constexpr int W = 256 / (int)sizeof(R);  // nodes per chunk
    __host__ __device__ static long long row_len(int nx) {  // elements per row of nodes
        return (long long)((nx + W - 1) / W) * W * kRec;
    }
    __host__ __device__ static uint32_t in_row(int x) {  // element offset of x within its row
        return (uint32_t)(x / W) * (uint32_t)(W * kRec) + (uint32_t)(x % W);
    }
};

// Sum over the weight classes of t_ref,k times the pulled rho^N of that class (the part of
// the colour differences record_dir leaves to the arithmetic type).
template <int Q, typename M>
__device__ __forceinline__ M ref_part(const Phys<M>& P, const M (&rn)[3]) {
    constexpr int i1 = 1, i2 = Q == 9 ? 5 : 7;
    M s = M(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = k == 0 ? 0 : (k == 1 ? i1 : i2);
        s += P.rho_ref * (M(restA<Q>(i)) + M(restB<Q>(i)) * P.alpha_ref) * rn[k];
    }
    return s;
}

// Pass 1 from records: pull (Eq. Stream) with every population rebuilt from the record of
// x - c_i (of x itself, opposite direction, where x - c_i is solid), then the sink and the
// moments exactly as k_moments.
template <int Q, typename S, typename M, bool WALLS, bool NTS>
__global__ __launch_bounds__(kTPBX) void k_pull_record(const RecT<S>* __restrict__ rec,
                                                       const uint8_t* __restrict__ flags,
                                                       const void* __restrict__ carry,
                                                       const void* __restrict__ phi_field,
                                                       MomT<S>* __restrict__ rhoN,
                                                       MomT<S>* __restrict__ mom,
                                                       double* __restrict__ acc_sink,
                                                       long long* __restrict__ acc_sites, Geo g,
                                                       Phys<M> P) {
    using R = RecT<S>;
    using E = RecE<R>;  // the rebuild's arithmetic type
    using L = RecLayout<R>;
    int x, y, z;
    long long n;
    const RowPos pos = xcd_row(g);
    const bool valid = node_xyz_at(g, pos, x, y, z, n);
    const long long rlen = L::row_len(g.nx);
    // rows y-1..y+1 and planes z-1..z+1 (row index y + ny z), x-1..x+1 within a row
    long long yr[3], zr[3];
    uint32_t xo[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        yr[d] = (long long)__builtin_amdgcn_readfirstlane(wrapc(pos.y - 1 + d, g.ny)) * rlen;
        zr[d] = (long long)__builtin_amdgcn_readfirstlane(wrapc(pos.z - 1 + d, g.nz)) * g.ny * rlen;
        xo[d] = L::in_row(wrapc((x < g.nx ? x : 0) - 1 + d, g.nx)) * (uint32_t)sizeof(R);
    }
    double v[2] = {0.0, 0.0};
    if (valid && !(WALLS && flags[n])) {
        M j[3] = {M(0), M(0), M(0)}, drho = M(0), dsum = M(0), rn[3] = {M(0), M(0), M(0)};
        const Nb b = WALLS ? wrap(g, x, y, z) : Nb{};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            E ar, dr, rr;
            if constexpr (WALLS) {
                const int cx = Lat<Q>::cx[i], cy = Lat<Q>::cy[i], cz = Lat<Q>::cz[i];
                int sx = cx == 1 ? b.xm : (cx == -1 ? b.xp : x);
                int sy = cy == 1 ? b.ym : (cy == -1 ? b.yp : y);
                int sz = cz == 1 ? b.zm : (cz == -1 ? b.zp : z);
                E sgn = E(1);
                if (i != 0 && flags[lin(g, sx, sy, sz)]) {  // halfway bounce-back: f_opp(i)*(x)
                    sx = x;
                    sy = y;
                    sz = z;
                    sgn = E(-1);
                }
                const R* base = rec + ((long long)sy + (long long)g.ny * sz) * rlen + L::in_row(sx);
                record_dir<Q, E>(i, sgn, [&](int sl) { return static_cast<E>(base[sl * L::W]); },
                                 ar, dr, rr);
            } else {
                const R* base = rec + yr[1 - Lat<Q>::cy[i]] + zr[1 - Lat<Q>::cz[i]];
                const uint32_t o = xo[1 - Lat<Q>::cx[i]];
                record_dir<Q, E>(i, E(1),
                                 [&](int sl) { return static_cast<E>(ld_at(base + sl * L::W, o)); },
                                 ar, dr, rr);
            }
            const M a = static_cast<M>(ar);
            drho += a;
            dsum += static_cast<M>(dr);
            rn[norm2<Q>(i)] += static_cast<M>(rr);
            if (Lat<Q>::cx[i]) j[0] += Lat<Q>::cx[i] * a;
            if (Lat<Q>::cy[i]) j[1] += Lat<Q>::cy[i] * a;
            if (Lat<Q>::cz[i]) j[2] += Lat<Q>::cz[i] * a;
        }
        dsum += ref_part<Q, M>(P, rn);
        const M rho = P.rho_ref + drho;
        M wgt;
        const M s = site_sink<S>(P, carry, phi_field, n, rho, dsum, wgt);
        dsum -= M(2) * s;
        v[0] = static_cast<double>(s);
        v[1] = is_site(wgt) ? 1.0 : 0.0;
        store_moments<NTS>(rhoN, mom, g, n, dsum / rho, drho, j);
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

// Pass 1 from records for D3Q19 (FP64, FP32 or half records): a block takes a 64 x TY tile of nodes
// through zc consecutive planes (zm_chunk).  One plane of records (the tile and one node
// around it) is staged in LDS at a time, in two buffers: while plane p is read, plane p + 1
// is copied into the other buffer, one barrier per plane.  Each thread keeps the partial
// moments of its nodes in planes p - 1, p and p + 1: staged plane p gives node p - 1 its
// directions with c_z = -1 (the node is then complete and finished), node p those with
// c_z = 0 and node p + 1 those with c_z = +1.  Every pulled population is rebuilt once, as
// in k_pull_record, and summed in the order in which the planes arrive (PullSums gives the
// precision of the sums).  With walls the solid flags of planes p - 1 .. p + 1 sit in a
// ring of four beside the records, and a direction whose source is solid takes the node's
// own record (halfway bounce-back) while the node's own plane is staged.  Staging one plane
// instead of three lets taller tiles fit (fewer halo rows per node) with more waves per CU.
// Staged values are E: FP64 for FP64 records (two buffers then take 148 KB, one block per
// CU), FP32 otherwise (half records are widened as they land).
template <int TY, typename E = float>
struct Zm {
    static constexpr int X = 64, W = X + 2, H = TY + 2;
    static constexpr int T = X * TY;                // threads
    static constexpr int P = kRec * H * W;          // staged values (type E) per buffer
    static constexpr int HaloSeg = 2 * kRec;        // 64-node segments of the two halo rows
    static constexpr int F = H * W;                 // staged flags per plane
    // blocks per CU as the LDS allows (two buffers of records, four of flags, the block
    // reduction)
    static constexpr int LdsBytes = 2 * P * (int)sizeof(E) + 4 * F + 256;
    static constexpr int PerCU = (160 * 1024) / LdsBytes < 2048 / T ? (160 * 1024) / LdsBytes
                                                                     : 2048 / T;
    static constexpr int Waves = PerCU * TY / 4;    // waves per SIMD
    static_assert(2 * kRec * H <= T && F <= 2 * T && PerCU >= 1, "staging layout");
};
constexpr int kZmY = 8;

// Site data of a node read a plane ahead of its finish, as loaded: the carried mask byte or
// the bits of ||F|| (as site_weight reads them) and the node's flux as stored (node_phi).
// Nothing is converted at the load, so no wait for it follows until the node is finished.
template <typename S>
struct SiteRaw {
    double c2;     // ||F|| (soft rule)
    uint32_t c0;   // mask byte (gradient rule)
    PhiT<S> phi;   // flux of the node (with a flux field)
};

template <typename S, typename M>
__device__ __forceinline__ void site_ahead(const Phys<M>& P, const void* __restrict__ carry,
                                           const void* __restrict__ phi_field, long long n,
                                           SiteRaw<S>& r) {
    if (P.site_rule == 2) r.c2 = static_cast<const double*>(carry)[n];
    if (P.site_rule == 0) r.c0 = static_cast<const uint8_t*>(carry)[n];
    if (phi_field) r.phi = static_cast<const PhiT<S>*>(phi_field)[n];
}

// site_sink on the data site_ahead read: the same weight and sink arithmetic.
template <typename S, typename M>
__device__ __forceinline__ M site_sink_ahead(const Phys<M>& P, const SiteRaw<S>& r,
                                             const void* __restrict__ phi_field, M rho, M dsum,
                                             M& w) {
    if (P.site_rule == 2) w = M(1) / (M(1) + exp(-(static_cast<M>(r.c2) - P.gamma) * P.inv_kappa));
    else if (P.site_rule == 0) w = r.c0 != 0u ? M(1) : M(0);
    else w = fabs(dsum / rho) < P.gamma ? M(1) : M(0);
    if (w == M(0)) return M(0);
    const M phi = phi_field ? static_cast<M>(r.phi) : P.phi;
    return w * (phi * P.inv_sbar);
}

// Partial moments of one node: delta rho, the colour sum and j in the rebuild's type E, and
// the pulled rho^N per weight class (ref_part) in the arithmetic type.  With FP32 E the sums
// take 5 to 9 FP32 rebuilds of FP32 record values and are stored as FP32 moments straight
// after, so they add a few units in the last place before that rounding; the class sums of
// rho^N, which ref_part weights by t_ref,k, stay in M, where FP32 rounding would repeat at
// every node and step.
template <typename M, typename E>
struct PullSums {
    E drho, dsum, j[3];
    M rn[3];
    __device__ __forceinline__ void clear() {
        drho = dsum = E(0);
        j[0] = j[1] = j[2] = E(0);
        rn[0] = rn[1] = rn[2] = M(0);
    }
};

// The D3Q19 directions with c_z = cz, in index order.
struct CzList {
    int n, i[9];
};
constexpr CzList cz_list(int cz) {
    CzList l{0, {0, 0, 0, 0, 0, 0, 0, 0, 0}};
    for (int d = 0; d < 19; ++d)
        if (Lat<19>::cz[d] == cz) l.i[l.n++] = d;
    return l;
}

template <typename S, int TY>
using ZmOf = Zm<TY, RecE<RecT<S>>>;

template <typename S, typename M, bool WALLS, int TY, bool NTS>
__global__ __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(ZmOf<S, TY>::Waves, ZmOf<S, TY>::Waves))) void
k_pull_record_zm(const RecT<S>* __restrict__ rec, const uint8_t* __restrict__ flags,
                 const void* __restrict__ carry, const void* __restrict__ phi_field,
                 MomT<S>* __restrict__ rhoN, MomT<S>* __restrict__ mom,
                 double* __restrict__ acc_sink, long long* __restrict__ acc_sites, Geo g,
                 Phys<M> P, int zc) {
    constexpr int Q = 19;
    using R = RecT<S>;  // double, float, or half (then staged through registers, below)
    using E = RecE<R>;  // the staged values and the rebuild: double, or float
    constexpr bool kHalf = std::is_same<R, _Float16>::value;
    using L = RecLayout<R>;
    using Z = ZmOf<S, TY>;
    // the two record buffers (plane p in ring0 when p - z0 is odd) and the flags of plane p
    // in slot p & 3 of fring
    __shared__ E ring0[Z::P];
    __shared__ E ring1[Z::P];
    __shared__ uint8_t fring[WALLS ? 4 * Z::F : 1];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + Z::X * ty;
    // tiles in XCD-contiguous order: XCD k (blocks are dealt round-robin by id) takes a run of
    // consecutive tiles, x fastest, then y, then the z-chunk, so tiles that share halo rows and
    // columns read them through the same L2 at about the same time
    const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
    const unsigned bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned xq = nb / kXcds, xrem = nb % kXcds, xk = bid % kXcds;
    const unsigned tile = xk * xq + (xk < xrem ? xk : xrem) + bid / kXcds;
    const int bx = __builtin_amdgcn_readfirstlane((int)(tile % gridDim.x));
    const int by = __builtin_amdgcn_readfirstlane((int)((tile / gridDim.x) % gridDim.y));
    const int bz = __builtin_amdgcn_readfirstlane((int)(tile / (gridDim.x * gridDim.y)));
    const int x0 = bx * Z::X, y0 = by * TY;
    const int z0 = bz * zc, z1 = min(z0 + zc, g.nz);
    const long long rlen = L::row_len(g.nx);
    const long long plane = (long long)g.ny * rlen;
    // Staging of one plane: row ry of value sl of the window (64 nodes) is row sl H + ry of a
    // buffer.  The rows are copied from HBM straight into LDS (global_load_lds: lane l's value
    // lands at the row's LDS base + 4 l, so a row takes one uniform LDS address and no
    // registers): wave w copies window row w + 1 (a row of the tile) of every value, from one
    // scalar row address with the value's 256-byte chunk slot as the immediate offset, and
    // the Z::HaloSeg rows 0 and H - 1 of the values are shared out over the waves.  Threads
    // tid < 2 kRec H load the two halo columns x0 - 1 and x0 + 64 through a register.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const uint32_t xin = L::in_row(wrapm(x0 + lane, g.nx)) * (uint32_t)sizeof(R);
    // FP64 records: a 64-value row is two 256 B copies; in copy c lane l moves dword l & 1 of
    // the value of node x0 + 32 c + l / 2
    constexpr int kCopies = (int)sizeof(E) / 4 > 1 && !kHalf ? 2 : 1;
    uint32_t xcp[kCopies];
#pragma unroll
    for (int c = 0; c < kCopies; ++c)
        xcp[c] = kCopies == 1 ? xin
                              : L::in_row(wrapm(x0 + 32 * c + (lane >> 1), g.nx)) *
                                        (uint32_t)sizeof(R) + (uint32_t)(lane & 1) * 4u;
    const int hseg = tid >> 1, hside = tid & 1;
    const bool halo = tid < 2 * kRec * Z::H;
    const uint32_t hoff =
        halo ? (uint32_t)(((long long)wrapm(y0 - 1 + hseg % Z::H, g.ny) * rlen +
                           L::in_row(wrapm(hside ? x0 + Z::X : x0 - 1, g.nx)) +
                           (hseg / Z::H) * L::W) * (long long)sizeof(R))
             : 0u;
    const int hlds = hseg * Z::W + (hside ? Z::W - 1 : 0);
    // plane-relative byte offsets (below 2^31: checked at launch) of the wave's tile row and of
    // the two halo rows
    const uint32_t row_own = (uint32_t)((long long)wrapm(y0 + wave, g.ny) * rlen * (long long)sizeof(R));
    const uint32_t row_lo = (uint32_t)((long long)wrapm(y0 - 1, g.ny) * rlen * (long long)sizeof(R));
    const uint32_t row_hi = (uint32_t)((long long)wrapm(y0 + TY, g.ny) * rlen * (long long)sizeof(R));
    // Half records: a row segment of 64 halves is 128 B, so a lane takes one dword, two nodes of
    // one value: lanes 0..31 value 2v and lanes 32..63 value 2v + 1 (the two segments are 256 B
    // apart in the record layout).  nx is even (checked at launch), so a pair never straddles
    // the periodic wrap or a layout chunk.
    const int pr_lane = lane & 31, pr_odd = lane >> 5;
    const uint32_t xpair = L::in_row(wrapm(x0 + 2 * pr_lane, g.nx)) * (uint32_t)sizeof(R);
    constexpr int kHaloPairs = kRec;  // (value pair, halo row) segments: 7 pairs x 2 rows
    struct HalfRows {
        uint32_t own[kRec / 2];
        uint32_t halo[(kHaloPairs + TY - 1) / TY];
        R col;
    };
    // flags: positions tid and tid + Z::T of the (H x W) plane window, in-plane index
    long long fo[2] = {0, 0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int pos = tid + Z::T * h;
        if (WALLS && pos < Z::F)
            fo[h] = wrapm(x0 - 1 + pos % Z::W, g.nx) +
                    (long long)g.nx * wrapm(y0 - 1 + pos / Z::W, g.ny);
    }
    __syncthreads();
    const long long fplane = (long long)g.nx * g.ny;
    // start the copy of plane zp into dst; its halo columns come back in hb (a value's
    // 256 B layout chunk holds 256 / sizeof(R) nodes, so values are 256 B apart)
    auto issue_plane = [&](int zp, E* dst, E& hb) {
        const char* base = reinterpret_cast<const char*>(rec + (long long)wrapm(zp, g.nz) * plane);
        const char* own = base + row_own;
#pragma unroll
        for (int sl = 0; sl < kRec; ++sl)
#pragma unroll
            for (int c = 0; c < kCopies; ++c)
                __builtin_amdgcn_global_load_lds(own + xcp[c] + sl * 256,
                                                 dst + (sl * Z::H + 1 + wave) * Z::W + 1 + 32 * c,
                                                 4, 0, 0);
#pragma unroll
        for (int m = 0; m < (Z::HaloSeg + TY - 1) / TY; ++m) {
            const int k = wave + TY * m;  // halo row segment: value k % kRec, row 0 or H - 1
            if (k < Z::HaloSeg) {
                const int sl = k % kRec, hi = k / kRec;
#pragma unroll
                for (int c = 0; c < kCopies; ++c)
                    __builtin_amdgcn_global_load_lds(
                        base + (hi ? row_hi : row_lo) + sl * 256 + xcp[c],
                        dst + (sl * Z::H + (hi ? Z::H - 1 : 0)) * Z::W + 1 + 32 * c, 4, 0, 0);
            }
        }
        if (halo) hb = ld_at(reinterpret_cast<const E*>(base), hoff);
    };
    // Half records: start the loads of plane zp into registers ...
    auto issue_half = [&](int zp, HalfRows& hr) {
        const char* base = reinterpret_cast<const char*>(rec + (long long)wrapm(zp, g.nz) * plane);
        const char* own = base + row_own;
#pragma unroll
        for (int v = 0; v < kRec / 2; ++v)
            hr.own[v] = ld_at(reinterpret_cast<const uint32_t*>(own),
                              xpair + (uint32_t)((2 * v + pr_odd) * L::W * 2));
#pragma unroll
        for (int m = 0; m < (kHaloPairs + TY - 1) / TY; ++m) {
            const int k = wave + TY * m;  // value pair k % 7, halo row k / 7 (0: y0 - 1)
            if (k < kHaloPairs)
                hr.halo[m] = ld_at(reinterpret_cast<const uint32_t*>(
                                       base + ((k / (kRec / 2)) ? row_hi : row_lo)),
                                   xpair + (uint32_t)((2 * (k % (kRec / 2)) + pr_odd) * L::W * 2));
        }
        if (halo) hr.col = ld_at(reinterpret_cast<const R*>(base), hoff);
    };
    // ... and put them into dst as floats, where issue_plane's copies land
    auto land_half = [&](E* dst, const HalfRows& hr) {
        auto put2 = [&](E* d, uint32_t w) {
            d[0] = static_cast<float>(__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu)));
            d[1] = static_cast<float>(__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)));
        };
#pragma unroll
        for (int v = 0; v < kRec / 2; ++v)
            put2(dst + ((2 * v + pr_odd) * Z::H + 1 + wave) * Z::W + 1 + 2 * pr_lane, hr.own[v]);
#pragma unroll
        for (int m = 0; m < (kHaloPairs + TY - 1) / TY; ++m) {
            const int k = wave + TY * m;
            if (k < kHaloPairs)
                put2(dst + ((2 * (k % (kRec / 2)) + pr_odd) * Z::H +
                            ((k / (kRec / 2)) ? Z::H - 1 : 0)) * Z::W + 1 + 2 * pr_lane,
                     hr.halo[m]);
        }
        if (halo) dst[hlds] = static_cast<E>(hr.col);
    };
    auto load_flags = [&](int zp, uint8_t (&fb)[2]) {
        const uint8_t* fbase = flags + (long long)wrapm(zp, g.nz) * fplane;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (tid + Z::T * h < Z::F) fb[h] = fbase[fo[h]];
    };
    auto store_flags = [&](int zp, const uint8_t (&fb)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (tid + Z::T * h < Z::F) fring[(zp & 3) * Z::F + tid + Z::T * h] = fb[h];
    };
    // the copies into LDS are complete (s_waitcnt 0) before the barrier publishes them
    auto publish = [&]() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };
    {
        if constexpr (kHalf) {
            HalfRows hr;
            issue_half(z0 - 1, hr);
            land_half(ring0, hr);
        } else {
            E hb = E(0);
            issue_plane(z0 - 1, ring0, hb);
            if (halo) ring0[hlds] = hb;
        }
        uint8_t fb[2] = {0, 0};
        if constexpr (WALLS) {
            load_flags(z0 - 1, fb);
            store_flags(z0 - 1, fb);
            load_flags(z0, fb);
            store_flags(z0, fb);
        }
        publish();
    }
    const int x = x0 + tx, y = y0 + ty;
    const bool valid = x < g.nx && y < g.ny;
    const int cen = (ty + 1) * Z::W + (tx + 1);
    auto solid = [&](int zp, int at) { return WALLS && fring[(zp & 3) * Z::F + at] != 0; };
    auto node = [&](int zp) { return x + (long long)g.nx * (y + (long long)g.ny * zp); };
    // The record values direction i reads from its source (dir_slots); without walls they are
    // fetched one direction ahead of their use, so the LDS latency of one direction overlaps
    // the arithmetic of the previous one.
    auto fetch = [&](int i, const E* src, E (&r)[kRec]) {
#pragma unroll
        for (int sl = 0; sl < kRec; ++sl)
            if ((dir_slots<Q>(i) >> sl) & 1u) r[sl] = src[sl * Z::H * Z::W];
    };
    // direction i of a node from fetched record values (sgn -1: the node's own, bounce-back)
    auto accum = [&](PullSums<M, E>& s, int i, const E (&r)[kRec], E sgn) {
        E ar, dr, rr;
        record_dir<Q, E>(i, sgn, [&](int sl) { return r[sl]; }, ar, dr, rr);
        s.drho += ar;
        s.dsum += dr;
        s.rn[norm2<Q>(i)] += static_cast<M>(rr);
        if (Lat<Q>::cx[i]) s.j[0] += Lat<Q>::cx[i] * ar;
        if (Lat<Q>::cy[i]) s.j[1] += Lat<Q>::cy[i] * ar;
        if (Lat<Q>::cz[i]) s.j[2] += Lat<Q>::cz[i] * ar;
        // the empty asm makes the sums of this direction exist here (otherwise they sink to the
        // node's finish and every direction's record values stay live until then)
        asm volatile("" : "+v"(s.drho), "+v"(s.dsum), "+v"(s.j[0]), "+v"(s.j[1]), "+v"(s.j[2]),
                     "+v"(s.rn[0]), "+v"(s.rn[1]), "+v"(s.rn[2]));
    };
    // The directions with c_z = CZ (the tag's value) into s: direction i from the record at
    // src_of(i) with sign sgn_of(i), skipped where take(i) is false.
    auto stage = [&](PullSums<M, E>& s, auto cz_tag, auto src_of, auto sgn_of, auto take) {
        constexpr CzList D = cz_list(decltype(cz_tag)::value);
        E r0[kRec], r1[kRec];
        if constexpr (WALLS) {  // no look-ahead: the flag ring leaves too few registers
#pragma unroll
            for (int k = 0; k < D.n; ++k) {
                fetch(D.i[k], src_of(D.i[k]), r0);
                if (take(D.i[k])) accum(s, D.i[k], r0, sgn_of(D.i[k]));
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            fetch(D.i[0], src_of(D.i[0]), r0);
#pragma unroll
            for (int k = 0; k < D.n; ++k) {
                if (k + 1 < D.n) fetch(D.i[k + 1], src_of(D.i[k + 1]), (k & 1) ? r0 : r1);
                if (take(D.i[k])) accum(s, D.i[k], (k & 1) ? r1 : r0, sgn_of(D.i[k]));
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    using Down = std::integral_constant<int, -1>;
    using Level = std::integral_constant<int, 0>;
    using Up = std::integral_constant<int, 1>;
    auto at_of = [&](int i) { return (ty + 1 - Lat<Q>::cy[i]) * Z::W + (tx + 1 - Lat<Q>::cx[i]); };
    PullSums<M, E> sa, sb;
    sa.clear();
    sb.clear();
    SiteRaw<S> site_fin{0.0, 0u, PhiT<S>(0)};
    double v[2] = {0.0, 0.0};
    // One plane: pl holds plane p, the copy of plane p + 1 goes to nxt; prev holds the partial
    // moments of node p - 1 and cur those of node p, and prev takes node p + 1's afterwards.
    auto march = [&](int p, const E* pl, E* nxt, PullSums<M, E>& prev, PullSums<M, E>& cur) {
        const bool next = p < z1;
        const bool own = valid && p >= z0 && p < z1 && !solid(p, cen);
        SiteRaw<S> site_next{0.0, 0u, PhiT<S>(0)};
        if (own) site_ahead<S, M>(P, carry, phi_field, node(p), site_next);
        E hb = E(0);
        HalfRows hr;
        uint8_t fb[2] = {0, 0};
        if (next) {
            if constexpr (kHalf) issue_half(p + 1, hr);
            else issue_plane(p + 1, nxt, hb);
            if constexpr (WALLS) load_flags(p + 2, fb);
        }
        auto from_plane = [&](int i) { return pl + at_of(i); };
        auto plus = [&](int i) { return E(1); };
        auto fluid_src = [&](int i) { return !solid(p, at_of(i)); };
        // node p - 1: the directions with c_z = -1, then the node is complete
        if (p - 1 >= z0 && valid && !solid(p - 1, cen)) {
            stage(prev, Down{}, from_plane, plus, fluid_src);
            const M dsum = static_cast<M>(prev.dsum) + ref_part<Q, M>(P, prev.rn);
            const M rho = P.rho_ref + static_cast<M>(prev.drho);
            M wgt;
            const M s = site_sink_ahead<S, M>(P, site_fin, phi_field, rho, dsum, wgt);
            const long long n = node(p - 1);
            v[0] += static_cast<double>(s);
            v[1] += is_site(wgt) ? 1.0 : 0.0;
            store_moments<NTS>(rhoN, mom, g, n, (dsum - M(2) * s) / rho, prev.drho, prev.j);
        }
        // node p: the directions with c_z = 0 (from the node's own record where the source is
        // solid), then those with c_z = +-1 whose source is solid
        if (own) {
            auto own_or_src = [&](int i) {
                return (i != 0 && solid(p, at_of(i))) ? pl + cen : pl + at_of(i);
            };
            auto own_sgn = [&](int i) { return (i != 0 && solid(p, at_of(i))) ? E(-1) : E(1); };
            auto all = [&](int i) { return true; };
            stage(cur, Level{}, own_or_src, own_sgn, all);
            if constexpr (WALLS) {
                E r[kRec];
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    if (Lat<Q>::cz[i] == 0 || !solid(p - Lat<Q>::cz[i], at_of(i))) continue;
                    fetch(i, pl + cen, r);
                    accum(cur, i, r, E(-1));
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        // node p + 1: the directions with c_z = +1
        prev.clear();
        if (p + 1 < z1 && valid && !solid(p + 1, cen))
            stage(prev, Up{}, from_plane, plus, fluid_src);
        site_fin = site_next;
        if (next) {
            if constexpr (kHalf) land_half(nxt, hr);
            else if (halo) nxt[hlds] = hb;
            if constexpr (WALLS) store_flags(p + 2, fb);
        }
        publish();
    };
    for (int p = z0 - 1; p <= z1; p += 2) {
        march(p, ring0, ring1, sa, sb);
        if (p + 1 <= z1) march(p + 1, ring1, ring0, sb, sa);
    }
    const bool is_max[2] = {false, false};
    double out[2];
    block_reduce<2>(v, is_max, tid, Z::T, out);
    if (tid == 0) {
        acc_sink[bid] += out[0];
        acc_sites[bid] += static_cast<long long>(out[1]);
    }
}

// Planes per z-chunk.  A chunk's blocks stage zc + 2 planes, and blocks run in rounds of
// Zm::PerCU per CU, so the pass takes about rounds x (planes per chunk + 2) plane-times; the
// chunk count that minimises this is taken.
template <typename E>
static int zm_chunk(const cge_ctx* c) {
    using Z = Zm<kZmY, E>;
    const Geo& g = c->g;
    if (c->zchunk > 0) return c->zchunk < g.nz ? c->zchunk : g.nz;
    const long long tiles = (long long)((g.nx + Z::X - 1) / Z::X) * ((g.ny + kZmY - 1) / kZmY);
    const long long slots = (long long)Z::PerCU * (c->cus > 0 ? c->cus : 1);
    long long best = -1, best_zc = g.nz;
    for (long long chunks = 1; chunks <= g.nz && chunks <= 4096; ++chunks) {
        const long long zc = (g.nz + chunks - 1) / chunks;
        const long long used = (g.nz + zc - 1) / zc;  // chunks of zc planes that cover nz
        const long long rounds = (tiles * used + slots - 1) / slots;
        const long long cost = rounds * (zc + 2);
        if (best < 0 || cost < best) {
            best = cost;
            best_zc = zc;
        }
    }
    return (int)best_zc;
}

static dim3 zm_grid(const Geo& g, int zc) {
    return dim3((g.nx + Zm<kZmY>::X - 1) / Zm<kZmY>::X, (g.ny + kZmY - 1) / kZmY,
                (g.nz + zc - 1) / zc);
}

// Pass 2 to records: gradient and moments as k_finish, then the node's record instead of its
// populations, and the next site data.
template <int Q, typename S, typename M, bool WALLS, bool NTS>
__global__ __launch_bounds__(kTPBX) __attribute__((amdgpu_waves_per_eu(5, 8))) void
k_finish_record(RecT<S>* __restrict__ rec, const uint8_t* __restrict__ flags,
                void* __restrict__ carry, const MomT<S>* __restrict__ rhoN,
                const MomT<S>* __restrict__ mom, Geo g, Phys<M> P, uint64_t salt) {
    using R = RecT<S>;
    int x, y, z;
    long long n;
    const RowPos pos = xcd_row(g);
    const bool valid = node_xyz_at(g, pos, x, y, z, n);
    const RowOff r = row_offsets_at<MomT<S>>(g, pos, x < g.nx ? x : 0);
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
    } else {  // F = 3 sum_i W_i rho^N(x + c_i) c_i, as k_finish
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
    M rv[kRec];
    const M Fn = record_values<Q, M>(drho, rho, static_cast<M>(rhoN[n]), u, F, P, rv);
    using L = RecLayout<R>;
    R* at = rec + ((long long)y + (long long)g.ny * z) * L::row_len(g.nx) + L::in_row(x);
#pragma unroll
    for (int sl = 0; sl < kRec; ++sl) {
        if (Q == 9 && (sl == kUz || sl == kNz)) continue;  // no z component in 2D
        // half records round stochastically, like half populations
        st_pol<NTS>(at + sl * L::W, enc<R, M>(rv[sl], sr_bits(salt, g.N, n, sl)));
    }
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
    timing_begin(c, "split step");
    by_policy(c->g.nt, kNtMom, [&](auto nts) {
        hipLaunchKernelGGL((k_moments<Q, S, M, WALLS, decltype(nts)::value>), gr, bl, 0, c->stream,
                           src, c->flags, carry_in, c->phi_field, rhoN, mom, c->acc_sink,
                           c->acc_sites, c->g, P);
    });
    if (WALLS) hipLaunchKernelGGL((k_wet<Q, MomT<S>>), gr, bl, 0, c->stream, c->flags, rhoN, c->g);
    timing_pass(c, "k_moments");
    if constexpr (Q == 19 && !WALLS && std::is_same<S, double>::value) {
        const dim3 tb(kTileX, kTileY, 1);
        const dim3 tg((c->g.nx + kTileX - 1) / kTileX, (c->g.ny + kTileY - 1) / kTileY, c->g.nz);
        by_policy(c->g.nt, kNtPop, [&](auto nts) {
            hipLaunchKernelGGL((k_finish_tile<S, M, decltype(nts)::value>), tg, tb, 0, c->stream,
                               dst, carry_out, rhoN, mom, c->g, P, salt);
        });
        timing_pass(c, "k_finish_tile");
    } else {
        by_policy(c->g.nt, kNtPop, [&](auto nts) {
            hipLaunchKernelGGL((k_finish<Q, S, M, WALLS, decltype(nts)::value>), gr, bl, 0,
                               c->stream, dst, c->flags, carry_out, rhoN, mom, c->g, P, salt);
        });
        timing_pass(c, "k_finish");
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

// The z-marching pass 1 serves D3Q19 (checked where it is launched) when its blocks fit the
// per-block sink accumulators and a plane of records is addressable with 32-bit offsets; half
// records also need an even nx (two nodes per lane).
template <typename R>
static bool zm_ok(const cge_ctx* c) {
    const dim3 gz = zm_grid(c->g, zm_chunk<RecE<R>>(c));
    const long long blocks = (long long)gz.x * gz.y * gz.z;
    const long long plane = (long long)c->g.ny * RecLayout<R>::row_len(c->g.nx) * (long long)sizeof(R);
    return blocks <= c->acc_len && plane < (1ll << 31) &&
           (!std::is_same<R, _Float16>::value || c->g.nx % 2 == 0);
}

// One step of the record form: pass 1 from populations (first step of a call) or records,
// pass 2 to populations (last step) or records.
template <int Q, typename S, typename M, bool WALLS>
static cge_status record_one(cge_ctx* c, bool first, bool last) {
    if (first && last) return split_one<Q, S, M, WALLS>(c, c->carry, c->carry, c->rhoN, c->mom);
    const Phys<M> P = phys<M>(c);
    const dim3 gr = node_grid(c->g), bl = node_block(c->g);
    MomT<S>* rhoN = static_cast<MomT<S>*>(c->rhoN);
    MomT<S>* mom = static_cast<MomT<S>*>(c->mom);
    RecT<S>* rec = static_cast<RecT<S>*>(c->rec);
    const S* src = static_cast<const S*>(c->pop[c->cur]);
    S* dst = static_cast<S*>(c->pop[1 - c->cur]);
    const uint64_t salt = mix64(mix64(c->p.seed) + (uint64_t)c->step) * 0x100000001B3ull;
    timing_begin(c, first ? "record step (from populations)"
                          : (last ? "record step (to populations)" : "record step"));
    const char* pass1 = "k_moments";
    if (first)
        by_policy(c->g.nt, kNtMom, [&](auto nts) {
            hipLaunchKernelGGL((k_moments<Q, S, M, WALLS, decltype(nts)::value>), gr, bl, 0,
                               c->stream, src, c->flags, c->carry, c->phi_field, rhoN, mom,
                               c->acc_sink, c->acc_sites, c->g, P);
        });
    else {
        bool marched = false;
        if constexpr (Q == 19) {
            if (zm_ok<RecT<S>>(c)) {
                const int zc = zm_chunk<RecE<RecT<S>>>(c);
                by_policy(c->g.nt, kNtMom, [&](auto nts) {
                    hipLaunchKernelGGL((k_pull_record_zm<S, M, WALLS, kZmY, decltype(nts)::value>),
                                       zm_grid(c->g, zc), dim3(Zm<kZmY>::X, kZmY, 1), 0, c->stream,
                                       rec, c->flags, c->carry, c->phi_field, rhoN, mom,
                                       c->acc_sink, c->acc_sites, c->g, P, zc);
                });
                marched = true;
                pass1 = "k_pull_record_zm";
            }
        }
        if (!marched) {
            by_policy(c->g.nt, kNtMom, [&](auto nts) {
                hipLaunchKernelGGL((k_pull_record<Q, S, M, WALLS, decltype(nts)::value>), gr, bl, 0,
                                   c->stream, rec, c->flags, c->carry, c->phi_field, rhoN, mom,
                                   c->acc_sink, c->acc_sites, c->g, P);
            });
            pass1 = "k_pull_record";
        }
    }
    if (WALLS) hipLaunchKernelGGL((k_wet<Q, MomT<S>>), gr, bl, 0, c->stream, c->flags, rhoN, c->g);
    timing_pass(c, pass1);
    if (!last) {
        by_policy(c->g.nt, kNtRec, [&](auto nts) {
            hipLaunchKernelGGL((k_finish_record<Q, S, M, WALLS, decltype(nts)::value>), gr, bl, 0,
                               c->stream, rec, c->flags, c->carry, rhoN, mom, c->g, P, salt);
        });
        timing_pass(c, "k_finish_record");
    } else if constexpr (Q == 19 && !WALLS && std::is_same<S, double>::value) {
        const dim3 tb(kTileX, kTileY, 1);
        const dim3 tg((c->g.nx + kTileX - 1) / kTileX, (c->g.ny + kTileY - 1) / kTileY, c->g.nz);
        by_policy(c->g.nt, kNtPop, [&](auto nts) {
            hipLaunchKernelGGL((k_finish_tile<S, M, decltype(nts)::value>), tg, tb, 0, c->stream,
                               dst, c->carry, rhoN, mom, c->g, P, salt);
        });
        timing_pass(c, "k_finish_tile");
    } else {
        by_policy(c->g.nt, kNtPop, [&](auto nts) {
            hipLaunchKernelGGL((k_finish<Q, S, M, WALLS, decltype(nts)::value>), gr, bl, 0,
                               c->stream, dst, c->flags, c->carry, rhoN, mom, c->g, P, salt);
        });
        timing_pass(c, "k_finish");
    }
    timing_end(c);
    if (cge_status s = check(c, hipGetLastError(), "record step launch")) return s;
    c->cur = 1 - c->cur;  // the populations of the last step land where the split step's would
    c->step += 1;
    return CGE_OK;
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status record_impl(cge_ctx* c, long long nsteps) {
    if (!split_supported(c)) return fail(c, CGE_EUNSUPPORTED, "record step needs tau = 1");
    if (!c->mom || !c->rec) return fail(c, CGE_ESTATE, "record scratch missing");
    for (long long t = 0; t < nsteps; ++t)
        if (cge_status s = record_one<Q, S, M, WALLS>(c, t == 0, t == nsteps - 1)) return s;
    return CGE_OK;
}

cge_status record_steps(cge_ctx* c, long long nsteps) { CGE_DISPATCH(c, record_impl, c, nsteps); }

size_t record_bytes(const cge_params* p) {
    const size_t rows = (size_t)p->ny * p->nz;
    if (p->precision == CGE_FP64) return rows * RecLayout<double>::row_len(p->nx) * sizeof(double);
    if (p->precision == CGE_FP16S)
        return rows * RecLayout<_Float16>::row_len(p->nx) * sizeof(_Float16);
    return rows * RecLayout<float>::row_len(p->nx) * sizeof(float);
}


cge_status split_step_into(cge_ctx* c, const void* carry_in, void* carry_out, void* rhoN,
                           void* mom) {
    if (!split_supported(c)) return fail(c, CGE_EUNSUPPORTED, "split step needs tau = 1");
    CGE_DISPATCH(c, split_one, c, carry_in, carry_out, rhoN, mom);
}

}  // namespace cge
