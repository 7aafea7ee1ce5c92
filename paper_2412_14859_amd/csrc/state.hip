// Saved states (cge_save_state, the checkpoints of cge_forward_ckpt) and their integrity check.
//
// Layout of a saved state, sizes from the parameters:
//   [0, pb)                 the current population buffer (pb = cge_population_bytes)
//   [coff, coff + cb)       the carried site data, coff = pb rounded up to 256 bytes
//   [toff, toff + 32)       the trailer, toff = coff + cb rounded up to 256 bytes:
//                           magic, fingerprint, covered bytes (pb + cb), checksum (u64 each,
//                           little-endian)
// checksum: the sum mod 2^64 over the 8-byte little-endian words w_i of the populations and then
// of the site data (each region zero-padded to a multiple of 8 bytes, the word index i running
// on from the first region into the second) of fin(w_i XOR (i * 0xD6E8FEB86659FD93)), where fin
// is one step of the splitmix64 generator applied to its argument (mix64).  Integer addition
// is exact and commutative, so blocks add their partial sums in any order.
// fingerprint: FNV-1a (64-bit) over the bytes of the int32 values lattice, nx, ny, nz,
// precision, site_rule, then the float64 values rho_in[0], rho_in[1] (they fix the layout and
// the encoding's shift), then the format version 1 as int32.
#include <cstring>

#include "internal.hpp"
#include "node.hpp"

namespace cge {

constexpr uint64_t kStateMagic = 0x5441545356454743ull;  // "CGEVSTAT"
constexpr uint64_t kWordKey = 0xD6E8FEB86659FD93ull;
constexpr int kFormatVersion = 1;

struct Trailer {
    uint64_t magic, fingerprint, bytes, checksum;
};

static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t state_carry_offset(const cge_params* p) { return up256(cge_population_bytes(p)); }
size_t state_trailer_offset(const cge_params* p) {
    return up256(state_carry_offset(p) + carry_bytes(p));
}
size_t state_bytes(const cge_params* p) {
    return cge_population_bytes(p) ? state_trailer_offset(p) + sizeof(Trailer) : 0;
}

static uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(data);
    for (size_t k = 0; k < n; ++k) {
        h ^= b[k];
        h *= 0x100000001B3ull;
    }
    return h;
}

static uint64_t fingerprint(const cge_params* p) {
    uint64_t h = 0xCBF29CE484222325ull;
    const int32_t ints[6] = {p->lattice, p->nx, p->ny, p->nz, p->precision, p->site_rule};
    h = fnv1a(h, ints, sizeof(ints));
    h = fnv1a(h, p->rho_in, 2 * sizeof(double));
    const int32_t v = kFormatVersion;
    return fnv1a(h, &v, sizeof(v));
}

// word i of a region of len bytes, zero-padded past its end (the bytes past len are not read)
__host__ __device__ __forceinline__ uint64_t region_word(const unsigned char* base, size_t len,
                                                         size_t j, bool aligned) {
    if (aligned && 8 * j + 8 <= len) return reinterpret_cast<const uint64_t*>(base)[j];
    uint64_t w = 0;
    for (size_t k = 8 * j; k < len && k < 8 * j + 8; ++k) w |= (uint64_t)base[k] << (8 * (k - 8 * j));
    return w;
}

__global__ __launch_bounds__(256) void k_checksum(const unsigned char* __restrict__ a, size_t la,
                                                  bool aa, const unsigned char* __restrict__ b,
                                                  size_t lb, bool ab,
                                                  unsigned long long* __restrict__ out) {
    const size_t na = (la + 7) / 8, nw = na + (lb + 7) / 8;
    unsigned long long s = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t w = i < na ? region_word(a, la, i, aa) : region_word(b, lb, i - na, ab);
        s += mix64(w ^ (i * kWordKey));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ unsigned long long sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, sh[0] + sh[1] + sh[2] + sh[3]);
}

// trailer fields with the checksum cleared (the checksum kernel adds into it)
__global__ void k_trailer_head(Trailer* t, uint64_t magic, uint64_t fp, uint64_t bytes) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        t->magic = magic;
        t->fingerprint = fp;
        t->bytes = bytes;
        t->checksum = 0;
    }
}

static bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

static hipError_t launch_checksum(const void* a, size_t la, const void* b, size_t lb,
                                  unsigned long long* out, hipStream_t s) {
    const size_t nw = (la + 7) / 8 + (lb + 7) / 8;
    const size_t blocks = (nw + 255) / 256;
    hipLaunchKernelGGL(k_checksum, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0,
                       s, static_cast<const unsigned char*>(a), la, aligned8(a),
                       static_cast<const unsigned char*>(b), lb, aligned8(b), out);
    return hipGetLastError();
}

// Copy the current state to dst; with seal, write its trailer too.
cge_status save_state(cge_ctx* c, void* dst, bool seal) {
    const size_t pb = cge_population_bytes(&c->p), cb = carry_bytes(&c->p);
    char* d = static_cast<char*>(dst);
    const size_t coff = state_carry_offset(&c->p);
    if (cge_status s = check(c, hipMemcpyAsync(d, c->pop[c->cur], pb, hipMemcpyDeviceToDevice,
                                               c->stream), "state save"))
        return s;
    if (cge_status s = check(c, hipMemcpyAsync(d + coff, c->carry, cb, hipMemcpyDeviceToDevice,
                                               c->stream), "state save"))
        return s;
    if (!seal) return CGE_OK;
    Trailer* t = reinterpret_cast<Trailer*>(d + state_trailer_offset(&c->p));
    hipLaunchKernelGGL(k_trailer_head, dim3(1), dim3(64), 0, c->stream, t, kStateMagic,
                       fingerprint(&c->p), (uint64_t)(pb + cb));
    return check(c, launch_checksum(d, pb, d + coff, cb,
                                    reinterpret_cast<unsigned long long*>(&t->checksum),
                                    c->stream),
                 "state seal");
}

// Load a saved state into the current buffers; with verify, check its trailer first (this
// synchronises the stream) and leave the state untouched when it fails.
cge_status load_state(cge_ctx* c, const void* src, bool verify) {
    const size_t pb = cge_population_bytes(&c->p), cb = carry_bytes(&c->p);
    const char* s0 = static_cast<const char*>(src);
    const size_t coff = state_carry_offset(&c->p);
    if (verify) {
        // the checksum is summed into a cleared trailer in the context's scratch
        Trailer* ck = reinterpret_cast<Trailer*>(c->ck);
        unsigned long long* sum = reinterpret_cast<unsigned long long*>(&ck->checksum);
        hipLaunchKernelGGL(k_trailer_head, dim3(1), dim3(64), 0, c->stream, ck, 0ull, 0ull, 0ull);
        if (cge_status s = check(c, launch_checksum(s0, pb, s0 + coff, cb, sum, c->stream),
                                 "state check"))
            return s;
        uint64_t got = 0;
        Trailer t{};
        if (cge_status s = check(c, hipMemcpyAsync(&got, sum, sizeof(got), hipMemcpyDeviceToHost,
                                                   c->stream), "state check"))
            return s;
        if (cge_status s = check(c, hipMemcpyAsync(&t, s0 + state_trailer_offset(&c->p),
                                                   sizeof(t), hipMemcpyDeviceToHost, c->stream),
                                 "state check"))
            return s;
        if (cge_status s = check(c, hipStreamSynchronize(c->stream), "state check")) return s;
        if (t.magic != kStateMagic)
            return fail(c, CGE_ECHECKPOINT, "not a saved state (no trailer)");
        if (t.fingerprint != fingerprint(&c->p) || t.bytes != pb + cb)
            return fail(c, CGE_ECHECKPOINT, "saved state belongs to other parameters");
        if (t.checksum != got)
            return fail(c, CGE_ECHECKPOINT, "saved state corrupted (checksum mismatch)");
    }
    if (cge_status s = check(c, hipMemcpyAsync(c->pop[c->cur], s0, pb, hipMemcpyDeviceToDevice,
                                               c->stream), "state load"))
        return s;
    return check(c, hipMemcpyAsync(c->carry, s0 + coff, cb, hipMemcpyDeviceToDevice, c->stream),
                 "state load");
}

// The same check on a snapshot in host memory.
cge_status verify_state_host(const cge_params* p, const void* snapshot) {
    const size_t pb = cge_population_bytes(p), cb = carry_bytes(p);
    const unsigned char* s0 = static_cast<const unsigned char*>(snapshot);
    Trailer t;
    std::memcpy(&t, s0 + state_trailer_offset(p), sizeof(t));
    if (t.magic != kStateMagic || t.fingerprint != fingerprint(p) || t.bytes != pb + cb)
        return CGE_ECHECKPOINT;
    const unsigned char* a = s0;
    const unsigned char* b = s0 + state_carry_offset(p);
    const size_t na = (pb + 7) / 8, nw = na + (cb + 7) / 8;
    uint64_t sum = 0;
    for (size_t i = 0; i < nw; ++i) {
        const unsigned char* base = i < na ? a : b;
        const size_t j = i < na ? i : i - na, len = i < na ? pb : cb;
        uint64_t w = 0;
        std::memcpy(&w, base + 8 * j, 8 * j + 8 <= len ? 8 : len - 8 * j);  // little-endian host
        sum += mix64(w ^ (i * kWordKey));
    }
    return sum == t.checksum ? CGE_OK : CGE_ECHECKPOINT;
}

}  // namespace cge
