// Lattice constants of the HIP path (D2Q9, D3Q19) and the per-run physical constants.
//
// Rest weights of the alpha-equilibrium (Eq. feq): t_i(a) = A_i + B_i a with A_0 = 0,
// B_0 = 1 and A_i = -B_i = W_i / (1 - W_0) for i >= 1, so that t_i(W_0) = W_i and
// zeta (1 - W_0) = c_s^2 (Appendix A).  Perturbation constants (Eq. perturb):
// C_0 = c_s^2 - (1 - W_0), C_i = W_i for i >= 1, which give sum_i C_i = c_s^2 and
// sum_i C_i c_ia c_ib = c_s^2 delta_ab.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace cge {

template <int Q>
struct Lat;

template <>
struct Lat<9> {
    static constexpr int D = 2;
    static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
    static constexpr double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w2 = 1.0 / 36.0;
    static constexpr double zeta = 3.0 / 5.0;
};

template <>
struct Lat<19> {
    static constexpr int D = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr double w0 = 1.0 / 3.0, w1 = 1.0 / 18.0, w2 = 1.0 / 36.0;
    static constexpr double zeta = 1.0 / 2.0;
};

template <int Q>
__host__ __device__ constexpr int norm2(int i) {
    return Lat<Q>::cx[i] * Lat<Q>::cx[i] + Lat<Q>::cy[i] * Lat<Q>::cy[i] +
           Lat<Q>::cz[i] * Lat<Q>::cz[i];
}
template <int Q>
__host__ __device__ constexpr double weight(int i) {
    return norm2<Q>(i) == 0 ? Lat<Q>::w0 : (norm2<Q>(i) == 1 ? Lat<Q>::w1 : Lat<Q>::w2);
}
template <int Q>
__host__ __device__ constexpr double restA(int i) {
    return i == 0 ? 0.0 : weight<Q>(i) / (1.0 - Lat<Q>::w0);
}
template <int Q>
__host__ __device__ constexpr double restB(int i) {
    return i == 0 ? 1.0 : -restA<Q>(i);
}
template <int Q>
__host__ __device__ constexpr double pertC(int i) {
    return i == 0 ? 1.0 / 3.0 - (1.0 - Lat<Q>::w0) : weight<Q>(i);
}
// 1/|c_i| (0 for the rest direction, whose cos(theta) is taken as 0)
template <int Q>
__host__ __device__ constexpr double inv_len(int i) {
    return norm2<Q>(i) == 0 ? 0.0 : (norm2<Q>(i) == 1 ? 1.0 : 0.70710678118654752440);
}

// Physical constants of one run in the arithmetic type M.
template <typename M>
struct Phys {
    M rho_ref;        // codec shift: rho_ref * t_i(alpha_ref) is subtracted from f_i
    M alpha_ref;
    M alpha_r, alpha_b;
    M rho_in_r, rho_in_b;  // bulk densities of the two components
    M omega_r, omega_b;  // 1/tau_k
    M sigma, beta;
    M gamma;
    M phi;            // uniform flux
    M inv_sbar;
    M inv_kappa;      // soft site rule width
    M inv_fade;       // 1 / recolor_fade, or 0 when the optional cos(theta) fade is off
    int site_rule;    // 0 grad, 1 phase, 2 soft
};

// cos(theta_i) and the perturbation are 0/0 forms at F = 0 (Eqs. perturb, recolor): both are
// taken as 0 where F.F is at most this (their limit; the perturbation is O(||F||)).
constexpr double kF2Cut = 1e-24;

// Optional regularisation of the recolouring angle (off when inv_fade == 0): cos(theta_i) is
// multiplied by clamp(||F|| / w - 1, 0, 1) for the width w = 1 / inv_fade.
template <typename M>
__host__ __device__ __forceinline__ M recolor_fade(M Fn, M inv_fade) {
    if (!(inv_fade > M(0))) return M(1);
    const M g = Fn * inv_fade - M(1);
    return g < M(0) ? M(0) : (g > M(1) ? M(1) : g);
}
// its derivative with respect to ||F||
template <typename M>
__host__ __device__ __forceinline__ M recolor_fade_slope(M Fn, M inv_fade) {
    if (!(inv_fade > M(0))) return M(0);
    const M g = Fn * inv_fade - M(1);
    return (g > M(0) && g < M(1)) ? inv_fade : M(0);
}

// Store policy of the step kernels (Geo::nt): which of the arrays a pass writes for the next
// pass go out with the non-temporal cache policy (kNtPop populations, kNtMom the moment
// record between the two passes, kNtRec the post-collision records).  The kernels take their
// bit as a template argument (by_policy picks the instance at launch): given a run-time
// flag, the compiler merged the two stores of each branch into one plain store.
enum : int { kNtPop = 1, kNtMom = 2, kNtRec = 4 };

// f(std::true_type) where bit is set in policy, else f(std::false_type)
template <typename F>
inline void by_policy(int policy, int bit, F&& f) {
    if (policy & bit)
        f(std::true_type{});
    else
        f(std::false_type{});
}

struct Geo {
    int nx, ny, nz;
    int nt;  // store policy (kNt* bits), in the padding before N
    long long N;
};

}  // namespace cge
