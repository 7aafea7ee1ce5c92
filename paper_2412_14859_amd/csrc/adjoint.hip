// Adjoint of the step (reverse mode), for periodic domains and the site rules GRAD_GT (sites
// held at those of the forward run) and SOFT.
//
// Notation: the state of step n is the pre-sink encoded populations (ft_i, dd_i) of every node
// plus the carried site data.  The adjoint of a state is lambda = dL/d(ft, dd).  Because the
// colour differences enter the step only through their sum (the phase field) and the phase
// field's dependence on rho adds the same term to every colour-blind direction, lambda of a
// node is kept as Q values mu'_i plus two scalars (a, b):
//     dL/dft_i = mu'_i + a,    dL/ddd_i = b    (all i).
// At unit relaxation times BGK returns the equilibrium, so the step depends on the old
// populations only through the post-sink moments (rho, j) and mu'_i = p0 + c_i . dj: the
// adjoint of a node is then D + 3 numbers, and the reverse step needs the forward's phase
// field and moments only (kept by the split step during the recomputation), not its
// populations.
//
// One reverse step n (state S_n, adjoint of S_{n+1} given):
//   local   per node: gather the adjoint of the post-collision values from x + c_i (reverse
//           of the pull), recompute the forward intermediates, and apply the transposed
//           Jacobian of collision, perturbation and recolouring (Eqs. collision, feq,
//           perturb, recolor); writes mu' (or p0, dj), the local dL/drho^N, rho, dL/dF;
//   gather  per node: dL/drho^N += sum_i 3 W_i c_i . dL/dF(x - c_i) (the transposed
//           gradient stencil), giving (a, b); the sink s = m phi / Sbar enters as
//           dd_0 -= 2 s, so dL/ds = -2 b, hence dL/dphi(x, n) = -2 b m / Sbar; for the
//           soft rule also dL/dm, which flows into dL/d||F_{n-1}|| and dL/dGamma.
// The forward states of a segment of K steps are recomputed from the segment's checkpoint.
#include <vector>

#include "internal.hpp"
#include "node.hpp"

namespace cge {

// adjoint workspace (doubles): mu[2][nmu][N], ab[2][2][N], aF[2][N], loc[2][N], lamF[3][N],
// then one gamma partial per block of the node grid; nmu = Q, or 4 (p0, dj) at unit tau
struct AdjWork {
    double *mu[2], *ab[2], *aF[2], *loc, *lamF, *gpart;
};

// Index 1 of mu, ab, aF is the input of a reverse step (adjoint of the later state) and
// index 0 its result; the two halves of the buffer swap roles with the parity of the step.
static AdjWork adj_work(const cge_ctx* c, void* base, int parity, int nmu) {
    const long long N = c->g.N;
    double* p = static_cast<double*>(base);
    AdjWork w;
    w.mu[parity] = p;
    w.mu[1 - parity] = p + nmu * N;
    p += 2 * (long long)c->Q * N;  // room for the general layout
    w.ab[parity] = p;
    w.ab[1 - parity] = p + 2 * N;
    p += 4 * N;
    w.aF[parity] = p;
    w.aF[1 - parity] = p + N;
    p += 2 * N;
    w.loc = p;
    p += 2 * N;
    w.lamF = p;
    p += 3 * N;
    w.gpart = p;
    return w;
}

size_t adjoint_bytes(const cge_params* pr) {
    const long long N = (long long)pr->nx * pr->ny * pr->nz;
    const long long Q = pr->lattice;
    const Geo g{pr->nx, pr->ny, pr->nz, 0, N};
    const dim3 gr = node_grid(g);
    const long long nblk = (long long)gr.x * gr.y * gr.z;
    return (size_t)(2 * Q * N + 4 * N + 2 * N + 2 * N + 3 * N + nblk) * sizeof(double);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static bool unit_tau(const cge_params* p) { return p->tau[0] == 1.0 && p->tau[1] == 1.0; }

// Slot of one recomputed step at unit tau: post-sink rho^N and the moment record (both
// double next to FP64 populations, float otherwise), the carried site data.
struct UnitSlot {
    size_t rhoN, mom, carry, bytes;
};
static UnitSlot unit_slot(const cge_params* p) {
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    UnitSlot s;
    s.rhoN = 0;
    s.mom = align256(N * (p->precision == CGE_FP64 ? 8 : 4));
    s.carry = s.mom + align256(split_scratch_bytes(p));
    s.bytes = s.carry + align256(carry_bytes(p));
    return s;
}

// Seed: lambda of S_T from dL/drho^N_T and dL/drho_T (either may be absent), with
// rho = rho_ref + sum ft and rho^N = sum dd / rho (pre-sink):
//     dL/dft_i = dL/drho - dL/drho^N rho^N / rho,    dL/ddd_i = dL/drho^N / rho.
template <int Q, typename S, typename M, int NMU, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_adj_seed(const S* __restrict__ src,
                                                    const uint8_t* __restrict__ flags,
                                                    const double* __restrict__ g_rhoN,
                                                    const double* __restrict__ g_rho,
                                                    double* __restrict__ mu, double* __restrict__ ab,
                                                    double* __restrict__ aF, Geo g, Phys<M> P) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (WALLS && flags[n]) {  // a solid node has no state and no adjoint; loss seeds there are ignored
#pragma unroll
        for (int i = 0; i < NMU; ++i) mu[(long long)i * g.N + n] = 0.0;
        if (NMU != 4) ab[n] = 0.0;
        ab[g.N + n] = 0.0;
        aF[n] = 0.0;
        return;
    }
    const Nb b = wrap(g, x, y, z);
    M ft[Q], dd[Q], j[3], drho, dsum;
    pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
    moments<Q>(ft, dd, drho, dsum, j);
    const double rho = static_cast<double>(P.rho_ref + drho);
    const double rN = static_cast<double>(dsum) / rho;
    const double gr = g_rhoN ? g_rhoN[n] : 0.0;
    const double a = (g_rho ? g_rho[n] : 0.0) - gr * rN / rho;
#pragma unroll
    for (int i = 0; i < NMU; ++i) mu[(long long)i * g.N + n] = 0.0;
    if (NMU == 4) mu[n] = a;  // unit layout: q0 = p0 + a
    else ab[n] = a;
    ab[g.N + n] = gr / rho;
    aF[n] = 0.0;
}

// Transposed Jacobian of equilibrium + BGK, perturbation and recolouring at one node, all in
// FP64.  Inputs: post-sink rho, rho^N, u, the colour gradient F, the adjoint aF1n of the
// carried ||F|| (soft rule), in(i, mus, etas) -> adjoint of this node's outputs ft*_i, dd*_i,
// and (general tau only) fpop(i) -> the pulled total population f_i.  Outputs: the local
// dL/drho^N, dL/drho, dL/dj, dL/dF; for general tau also xi(i, v) with v the direct part
// (1 - 1/tau) dL/df''_i of dL/dft_i.
template <int Q, bool UNIT, class In, class Fpop, class Xi>
__device__ __forceinline__ void adj_node(const Phys<double>& P, double rho, double rN,
                                         const double (&u)[3], const double (&F)[3], double aF1n,
                                         In in, Fpop fpop, Xi xi, double& drN_o, double& drho_o,
                                         double (&dj_o)[3], double (&lamF_o)[3]) {
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double pr = 0.5 * (1.0 + rN), pb = 0.5 * (1.0 - rN);
    const double om = UNIT ? 1.0 : pr * P.omega_r + pb * P.omega_b;
    const double abar = pr * P.alpha_r + pb * P.alpha_b;
    const double F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    const double Fn = F2 > 0.0 ? sqrt(F2) : 0.0;
    const double iFc = F2 > 0.0 ? 1.0 / Fn : 0.0;  // d||F||/dF = F iFc (the carried ||F||)
    // cos(theta) and the perturbation are cut where F.F <= kF2Cut (as in the forward step)
    const bool hg = F2 > kF2Cut;
    const double Fp = hg ? Fn : 0.0;
    const double iF = hg ? iFc : 0.0;
    const double fade = recolor_fade(Fn, P.inv_fade);
    const double dfade = recolor_fade_slope(Fn, P.inv_fade);
    const double kp = 2.25 * P.sigma * om;
    const double sep = 0.5 * P.beta * (1.0 - rN * rN) * rho;

    double dsep = 0.0, dab = 0.0, dkp = 0.0, dom = 0.0, drho_p = 0.0, drN = 0.0;
    double du[3] = {0.0, 0.0, 0.0}, dF[3] = {0.0, 0.0, 0.0}, sF = 0.0;  // dF += sF * F
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cx = Lat<Q>::cx[i], cy = Lat<Q>::cy[i], cz = Lat<Q>::cz[i];
        const double A = restA<Q>(i), B = restB<Q>(i), W = weight<Q>(i);
        const double cu = cx * u[0] + cy * u[1] + cz * u[2];
        const double Fc = cx * F[0] + cy * F[1] + cz * F[2];
        const double t = A + B * abar;
        const double feq = rho * (t + W * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        const double Pq = W * Fc * Fc * iF - pertC<Q>(i) * Fp;
        double f2, f = 0.0;
        if constexpr (UNIT) {
            f2 = feq + kp * Pq;
        } else {
            f = fpop(i);
            f2 = f - om * (f - feq) + kp * Pq;
        }
        const double il = inv_len<Q>(i);
        const double cosf = Fc * iF * fade * il;
        double mus, etas;
        in(i, mus, etas);
        // dd* = rN f2 + sep cosf t ; ft* = f2 - tref
        const double x2 = mus + rN * etas;
        drN += f2 * etas;
        dsep += etas * cosf * t;
        dab += etas * sep * cosf * B;
        // d(Fc fade / |F|)/dF = fade (c/|F| - Fc F/|F|^3) + dfade (Fc/|F|) F/|F|
        const double q = etas * sep * t * il;
        dF[0] += q * fade * iF * cx;
        dF[1] += q * fade * iF * cy;
        dF[2] += q * fade * iF * cz;
        sF += q * Fc * (dfade * iF * iF - fade * iF * iF * iF);
        // f2 = f1 + kp Pq, Pq = W Fc^2/|F| - C |F|
        const double pv = x2 * kp * 2.0 * W * Fc * iF;
        dF[0] += pv * cx;
        dF[1] += pv * cy;
        dF[2] += pv * cz;
        sF += x2 * kp * (-W * Fc * Fc * iF * iF * iF - pertC<Q>(i) * iF);
        // f1 = f - om (f - feq)
        if constexpr (!UNIT) {
            dkp += x2 * Pq;
            dom += x2 * (feq - f);
            xi(i, (1.0 - om) * x2);
        }
        const double dfeq = om * x2;
        drho_p += dfeq * feq / rho;
        dab += dfeq * rho * B;
        const double g3 = dfeq * rho * W * (3.0 + 9.0 * cu);
        du[0] += g3 * cx - dfeq * rho * W * 3.0 * u[0];
        du[1] += g3 * cy - dfeq * rho * W * 3.0 * u[1];
        du[2] += g3 * cz - dfeq * rho * W * 3.0 * u[2];
    }
    // om and abar depend on rN through pr = (1 + rN)/2 (om is constant at unit tau)
    if constexpr (!UNIT) {
        dom += 2.25 * P.sigma * dkp;
        drN += 0.5 * (P.omega_r - P.omega_b) * dom;
    }
    drN += 0.5 * (P.alpha_r - P.alpha_b) * dab;
    // sep = beta (1 - rN^2) rho / 2
    drN += dsep * (-P.beta * rN * rho);
    drho_p += dsep * 0.5 * P.beta * (1.0 - rN * rN);
    // u = j / rho
    dj_o[0] = du[0] / rho;
    dj_o[1] = du[1] / rho;
    dj_o[2] = du[2] / rho;
    drho_p -= (du[0] * u[0] + du[1] * u[1] + du[2] * u[2]) / rho;
    drN_o = drN;
    drho_o = drho_p;
    // the carried ||F_n|| feeds the next step's soft site weight
    const double aFn = aF1n * iFc;
    lamF_o[0] = dF[0] + (sF + aFn) * F[0];
    lamF_o[1] = dF[1] + (sF + aFn) * F[1];
    lamF_o[2] = dF[2] + (sF + aFn) * F[2];
}

// The same transposed Jacobian at unit relaxation times (1/tau = 1 everywhere), arranged by
// weight class k (rest, axis, diagonal).  Every accumulation above is linear in the inputs
// (mus_i, etas_i) with coefficients that depend on the direction only through its class and
// through c_i.u and c_i.F, so each direction adds into a few per-class sums
//     X0 = sum x2,  E1 = sum etas Fc,  EV = sum etas c,  XV = sum x2 Fc c,  X2 = sum x2 Fc^2,
//     XC = sum x2 (3 + 9 cu) c        (x2 = mus + rho^N etas, Fc = c.F, cu = c.u)
// and the class coefficients are applied once per node.  Same outputs as adj_node<Q, true>.
template <int Q, class In>
__device__ __forceinline__ void adj_node_unit(const Phys<double>& P, double rho, double rN,
                                              const double (&u)[3], const double (&F)[3],
                                              double aF1n, In in, double& drN_o, double& drho_o,
                                              double (&dj_o)[3], double (&lamF_o)[3]) {
    constexpr int D = Lat<Q>::D;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double pr = 0.5 * (1.0 + rN), pb = 0.5 * (1.0 - rN);
    const double abar = pr * P.alpha_r + pb * P.alpha_b;
    const double F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    const double Fn = F2 > 0.0 ? sqrt(F2) : 0.0;
    const double iFc = F2 > 0.0 ? 1.0 / Fn : 0.0;
    const bool hg = F2 > kF2Cut;
    const double Fp = hg ? Fn : 0.0;
    const double iF = hg ? iFc : 0.0;
    const double fade = recolor_fade(Fn, P.inv_fade);
    const double dfade = recolor_fade_slope(Fn, P.inv_fade);
    const double kp = 2.25 * P.sigma;
    const double sep = 0.5 * P.beta * (1.0 - rN * rN) * rho;
    // class constants: k = 0 rest, 1 axis, 2 diagonal
    constexpr int i1 = 1, i2 = Q == 9 ? 5 : 7;
    double t[3], base[3], wr[3], pf[3], kc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = k == 0 ? 0 : (k == 1 ? i1 : i2);
        const double W = weight<Q>(i);
        t[k] = restA<Q>(i) + restB<Q>(i) * abar;
        wr[k] = rho * W;
        base[k] = rho * t[k] - 1.5 * wr[k] * uu;
        pf[k] = kp * W * iF;
        kc[k] = kp * pertC<Q>(i) * Fp;
    }
    double drN = 0.0, Sxf = 0.0;
    double X0[3] = {0.0, 0.0, 0.0}, E1[3] = {0.0, 0.0, 0.0}, X2[3] = {0.0, 0.0, 0.0};
    double EV[3][3] = {}, XV[3][3] = {}, XC[3][3] = {};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int k = norm2<Q>(i);
        const int c[3] = {Lat<Q>::cx[i], Lat<Q>::cy[i], Lat<Q>::cz[i]};
        double mus, etas;
        in(i, mus, etas);
        const double x2 = mus + rN * etas;
        X0[k] += x2;
        if (k == 0) {
            const double feq = base[0];
            drN += (feq - kc[0]) * etas;
            Sxf += x2 * feq;
            continue;
        }
        double cu = 0.0, Fc = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (c[a]) {
                cu += c[a] * u[a];
                Fc += c[a] * F[a];
            }
        const double feq = base[k] + wr[k] * cu * (3.0 + 4.5 * cu);
        drN += (feq + pf[k] * Fc * Fc - kc[k]) * etas;
        Sxf += x2 * feq;
        E1[k] += etas * Fc;
        const double xf = x2 * Fc;
        X2[k] += xf * Fc;
        const double xc = x2 * (3.0 + 9.0 * cu);
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (c[a]) {
                EV[k][a] += c[a] * etas;
                XV[k][a] += c[a] * xf;
                XC[k][a] += c[a] * xc;
            }
    }
    // class coefficients
    double dsep = 0.0, dab = 0.0, sF = 0.0, dF[3] = {0.0, 0.0, 0.0}, du[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = k == 0 ? 0 : (k == 1 ? i1 : i2);
        const double il = inv_len<Q>(i), B = restB<Q>(i), C = pertC<Q>(i);
        const double cw = iF * fade * il;
        dsep += cw * t[k] * E1[k];
        dab += sep * B * cw * E1[k] + rho * B * X0[k];
        sF += sep * t[k] * il * (dfade * iF * iF - fade * iF * iF * iF) * E1[k] -
              pf[k] * iF * iF * X2[k] - kp * C * iF * X0[k];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            dF[a] += sep * t[k] * cw * EV[k][a] + 2.0 * pf[k] * XV[k][a];
            du[a] += wr[k] * (XC[k][a] - 3.0 * u[a] * X0[k]);
        }
    }
    double drho_p = Sxf / rho;
    drN += 0.5 * (P.alpha_r - P.alpha_b) * dab;
    drN += dsep * (-P.beta * rN * rho);
    drho_p += dsep * 0.5 * P.beta * (1.0 - rN * rN);
    dj_o[0] = du[0] / rho;
    dj_o[1] = du[1] / rho;
    dj_o[2] = du[2] / rho;
    drho_p -= (du[0] * u[0] + du[1] * u[1] + du[2] * u[2]) / rho;
    drN_o = drN;
    drho_o = drho_p;
    const double aFn = aF1n * iFc;
    lamF_o[0] = dF[0] + (sF + aFn) * F[0];
    lamF_o[1] = dF[1] + (sF + aFn) * F[1];
    lamF_o[2] = dF[2] + (sF + aFn) * F[2];
}

// General relaxation times: recompute from the stored populations.
template <int Q, typename S, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_adj_local(
    const S* __restrict__ src, const uint8_t* __restrict__ flags, const MomT<S>* __restrict__ rhoNf,
    const double* __restrict__ mu1, const double* __restrict__ ab1,
    const double* __restrict__ aF1, double* __restrict__ mu0, double* __restrict__ loc,
    double* __restrict__ lamF, Geo g, Phys<double> P) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (WALLS && flags[n]) {
#pragma unroll
        for (int i = 0; i < Q; ++i) mu0[(long long)i * g.N + n] = 0.0;
        loc[n] = 0.0;
        loc[g.N + n] = 1.0;
        lamF[n] = lamF[g.N + n] = lamF[2 * g.N + n] = 0.0;
        return;
    }
    const Nb nb = wrap(g, x, y, z);
    M ftm[Q], ddm[Q], jm[3], drhom, dsumm;
    pull<Q, WALLS>(src, flags, g, nb, x, y, z, n, ftm, ddm);
    moments<Q>(ftm, ddm, drhom, dsumm, jm);
    const double rho = P.rho_ref + static_cast<double>(drhom);
    const double rN = static_cast<double>(rhoNf[n]);
    const double u[3] = {static_cast<double>(jm[0]) / rho, static_cast<double>(jm[1]) / rho,
                         static_cast<double>(jm[2]) / rho};
    double F[3];
    gradient<Q>(rhoNf, g, nb, x, y, z, F);
    double xi[Q];
    double drN, drho, dj[3], lf[3];
    adj_node<Q, false>(
        P, rho, rN, u, F, aF1[n],
        [&](int i, double& mus, double& etas) {
            // f*_i(x) is pulled by x + c_i, or bounced back into x as direction opp(i)
            const long long xn = shifted<Q, 1>(g, nb, x, y, z, i);
            if (WALLS && flags[xn]) {
                mus = mu1[(long long)Lat<Q>::opp[i] * g.N + n] + ab1[n];
                etas = ab1[g.N + n];
            } else {
                mus = mu1[(long long)i * g.N + xn] + ab1[xn];
                etas = ab1[g.N + xn];
            }
        },
        [&](int i) {
            return static_cast<double>(ftm[i]) +
                   P.rho_ref * (restA<Q>(i) + restB<Q>(i) * P.alpha_ref);
        },
        [&](int i, double v) { xi[i] = v; }, drN, drho, dj, lf);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        mu0[(long long)i * g.N + n] = xi[i] + drho + Lat<Q>::cx[i] * dj[0] +
                                      Lat<Q>::cy[i] * dj[1] + Lat<Q>::cz[i] * dj[2];
    loc[n] = drN;
    loc[g.N + n] = rho;
    lamF[n] = lf[0];
    lamF[g.N + n] = lf[1];
    lamF[2 * g.N + n] = lf[2];
}

// Unit relaxation times: the forward's phase field and moments of this step are given; the
// adjoint of a node is (q0, dj, b) with dL/dft_i = q0 + c_i . dj (q0 = p0 + a) and dL/ddd_i = b.
// One block is one x-row segment, so the neighbours' row and plane offsets are uniform.
template <int Q, typename S, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_adj_local_unit(
    const uint8_t* __restrict__ flags, const MomT<S>* __restrict__ rhoNf,
    const MomT<S>* __restrict__ mom,
    const double* __restrict__ mu1,
    const double* __restrict__ ab1, const double* __restrict__ aF1, double* __restrict__ mu0,
    double* __restrict__ loc, double* __restrict__ lamF, Geo g, Phys<double> P) {
    int x, y, z;
    long long n;
    const bool valid = node_xyz(g, x, y, z, n);
    const RowOff r = row_offsets<char>(g, x < g.nx ? x : 0);  // element offsets
    if (!valid) return;
    if (WALLS && flags[n]) {
        mu0[n] = mu0[g.N + n] = mu0[2 * g.N + n] = 0.0;
        if (Lat<Q>::D == 3) mu0[3 * g.N + n] = 0.0;
        loc[n] = 0.0;
        loc[g.N + n] = 1.0;
        lamF[n] = lamF[g.N + n] = 0.0;
        if (Lat<Q>::D == 3) lamF[2 * g.N + n] = 0.0;
        return;
    }
    const double rho = P.rho_ref + static_cast<double>(static_cast<M>(mom[n]));
    const double rN = static_cast<double>(rhoNf[n]);
    const double ir = 1.0 / rho;
    const double u[3] = {static_cast<double>(static_cast<M>(mom[g.N + n])) * ir,
                         static_cast<double>(static_cast<M>(mom[2 * g.N + n])) * ir,
                         static_cast<double>(static_cast<M>(mom[3 * g.N + n])) * ir};
    double F[3] = {0.0, 0.0, 0.0};  // F = 3 sum_i W_i rho^N(x + c_i) c_i
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const long long m = r.yrow[1 + Lat<Q>::cy[i]] + r.zpl[1 + Lat<Q>::cz[i]] +
                            r.xo[1 + Lat<Q>::cx[i]];
        const double v = weight<Q>(i) * static_cast<double>(rhoNf[m]);
        if (Lat<Q>::cx[i]) F[0] += Lat<Q>::cx[i] * v;
        if (Lat<Q>::cy[i]) F[1] += Lat<Q>::cy[i] * v;
        if (Lat<Q>::cz[i]) F[2] += Lat<Q>::cz[i] * v;
    }
    F[0] *= 3.0;
    F[1] *= 3.0;
    F[2] *= 3.0;
    double drN, drho, dj[3], lf[3];
    adj_node_unit<Q>(
        P, rho, rN, u, F, aF1[n],
        [&](int i, double& mus, double& etas) {
            long long xn = r.yrow[1 + Lat<Q>::cy[i]] + r.zpl[1 + Lat<Q>::cz[i]] +
                           r.xo[1 + Lat<Q>::cx[i]];
            // pulled by x + c_i as direction i, or bounced back into x as direction opp(i),
            // whose adjoint is q0(x) + c_opp(i) . dj(x) = q0(x) - c_i . dj(x)
            const double sgn = (WALLS && flags[xn]) ? -1.0 : 1.0;
            if (WALLS && flags[xn]) xn = n;
            double m = mu1[xn];
            if (Lat<Q>::cx[i]) m += sgn * Lat<Q>::cx[i] * mu1[g.N + xn];
            if (Lat<Q>::cy[i]) m += sgn * Lat<Q>::cy[i] * mu1[2 * g.N + xn];
            if (Lat<Q>::cz[i]) m += sgn * Lat<Q>::cz[i] * mu1[3 * g.N + xn];
            mus = m;
            etas = ab1[g.N + xn];
        },
        drN, drho, dj, lf);
    mu0[n] = drho;
    mu0[g.N + n] = dj[0];
    mu0[2 * g.N + n] = dj[1];
    if (Lat<Q>::D == 3) mu0[3 * g.N + n] = dj[2];
    loc[n] = drN;
    loc[g.N + n] = rho;
    lamF[n] = lf[0];
    lamF[g.N + n] = lf[1];
    if (Lat<Q>::D == 3) lamF[2 * g.N + n] = lf[2];
}

// Adjoint of the neutral-wetting value at solid nodes: the solid node s's rho^N enters the
// gradient of its fluid neighbours, so dL/drho^N(s) = sum_i 3 W_i c_i . dL/dF(s - c_i); its
// value is sum_k W_k rho^N(s + c_k) / den_s over fluid neighbours, so the gather adds
// W_k dL/drho^N(s) / den_s to fluid node s + c_k.  Writes dL/drho^N(s) / den_s into loc[s].
template <int Q>
__global__ __launch_bounds__(kTPBX) void k_adj_wet(const uint8_t* __restrict__ flags,
                                                   double* __restrict__ loc,
                                                   const double* __restrict__ lamF, Geo g) {
    int x, y, z;
    long long n;
    const bool valid = node_xyz(g, x, y, z, n);
    const RowOff r = row_offsets<char>(g, x < g.nx ? x : 0);  // element offsets
    if (!valid || !flags[n]) return;
    double G = 0.0, den = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const long long m = r.yrow[1 - Lat<Q>::cy[i]] + r.zpl[1 - Lat<Q>::cz[i]] +
                            r.xo[1 - Lat<Q>::cx[i]];  // s - c_i
        double v = 0.0;
        if (Lat<Q>::cx[i]) v += Lat<Q>::cx[i] * lamF[m];
        if (Lat<Q>::cy[i]) v += Lat<Q>::cy[i] * lamF[g.N + m];
        if (Lat<Q>::cz[i]) v += Lat<Q>::cz[i] * lamF[2 * g.N + m];
        G += 3.0 * weight<Q>(i) * v;
        const long long k = r.yrow[1 + Lat<Q>::cy[i]] + r.zpl[1 + Lat<Q>::cz[i]] +
                            r.xo[1 + Lat<Q>::cx[i]];  // s + c_i
        if (!flags[k]) den += weight<Q>(i);
    }
    loc[n] = den > 0.0 ? G / den : 0.0;
}

// Transposed gradient stencil, assembly of (a, b), and the sink adjoint.
// At unit tau the result a is folded into q0 = p0 + a (mu0, written by the local kernel).
template <int Q, typename S, typename M, bool UNIT, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_adj_gather(
    const uint8_t* __restrict__ flags, const void* __restrict__ carry,
    const void* __restrict__ phi_field,
    const MomT<S>* __restrict__ rhoNf,
    const double* __restrict__ loc, const double* __restrict__ lamF,
    double* __restrict__ q0, double* __restrict__ ab0, double* __restrict__ aF0,
    double* __restrict__ grad_phi, double* __restrict__ grad_phi_t, double* __restrict__ gpart,
    Geo g, Phys<double> P) {
    int x, y, z;
    long long n;
    const bool valid = node_xyz(g, x, y, z, n);
    const RowOff r = row_offsets<char>(g, x < g.nx ? x : 0);  // element offsets
    double gg = 0.0;
    if (valid && WALLS && flags[n]) {  // solid: no sink, no adjoint state
        if constexpr (!UNIT) ab0[n] = 0.0;
        ab0[g.N + n] = 0.0;
        aF0[n] = 0.0;
        if (grad_phi_t) grad_phi_t[n] = 0.0;
    } else if (valid) {
        double G = loc[n];
#pragma unroll
        for (int i = 1; i < Q; ++i) {  // F(x - c_i) contains 3 W_i c_i rho^N(x)
            const long long m = r.yrow[1 - Lat<Q>::cy[i]] + r.zpl[1 - Lat<Q>::cz[i]] +
                                r.xo[1 - Lat<Q>::cx[i]];
            double v = 0.0;
            if (Lat<Q>::cx[i]) v += Lat<Q>::cx[i] * lamF[m];
            if (Lat<Q>::cy[i]) v += Lat<Q>::cy[i] * lamF[g.N + m];
            if (Lat<Q>::cz[i]) v += Lat<Q>::cz[i] * lamF[2 * g.N + m];
            G += 3.0 * weight<Q>(i) * v;
            // the wetting value of a solid x - c_i is a mean that includes rho^N(x)
            if (WALLS && flags[m]) G += weight<Q>(i) * loc[m];
        }
        const double rho = loc[g.N + n];
        const double rN = static_cast<double>(rhoNf[n]);
        const double b = G / rho;
        if constexpr (UNIT) q0[n] += -G * rN / rho;
        else ab0[n] = -G * rN / rho;
        ab0[g.N + n] = b;
        const double dLds = -2.0 * b;
        const double w = site_weight<double>(P, carry, n, 1.0, 0.0);
        const double gphi = dLds * w * P.inv_sbar;
        grad_phi[n] += gphi;
        if (grad_phi_t) grad_phi_t[n] = gphi;
        if (P.site_rule == CGE_SITE_SOFT) {
            const double phi = node_phi<S, double>(P, phi_field, n);
            const double dLdw = dLds * phi * P.inv_sbar;
            const double sp = w * (1.0 - w) * P.inv_kappa;  // dw / d||F_{n-1}||
            aF0[n] = dLdw * sp;
            gg = -dLdw * sp;
        } else {
            aF0[n] = 0.0;
        }
    }
    const bool is_max[1] = {false};
    double v[1] = {gg}, out[1];
    block_reduce<1>(v, is_max, threadIdx.x, blockDim.x, out);
    if (threadIdx.x == 0) {
        const long long bid =
            blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
        gpart[bid] += out[0];
    }
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ p, long long n) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

static hipError_t zero(double* p, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// post-sink rho^N of a stored state (same arithmetic as the forward first pass, stored at
// the same precision)
template <int Q, typename S, typename M, bool WALLS>
__global__ __launch_bounds__(kTPBX) void k_phase_state(const S* __restrict__ src,
                                                       const uint8_t* __restrict__ flags,
                                                       const void* __restrict__ carry,
                                                       const void* __restrict__ phi_field,
                                                       MomT<S>* __restrict__ rhoN, Geo g,
                                                       Phys<M> P) {
    int x, y, z;
    long long n;
    if (!node_xyz(g, x, y, z, n)) return;
    if (WALLS && flags[n]) return;  // the wetting value follows (k_wet)
    const Nb b = wrap(g, x, y, z);
    M ft[Q], dd[Q], j[3], drho, dsum;
    pull<Q, WALLS>(src, flags, g, b, x, y, z, n, ft, dd);
    moments<Q>(ft, dd, drho, dsum, j);
    const M rho = P.rho_ref + drho;
    dsum -= M(2) * site_sink<S>(P, carry, phi_field, n, rho, dsum);
    rhoN[n] = static_cast<MomT<S>>(dsum / rho);
}

template <int Q, typename S, typename M, bool WALLS>
static cge_status seed_impl(cge_ctx* c, const double* g_rhoN, const double* g_rho, AdjWork w,
                            bool unit) {
    const dim3 gr = node_grid(c->g), bl = node_block(c->g);
    const S* src = static_cast<const S*>(c->pop[c->cur]);
    if (unit)
        hipLaunchKernelGGL((k_adj_seed<Q, S, M, 4, WALLS>), gr, bl, 0, c->stream, src, c->flags,
                           g_rhoN, g_rho, w.mu[1], w.ab[1], w.aF[1], c->g, phys<M>(c));
    else
        hipLaunchKernelGGL((k_adj_seed<Q, S, M, Q, WALLS>), gr, bl, 0, c->stream, src, c->flags,
                           g_rhoN, g_rho, w.mu[1], w.ab[1], w.aF[1], c->g, phys<M>(c));
    return check(c, hipGetLastError(), "adjoint seed");
}

// One reverse step, adjoint 1 -> 0.  General tau: from the stored state (pop, carry).  Unit
// tau: from the step's phase field, moments and carry (pop unused).  With solid nodes the
// phase field holds the wetting values there, as in the forward.
template <int Q, typename S, typename M, bool WALLS>
static cge_status rstep_impl(cge_ctx* c, const void* pop, const void* rhoN_in, const void* mom,
                             const void* carry, AdjWork w, double* grad_phi, double* grad_phi_t) {
    const Phys<double> P = phys<double>(c);
    const dim3 gr = node_grid(c->g), bl = node_block(c->g);
    if (pop) {
        MomT<S>* r = static_cast<MomT<S>*>(c->rhoN);
        hipLaunchKernelGGL((k_phase_state<Q, S, M, WALLS>), gr, bl, 0, c->stream,
                           static_cast<const S*>(pop), c->flags, carry, c->phi_field, r, c->g,
                           phys<M>(c));
        if (WALLS)
            hipLaunchKernelGGL((k_wet<Q, MomT<S>>), gr, bl, 0, c->stream, c->flags, r, c->g);
        hipLaunchKernelGGL((k_adj_local<Q, S, M, WALLS>), gr, bl, 0, c->stream,
                           static_cast<const S*>(pop), c->flags, r, w.mu[1], w.ab[1], w.aF[1],
                           w.mu[0], w.loc, w.lamF, c->g, P);
        if (WALLS)
            hipLaunchKernelGGL((k_adj_wet<Q>), gr, bl, 0, c->stream, c->flags, w.loc, w.lamF,
                               c->g);
        hipLaunchKernelGGL((k_adj_gather<Q, S, M, false, WALLS>), gr, bl, 0, c->stream, c->flags,
                           carry, c->phi_field, r, w.loc, w.lamF, w.mu[0], w.ab[0], w.aF[0],
                           grad_phi, grad_phi_t, w.gpart, c->g, P);
    } else {
        // rho^N as the split step stores it (the moment record's type)
        const MomT<S>* rhoN = static_cast<const MomT<S>*>(rhoN_in);
        hipLaunchKernelGGL((k_adj_local_unit<Q, S, M, WALLS>), gr, bl, 0, c->stream, c->flags,
                           rhoN, static_cast<const MomT<S>*>(mom), w.mu[1], w.ab[1], w.aF[1],
                           w.mu[0], w.loc, w.lamF, c->g, P);
        if (WALLS)
            hipLaunchKernelGGL((k_adj_wet<Q>), gr, bl, 0, c->stream, c->flags, w.loc, w.lamF,
                               c->g);
        hipLaunchKernelGGL((k_adj_gather<Q, S, M, true, WALLS>), gr, bl, 0, c->stream, c->flags,
                           carry, c->phi_field, rhoN, w.loc, w.lamF, w.mu[0], w.ab[0], w.aF[0],
                           grad_phi, grad_phi_t, w.gpart, c->g, P);
    }
    return check(c, hipGetLastError(), "adjoint step");
}

static cge_status adjoint_seed(cge_ctx* c, const double* g_rhoN, const double* g_rho,
                               void* work, int parity, bool unit) {
    AdjWork w = adj_work(c, work, parity, unit ? 4 : c->Q);
    CGE_DISPATCH(c, seed_impl, c, g_rhoN, g_rho, w, unit);
}

static cge_status adjoint_rstep(cge_ctx* c, const void* pop, const void* rhoN, const void* mom,
                                const void* carry, void* work, int parity, double* grad_phi,
                                double* grad_phi_t) {
    AdjWork w = adj_work(c, work, parity, pop ? c->Q : 4);
    CGE_DISPATCH(c, rstep_impl, c, pop, rhoN, mom, carry, w, grad_phi, grad_phi_t);
}

}  // namespace cge

using namespace cge;

extern "C" {

size_t cge_adjoint_bytes(const cge_params* p) {
    if (!cge_population_bytes(p)) return 0;
    return adjoint_bytes(p);
}

size_t cge_segment_bytes(const cge_params* p, int K) {
    if (!cge_population_bytes(p) || K < 1) return 0;
    const size_t slot = unit_tau(p) ? unit_slot(p).bytes : align256(cge_state_bytes(p));
    return (size_t)K * slot;
}

cge_status cge_forward_ckpt(cge_ctx* c, long long nsteps, int K, void* const* ckpt) {
    TraceRange trace_("cge_forward_ckpt");
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (nsteps < 1 || K < 1 || !ckpt) return fail(c, CGE_EINVAL, "nsteps >= 1, K >= 1, ckpt");
    if (c->hf_every > 0 || c->out_lo || c->out_hi)
        return fail(c, CGE_EUNSUPPORTED, "the adjoint supports neither the height flux nor outlets");
    // at unit tau the backward recomputes with the split step, so the forward uses it too and
    // the recomputed trajectory is the forward's bit for bit (with or without solid nodes)
    const bool split = unit_tau(&c->p);
    const long long nseg = (nsteps + K - 1) / K;
    for (long long j = 0; j <= nseg; ++j)
        if (!ckpt[j]) return fail(c, CGE_EINVAL, "NULL checkpoint buffer");
    for (long long n0 = 0, j = 0; n0 < nsteps; n0 += K, ++j) {
        if (cge_status s = cge_save_state(c, ckpt[j])) return s;
        const long long n = nsteps - n0 < K ? nsteps - n0 : K;
        if (cge_status s = split ? split_steps(c, n) : cge_step(c, n)) return s;
    }
    return cge_save_state(c, ckpt[nseg]);  // the final state seeds the backward
}

cge_status cge_backward(cge_ctx* c, long long nsteps, int K, void* const* ckpt, void* seg,
                        void* work, const double* dL_drhoN, const double* dL_drho,
                        double* grad_phi, double* grad_phi_t, double* grad_gamma) {
    TraceRange trace_("cge_backward");
    if (!c) return CGE_EINVAL;
    if (!c->bound) return fail(c, CGE_ESTATE, "cge_bind first");
    if (nsteps < 1 || K < 1 || !ckpt || !seg || !work || (!dL_drhoN && !dL_drho) || !grad_phi)
        return fail(c, CGE_EINVAL, "missing argument");
    if (c->hf_every > 0 || c->out_lo || c->out_hi)
        return fail(c, CGE_EUNSUPPORTED, "the adjoint supports neither the height flux nor outlets");
    if (c->p.site_rule == CGE_SITE_PHASE_LT)
        return fail(c, CGE_EUNSUPPORTED, "adjoint supports the gradient site rules only");
    const long long N = c->g.N;
    const bool unit = unit_tau(&c->p);
    const UnitSlot us = unit_slot(&c->p);
    const size_t sb = unit ? us.bytes : align256(cge_state_bytes(&c->p));
    // layout of a saved state: populations, then the carried site data at a 256-byte boundary
    const size_t carry_at = align256(cge_population_bytes(&c->p));
    const size_t cb = carry_bytes(&c->p);
    char* segb = static_cast<char*>(seg);
    // forward bookkeeping is restored after the recomputation
    const long long step0 = c->step;
    std::vector<char> acc_save((size_t)c->acc_len * (sizeof(double) + sizeof(long long)));
    if (cge_status s = check(c, hipMemcpyAsync(acc_save.data(), c->acc_sink,
                                               c->acc_len * sizeof(double),
                                               hipMemcpyDeviceToHost, c->stream), "acc save"))
        return s;
    if (cge_status s = check(c, hipMemcpyAsync(acc_save.data() + c->acc_len * sizeof(double),
                                               c->acc_sites, c->acc_len * sizeof(long long),
                                               hipMemcpyDeviceToHost, c->stream), "acc save"))
        return s;
    if (cge_status s = check(c, hipStreamSynchronize(c->stream), "sync")) return s;

    const dim3 gr = node_grid(c->g);
    const long long nblk = (long long)gr.x * gr.y * gr.z;
    AdjWork w0 = adj_work(c, work, 0, c->Q);
    if (zero(grad_phi, N, c->stream) != hipSuccess || zero(w0.gpart, nblk, c->stream) != hipSuccess)
        return fail(c, CGE_EDEVICE, "clearing gradients failed");
    // seed from the state after nsteps (the last checkpoint)
    const long long nseg = (nsteps + K - 1) / K;
    for (long long j = 0; j <= nseg; ++j)
        if (!ckpt[j]) return fail(c, CGE_EINVAL, "NULL checkpoint buffer");
    if (cge_status s = cge_load_state(c, ckpt[nseg])) return s;
    int parity = 0;
    if (cge_status s = adjoint_seed(c, dL_drhoN, dL_drho, work, parity, unit)) return s;
    for (long long j = nseg - 1; j >= 0; --j) {
        const long long n0 = j * K;
        const long long len = nsteps - n0 < K ? nsteps - n0 : K;
        TraceRange seg_trace_("adjoint segment (recompute, reverse steps)");
        if (cge_status s = cge_load_state(c, ckpt[j])) return s;
        c->step = step0 - nsteps + n0;  // the recomputed steps draw the same rounding keys
        if (unit) {
            // split steps keep each step's phase field, moments and incoming site data
            if (cge_status s = check(c, hipMemcpyAsync(segb + us.carry, c->carry, cb,
                                                       hipMemcpyDeviceToDevice, c->stream),
                                     "segment carry"))
                return s;
            for (long long t = 0; t < len; ++t) {
                char* sl = segb + t * sb;
                void* cout = t + 1 < len ? static_cast<void*>(sl + sb + us.carry)
                                         : static_cast<void*>(c->carry);
                if (cge_status s = split_step_into(c, sl + us.carry, cout, sl + us.rhoN,
                                                   sl + us.mom))
                    return s;
            }
        } else {
            for (long long t = 0; t < len; ++t) {  // states n0 .. n0 + len - 1
                if (cge_status s = save_state(c, segb + t * sb, false)) return s;
                if (t + 1 < len)
                    if (cge_status s = cge_step(c, 1)) return s;
            }
        }
        for (long long t = len - 1; t >= 0; --t) {
            double* gt = grad_phi_t ? grad_phi_t + (n0 + t) * N : nullptr;
            char* sl = segb + t * sb;
            const cge_status s =
                unit ? adjoint_rstep(c, nullptr, sl + us.rhoN, sl + us.mom, sl + us.carry, work,
                                     parity, grad_phi, gt)
                     : adjoint_rstep(c, sl, nullptr, nullptr, sl + carry_at, work, parity,
                                     grad_phi, gt);
            if (s) return s;
            parity = 1 - parity;
        }
    }
    // dL/dGamma: fixed-order sum of the per-block partials
    std::vector<double> gp((size_t)nblk);
    if (cge_status s = check(c, hipMemcpyAsync(gp.data(), w0.gpart, nblk * sizeof(double),
                                               hipMemcpyDeviceToHost, c->stream), "gamma copy"))
        return s;
    if (cge_status s = check(c, hipMemcpyAsync(c->acc_sink, acc_save.data(),
                                               c->acc_len * sizeof(double),
                                               hipMemcpyHostToDevice, c->stream), "acc restore"))
        return s;
    if (cge_status s = check(c, hipMemcpyAsync(c->acc_sites,
                                               acc_save.data() + c->acc_len * sizeof(double),
                                               c->acc_len * sizeof(long long),
                                               hipMemcpyHostToDevice, c->stream), "acc restore"))
        return s;
    // the context is left as the forward run left it: final state, step counter, bookkeeping
    if (cge_status s = cge_load_state(c, ckpt[nseg])) return s;
    if (cge_status s = check(c, hipStreamSynchronize(c->stream), "sync")) return s;
    c->step = step0;
    double gsum = 0.0;
    for (double v : gp) gsum += v;
    if (grad_gamma) *grad_gamma = gsum;
    return CGE_OK;
}

}  // extern "C"
