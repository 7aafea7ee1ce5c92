/*
 * cg_oracle.c -- plain, slow FP64 CPU oracle for the two-component colour-gradient
 * lattice Boltzmann step with reaction-limited evaporation (Nath, Aouane, Harting,
 * "Reaction-limited evaporation for the color-gradient lattice Boltzmann model",
 * arXiv:2412.14859).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  The product path (the HIP library) shares no
 * code, header, table or helper with it.
 *
 * What it computes (Sec. II, method summary at the end of Sec. II.B), node by node, in
 * the paper's order, in IEEE double precision:
 *   1. sink per step  s(x) = phi(x) dt / (Sbar dx)                (Eq. relation, dx=dt=1)
 *   2. evaporation sites  ||F_{n-1}(x)|| > Gamma, using the colour gradient of the
 *      previous step (remark after the method summary)          (site criterion)
 *   3. rest-population exchange f0^r -= s, f0^b += s at sites    (Eq. exchange)
 *   4. colour-blind moments rho_k, rho, u, rho^N                  (Sec. II.A)
 *   5. colour gradient by the compact isotropic stencil           (Eq. cg + stencil)
 *      BGK collision with harmonic tau                            (Eq. collision)
 *      alpha-equilibrium                                          (Eq. feq)
 *      perturbation (surface tension)                             (Eq. perturb)
 *      recolouring                                                (Eq. recolor)
 *   6. streaming, periodic, with halfway bounce-back at solid nodes (Eq. Stream, Sec. III)
 *
 * Readings of points the paper leaves open (each is listed in the design notes):
 *   - A_i, B_i, C_i, zeta are deferred to Leclaire et al. (2017).  Rest weights
 *     t_i(alpha) = A_i + B_i alpha with A_0 = 0, B_0 = 1, A_i = -B_i = W_i/(1-W_0)
 *     (i >= 1), so that t_i(W_0) = W_i and zeta (1 - W_0) = c_s^2 as Appendix A needs.
 *     C_i = W_i (i >= 1), C_0 = c_s^2 - (1 - W_0): sum C_i = c_s^2 and
 *     sum C_i c_ia c_ib = c_s^2 delta_ab, which fixes the interfacial stress to sigma.
 *   - D2Q9 is built with the same constructions (the paper uses D3Q19 only).
 *   - The angle theta_i between F and c_i is undefined at F = 0: cos(theta_i) =
 *     F.c_i / (||F|| ||c_i||) (Eq. recolor) where F.F > 1e-24, and 0 otherwise; the
 *     perturbation (Eq. perturb), which vanishes continuously with ||F||, is cut at the same
 *     place.  cos(theta_0) = 0 for the rest direction.  An optional regularisation, off by
 *     default (recolor_fade = 0) and not part of the paper's model, multiplies cos(theta_i)
 *     by g(||F||) = clamp(||F|| / w - 1, 0, 1) for a width w = recolor_fade > 0: zero up to
 *     ||F|| = w, one from 2w.  It exists for small periodic boxes, where F vanishes by
 *     symmetry at mixed nodes between a drop and its images and its direction there is
 *     rounding noise.
 *   - Step 0 uses the gradient of the initial phase field as the "previous" gradient.
 *   - Site criterion is strict (>).  An alternative local rule |rho^N_pre| < Gamma
 *     (site_rule = 1) uses the current pre-sink phase field.  A soft rule (site_rule = 2)
 *     weights the sink by the logistic function of (||F_prev|| - Gamma)/kappa; it stands in
 *     for the threshold where derivatives with respect to Gamma are taken (sites counted
 *     where the weight exceeds 1/2).
 *   - Solid nodes carry no populations; for the gradient stencil a solid node takes the
 *     W-weighted mean of rho^N over its fluid neighbours (neutral wetting).
 *   - Blue recolouring uses F_br = -F_rb, i.e. cos(theta_br) = -cos(theta_rb).
 *   - No clamp of negative populations; they are only counted.
 *
 * Threads: with threads > 1 (ora_set_threads, OpenMP builds only) the loops over nodes that
 * are independent node by node (phase field, collision, streaming) run in parallel; the sink
 * loop, which adds up the bookkeeping, and every reduction stay sequential, so the results are
 * the same bits for any thread count.
 *
 * Storage: populations f[(k*Q + i)*N + n], k = 0 red (evaporating), k = 1 blue,
 * node n = x + nx*(y + ny*z).  The state between steps is the post-streaming,
 * pre-sink distribution.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_MAXQ 19

typedef struct {
    int Q, D;
    int c[ORA_MAXQ][3];
    double W[ORA_MAXQ];
    double A[ORA_MAXQ], B[ORA_MAXQ];
    double C[ORA_MAXQ];
    double cs2, zeta;
    int opp[ORA_MAXQ];
} ora_lattice;

typedef struct {
    int Q, nx, ny, nz;
    double rho_in[2], tau[2], sigma, beta;
    double phi, sbar, gamma;
    int site_rule; /* 0: ||F_prev|| > gamma (paper); 1: |rho^N_pre| < gamma;
                      2: soft weight 1 / (1 + exp(-(||F_prev|| - gamma) / kappa)) */
    double kappa;
    double recolor_fade; /* 0: Eq. recolor as printed; w > 0: cos(theta) faded out below 2w */
} ora_params;

typedef struct {
    long long step, n_sites, v_half, n_negative, site_steps;
    double mass_r, mass_b, sink_total, v_mass, perim_sites, perim_grad, max_u, p_in, p_out,
        max_rho_r;
} ora_obs;

typedef struct ora_ctx {
    ora_params p;
    ora_lattice L;
    long long N;
    double alpha[2];
    double *f, *fpost, *rhoN, *fmag, *phi_field;
    long long* nbr; /* nbr[i*N + n]: node n + c_i with periodic wrap */
    unsigned char *solid;
    long long step, site_steps;
    double sink_total;
    /* height-dependent flux (Eq. heated): active when hf_every > 0 */
    long long hf_every;
    double hf_phi, hf_K, hf_hs;
    /* pressure outlets for the blue component at the ends of the last axis (Sec. III, density
       contrast): out_lo, out_hi switch the planes at index 0 and the last index */
    int out_lo, out_hi;
    double out_rho;
    int threads; /* OpenMP threads of the per-node loops (1 = sequential) */
} ora_ctx;

/* ------------------------------------------------------------------ lattices */

static void lattice_fill_common(ora_lattice* L) {
    L->cs2 = 1.0 / 3.0;
    for (int i = 0; i < L->Q; ++i) {
        if (i == 0) {
            L->A[i] = 0.0;
            L->B[i] = 1.0;
            L->C[i] = L->cs2 - (1.0 - L->W[0]);
        } else {
            L->A[i] = L->W[i] / (1.0 - L->W[0]);
            L->B[i] = -L->A[i];
            L->C[i] = L->W[i];
        }
    }
    /* zeta from the second moment of the rest weights: sum_i A_i c_ix^2 */
    double z = 0.0;
    for (int i = 0; i < L->Q; ++i) z += L->A[i] * L->c[i][0] * L->c[i][0];
    L->zeta = z;
    for (int i = 0; i < L->Q; ++i) {
        for (int j = 0; j < L->Q; ++j) {
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
                L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
        }
    }
}

static void lattice_d2q9(ora_lattice* L) {
    static const int c[9][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    L->Q = 9;
    L->D = 2;
    for (int i = 0; i < 9; ++i) {
        for (int a = 0; a < 3; ++a) L->c[i][a] = c[i][a];
        int n2 = c[i][0] * c[i][0] + c[i][1] * c[i][1];
        L->W[i] = n2 == 0 ? 4.0 / 9.0 : (n2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    lattice_fill_common(L);
}

static void lattice_d3q19(ora_lattice* L) {
    static const int c[19][3] = {
        {0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
        {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
        {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    L->Q = 19;
    L->D = 3;
    for (int i = 0; i < 19; ++i) {
        for (int a = 0; a < 3; ++a) L->c[i][a] = c[i][a];
        int n2 = c[i][0] * c[i][0] + c[i][1] * c[i][1] + c[i][2] * c[i][2];
        L->W[i] = n2 == 0 ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    lattice_fill_common(L);
}

static int lattice_make(int Q, ora_lattice* L) {
    if (Q == 9) lattice_d2q9(L);
    else if (Q == 19) lattice_d3q19(L);
    else return -1;
    return 0;
}

/* Lattice tables for the pin tests: W, A, B, C (Q each), c (3Q), opp (Q), zeta. */
int ora_tables(int Q, double* W, double* A, double* B, double* C, int* c, int* opp,
               double* zeta) {
    ora_lattice L;
    if (lattice_make(Q, &L)) return -1;
    for (int i = 0; i < Q; ++i) {
        W[i] = L.W[i];
        A[i] = L.A[i];
        B[i] = L.B[i];
        C[i] = L.C[i];
        opp[i] = L.opp[i];
        for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    }
    *zeta = L.zeta;
    return 0;
}

/* ------------------------------------------------------------------ helpers */

static long long node_index(const ora_ctx* s, int x, int y, int z) {
    return (long long)x + (long long)s->p.nx * ((long long)y + (long long)s->p.ny * z);
}

/* neighbour of node n along +c_i (sgn = +1) or -c_i (sgn = -1), periodic wrap */
static long long neighbour(const ora_ctx* s, long long n, int i, int sgn) {
    return s->nbr[(long long)(sgn > 0 ? i : s->L.opp[i]) * s->N + n];
}

static void build_neighbours(ora_ctx* s) {
    int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    for (int i = 0; i < s->L.Q; ++i)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    int xx = ((x + s->L.c[i][0]) % nx + nx) % nx;
                    int yy = ((y + s->L.c[i][1]) % ny + ny) % ny;
                    int zz = ((z + s->L.c[i][2]) % nz + nz) % nz;
                    s->nbr[(long long)i * s->N + node_index(s, x, y, z)] = node_index(s, xx, yy, zz);
                }
}

static double* F(ora_ctx* s, int k, int i) { return s->f + ((long long)k * s->L.Q + i) * s->N; }
static double* FP(ora_ctx* s, int k, int i) {
    return s->fpost + ((long long)k * s->L.Q + i) * s->N;
}
static int is_solid(const ora_ctx* s, long long n) { return s->solid && s->solid[n]; }

/* rest weight t_i(alpha) = A_i + B_i alpha (Eq. feq) */
static double rest_weight(const ora_lattice* L, int i, double alpha) {
    return L->A[i] + L->B[i] * alpha;
}

/* alpha_k: least dense component W_0, others 1 - (1 - W_0)/gamma_k (Sec. II.A) */
static void component_alphas(const ora_lattice* L, const double rho_in[2], double alpha[2]) {
    double rmin = rho_in[0] < rho_in[1] ? rho_in[0] : rho_in[1];
    for (int k = 0; k < 2; ++k) {
        double g = rho_in[k] / rmin;
        alpha[k] = (rho_in[k] == rmin) ? L->W[0] : 1.0 - (1.0 - L->W[0]) / g;
    }
}

/* rho^N of every fluid node from the current populations (Sec. II.A) */
static void phase_field_fluid(ora_ctx* s) {
    int Q = s->L.Q;
#pragma omp parallel for schedule(static) num_threads(s->threads) if (s->threads > 1)
    for (long long n = 0; n < s->N; ++n) {
        if (is_solid(s, n)) continue;
        double rr = 0.0, rb = 0.0;
        for (int i = 0; i < Q; ++i) {
            rr += F(s, 0, i)[n];
            rb += F(s, 1, i)[n];
        }
        s->rhoN[n] = (rr - rb) / (rr + rb);
    }
}

/* neutral wetting: a solid node takes the W-weighted mean of its fluid neighbours */
static void phase_field_solid(ora_ctx* s) {
    if (!s->solid) return;
    int Q = s->L.Q;
#pragma omp parallel for schedule(static) num_threads(s->threads) if (s->threads > 1)
    for (long long n = 0; n < s->N; ++n) {
        if (!is_solid(s, n)) continue;
        double num = 0.0, den = 0.0;
        for (int i = 1; i < Q; ++i) {
            long long m = neighbour(s, n, i, +1);
            if (is_solid(s, m)) continue;
            num += s->L.W[i] * s->rhoN[m];
            den += s->L.W[i];
        }
        s->rhoN[n] = den > 0.0 ? num / den : 0.0;
    }
}

/* compact isotropic gradient: dF_a = (1/c_s^2) sum_i W_i rho^N(x + c_i) c_ia */
static void colour_gradient(const ora_ctx* s, long long n, double Fv[3]) {
    Fv[0] = Fv[1] = Fv[2] = 0.0;
    for (int i = 1; i < s->L.Q; ++i) {
        long long m = neighbour(s, n, i, +1);
        for (int a = 0; a < 3; ++a) Fv[a] += s->L.W[i] * s->rhoN[m] * s->L.c[i][a];
    }
    for (int a = 0; a < 3; ++a) Fv[a] /= s->L.cs2;
}

/* ------------------------------------------------------------------ lifecycle */

ora_ctx* ora_create(const ora_params* p, const unsigned char* solid, const double* phi_field) {
    ora_ctx* s = (ora_ctx*)calloc(1, sizeof(ora_ctx));
    if (!s) return NULL;
    s->p = *p;
    if (lattice_make(p->Q, &s->L) || p->nx < 1 || p->ny < 1 || p->nz < 1 ||
        (p->Q == 9 && p->nz != 1)) {
        free(s);
        return NULL;
    }
    s->N = (long long)p->nx * p->ny * p->nz;
    s->threads = 1;
    component_alphas(&s->L, p->rho_in, s->alpha);
    long long nf = 2LL * s->L.Q * s->N;
    s->f = (double*)calloc(nf, sizeof(double));
    s->fpost = (double*)calloc(nf, sizeof(double));
    s->rhoN = (double*)calloc(s->N, sizeof(double));
    s->fmag = (double*)calloc(s->N, sizeof(double));
    s->nbr = (long long*)malloc((size_t)s->L.Q * s->N * sizeof(long long));
    if (solid) {
        s->solid = (unsigned char*)malloc(s->N);
        if (s->solid) memcpy(s->solid, solid, s->N);
    }
    if (phi_field) {
        s->phi_field = (double*)malloc(s->N * sizeof(double));
        if (s->phi_field) memcpy(s->phi_field, phi_field, s->N * sizeof(double));
    }
    if (!s->f || !s->fpost || !s->rhoN || !s->fmag || !s->nbr || (solid && !s->solid) ||
        (phi_field && !s->phi_field)) {
        free(s->f); free(s->fpost); free(s->rhoN); free(s->fmag); free(s->nbr); free(s->solid);
        free(s->phi_field); free(s);
        return NULL;
    }
    build_neighbours(s);
    return s;
}

void ora_destroy(ora_ctx* s) {
    if (!s) return;
    free(s->f);
    free(s->fpost);
    free(s->rhoN);
    free(s->fmag);
    free(s->nbr);
    free(s->solid);
    free(s->phi_field);
    free(s);
}

/* ||F|| of the current (pre-sink) state, used as the "previous" gradient at step 0 */
void ora_recompute_fmag(ora_ctx* s) {
    phase_field_fluid(s);
    phase_field_solid(s);
    for (long long n = 0; n < s->N; ++n) {
        if (is_solid(s, n)) { s->fmag[n] = 0.0; continue; }
        double Fv[3];
        colour_gradient(s, n, Fv);
        s->fmag[n] = sqrt(Fv[0] * Fv[0] + Fv[1] * Fv[1] + Fv[2] * Fv[2]);
    }
}

/* f_i^k = rho_k [t_i(alpha_k) + W_i (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)]  (Eq. feq per component) */
static void apply_outlets(ora_ctx* s);

int ora_init_equilibrium(ora_ctx* s, const double* rho_r, const double* rho_b, const double* u) {
    int Q = s->L.Q;
    for (long long n = 0; n < s->N; ++n) {
        double uv[3] = {0.0, 0.0, 0.0};
        if (u)
            for (int a = 0; a < s->L.D; ++a) uv[a] = u[a * s->N + n];
        double uu = uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2];
        for (int i = 0; i < Q; ++i) {
            double cu = s->L.c[i][0] * uv[0] + s->L.c[i][1] * uv[1] + s->L.c[i][2] * uv[2];
            double vel = s->L.W[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            if (is_solid(s, n)) {
                F(s, 0, i)[n] = 0.0;
                F(s, 1, i)[n] = 0.0;
            } else {
                F(s, 0, i)[n] = rho_r[n] * (rest_weight(&s->L, i, s->alpha[0]) + vel);
                F(s, 1, i)[n] = rho_b[n] * (rest_weight(&s->L, i, s->alpha[1]) + vel);
            }
        }
    }
    ora_recompute_fmag(s);
    s->step = 0;
    s->site_steps = 0;
    s->sink_total = 0.0;
    apply_outlets(s);
    return 0;
}

int ora_set_populations(ora_ctx* s, const double* f) {
    memcpy(s->f, f, 2ULL * s->L.Q * s->N * sizeof(double));
    apply_outlets(s);
    return 0;
}
int ora_get_populations(const ora_ctx* s, double* f) {
    memcpy(f, s->f, 2ULL * s->L.Q * s->N * sizeof(double));
    return 0;
}
int ora_set_fmag(ora_ctx* s, const double* g) {
    memcpy(s->fmag, g, s->N * sizeof(double));
    return 0;
}
int ora_get_fmag(const ora_ctx* s, double* g) {
    memcpy(g, s->fmag, s->N * sizeof(double));
    return 0;
}
void ora_set_counters(ora_ctx* s, long long step, long long site_steps, double sink_total) {
    s->step = step;
    s->site_steps = site_steps;
    s->sink_total = sink_total;
}

/* ------------------------------------------------------------------ one time step */

/* Site weight of node n: 0 or 1 for the sharp rules; for the soft rule (a differentiable
 * stand-in for the threshold, used to take derivatives with respect to Gamma) the logistic
 * function of (||F_prev|| - Gamma) / kappa. */
static double site_weight(ora_ctx* s, long long n) {
    if (s->p.site_rule == 2) return 1.0 / (1.0 + exp(-(s->fmag[n] - s->p.gamma) / s->p.kappa));
    if (s->p.site_rule == 0) return s->fmag[n] > s->p.gamma ? 1.0 : 0.0;
    double rr = 0.0, rb = 0.0;
    for (int i = 0; i < s->L.Q; ++i) {
        rr += F(s, 0, i)[n];
        rb += F(s, 1, i)[n];
    }
    return fabs((rr - rb) / (rr + rb)) < s->p.gamma ? 1.0 : 0.0;
}

static int site_of(ora_ctx* s, long long n) {
    if (s->p.site_rule == 0) return s->fmag[n] > s->p.gamma;
    if (s->p.site_rule == 2) return site_weight(s, n) > 0.5;
    double rr = 0.0, rb = 0.0;
    for (int i = 0; i < s->L.Q; ++i) {
        rr += F(s, 0, i)[n];
        rb += F(s, 1, i)[n];
    }
    return fabs((rr - rb) / (rr + rb)) < s->p.gamma;
}

/* Pressure outlet (Zou and He) for the blue component on one end plane of the last lattice
 * axis a (z for D3Q19, y for D2Q9); hi = 1 for the plane at the last index (outward normal
 * +a), 0 for index 0 (outward normal -a).  The populations entering through the plane
 * (c_i . n = -1) are unknown after streaming.  With the blue density held at out_rho and no
 * tangential velocity:
 *   u_n = (sum_{c.n=0} f + 2 sum_{c.n=1} f) / rho - 1                       (normal velocity)
 *   f_i = f_opp(i) - 6 W_i rho u_n - sum_t c_it N_t,  N_t = (1/2) sum_{c.n=0} f_j c_jt
 * (the odd part of the equilibrium, 6 W_i rho c_i.u, is the same for every alpha; N_t removes
 * the tangential momentum, two unknowns have c_it != 0 per tangential axis t).  No red fluid
 * enters: its unknown populations are 0. */
static void outlet_plane(ora_ctx* s, int hi) {
    const ora_lattice* L = &s->L;
    const int Q = L->Q, a = L->D == 3 ? 2 : 1;
    const int sgn = hi ? 1 : -1;
    const long long nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    const long long idx = hi ? (a == 2 ? nz : ny) - 1 : 0;
    for (long long z = 0; z < nz; ++z)
        for (long long y = 0; y < ny; ++y)
            for (long long x = 0; x < nx; ++x) {
                if ((a == 2 ? z : y) != idx) continue;
                const long long n = x + nx * (y + ny * z);
                if (is_solid(s, n)) continue;
                double s0 = 0.0, s1 = 0.0, N[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < Q; ++i) {
                    const int cn = sgn * L->c[i][a];
                    const double f = F(s, 1, i)[n];
                    if (cn == 0) {
                        s0 += f;
                        for (int t = 0; t < 3; ++t)
                            if (t != a) N[t] += 0.5 * f * L->c[i][t];
                    } else if (cn == 1) {
                        s1 += f;
                    }
                }
                const double rho = s->out_rho;
                const double un = (s0 + 2.0 * s1) / rho - 1.0;
                for (int i = 0; i < Q; ++i) {
                    if (sgn * L->c[i][a] != -1) continue;
                    double f = F(s, 1, L->opp[i])[n] - 6.0 * L->W[i] * rho * un;
                    for (int t = 0; t < 3; ++t)
                        if (t != a) f -= L->c[i][t] * N[t];
                    F(s, 1, i)[n] = f;
                    F(s, 0, i)[n] = 0.0;
                }
            }
}

/* The outlet planes hold their values in every state: after streaming, and whenever a
 * state is set or the outlets are switched on. */
static void apply_outlets(ora_ctx* s) {
    if (s->out_lo) outlet_plane(s, 0);
    if (s->out_hi) outlet_plane(s, 1);
}

static void one_step(ora_ctx* s, const unsigned char* mask_in, unsigned char* mask_out) {
    const ora_lattice* L = &s->L;
    const int Q = L->Q;

    /* steps 1-3: sink rate, sites from the previous gradient, rest-population exchange */
    for (long long n = 0; n < s->N; ++n) {
        if (is_solid(s, n)) {
            if (mask_out) mask_out[n] = 0;
            continue;
        }
        double m = mask_in ? (mask_in[n] != 0 ? 1.0 : 0.0) : site_weight(s, n);
        if (mask_out) mask_out[n] = (unsigned char)(m > 0.5);
        if (m == 0.0) continue;
        double phi = s->phi_field ? s->phi_field[n] : s->p.phi;
        double sink = m * (phi / s->p.sbar); /* phi = Sbar * varphi * dx, removed mass varphi*dt */
        F(s, 0, 0)[n] -= sink;
        F(s, 1, 0)[n] += sink;
        s->sink_total += sink;
        if (m > 0.5) s->site_steps += 1;
    }

    /* step 4: colour-blind moments and phase field, for all nodes before any gradient */
    phase_field_fluid(s);
    phase_field_solid(s);

    /* step 5: gradient, collision, perturbation, recolouring at every fluid node */
#pragma omp parallel for schedule(static) num_threads(s->threads) if (s->threads > 1)
    for (long long n = 0; n < s->N; ++n) {
        if (is_solid(s, n)) {
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < Q; ++i) FP(s, k, i)[n] = 0.0;
            s->fmag[n] = 0.0;
            continue;
        }
        double rho_k[2] = {0.0, 0.0}, fcb[ORA_MAXQ], j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            rho_k[0] += F(s, 0, i)[n];
            rho_k[1] += F(s, 1, i)[n];
            fcb[i] = F(s, 0, i)[n] + F(s, 1, i)[n]; /* colour-blind population */
        }
        double rho = rho_k[0] + rho_k[1];
        for (int i = 0; i < Q; ++i)
            for (int a = 0; a < 3; ++a) j[a] += fcb[i] * L->c[i][a];
        double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

        /* harmonic relaxation time and density-weighted alpha (Sec. II.A) */
        double inv_tau = (rho_k[0] / rho) / s->p.tau[0] + (rho_k[1] / rho) / s->p.tau[1];
        double tau = 1.0 / inv_tau;
        double abar = (rho_k[0] / rho) * s->alpha[0] + (rho_k[1] / rho) * s->alpha[1];

        /* colour gradient from the post-sink phase field */
        double Fv[3];
        colour_gradient(s, n, Fv);
        double F2 = Fv[0] * Fv[0] + Fv[1] * Fv[1] + Fv[2] * Fv[2];
        double Fn = sqrt(F2);
        /* cos(theta) and the perturbation are 0/0 forms at F = 0: both are taken as 0 where
           F.F <= 1e-24 (their limit; the perturbation is O(||F||)) */
        int has_grad = F2 > 1e-24;
        double fade = 1.0; /* optional regularisation, off unless recolor_fade > 0 */
        if (s->p.recolor_fade > 0.0) {
            fade = Fn / s->p.recolor_fade - 1.0;
            if (fade < 0.0) fade = 0.0;
            if (fade > 1.0) fade = 1.0;
        }

        for (int i = 0; i < Q; ++i) {
            double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
            double feq = rho * (rest_weight(L, i, abar) +
                                L->W[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
            /* BGK collision (Eq. collision), dt = 1 */
            double fc = fcb[i] - (fcb[i] - feq) / tau;
            /* perturbation (Eq. perturb) */
            double cosv = 0.0;
            if (has_grad) {
                double Fc = Fv[0] * L->c[i][0] + Fv[1] * L->c[i][1] + Fv[2] * L->c[i][2];
                fc += 2.25 * (s->p.sigma / tau) * Fn * (L->W[i] * Fc * Fc / F2 - L->C[i]);
                if (i != 0) {
                    double cn = sqrt((double)(L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] +
                                              L->c[i][2] * L->c[i][2]));
                    cosv = Fc / (Fn * cn) * fade;
                }
            }
            /* recolouring (Eq. recolor); f_i^eq(rho, 0) = rho t_i(abar) */
            double feq0 = rho * rest_weight(L, i, abar);
            double sep = s->p.beta * rho_k[0] * rho_k[1] / (rho * rho) * cosv * feq0;
            FP(s, 0, i)[n] = rho_k[0] / rho * fc + sep;
            FP(s, 1, i)[n] = rho_k[1] / rho * fc - sep;
        }
        s->fmag[n] = Fn; /* carried to the next step's site selection */
    }

    /* step 6: streaming (pull form), halfway bounce-back from solid neighbours; then the
       populations that enter through an outlet plane */
#pragma omp parallel for schedule(static) num_threads(s->threads) if (s->threads > 1)
    for (long long n = 0; n < s->N; ++n) {
        for (int i = 0; i < Q; ++i) {
            if (is_solid(s, n)) {
                F(s, 0, i)[n] = 0.0;
                F(s, 1, i)[n] = 0.0;
                continue;
            }
            long long src = neighbour(s, n, i, -1);
            for (int k = 0; k < 2; ++k)
                F(s, k, i)[n] = is_solid(s, src) ? FP(s, k, L->opp[i])[n] : FP(s, k, i)[src];
        }
    }
    apply_outlets(s);
    s->step += 1;
}

/* Height-dependent flux (Sec. III, space- and time-varying flux; Eq. heated):
 * Phi = phi_S / (K + h / h_s), where h is the local drop height above the substrate.  The
 * substrate normal is the last lattice axis (z for D3Q19, y for D2Q9).  h of a column is
 * its red thickness, the sum over its fluid nodes of the red fraction (1 + rho^N)/2 of the
 * current (pre-sink) state; every node of the column gets the column's flux. */
static void height_flux(ora_ctx* s) {
    const int Q = s->L.Q;
    const long long nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    const long long ncol = s->L.D == 3 ? nx * ny : nx;   /* columns */
    const long long len = s->L.D == 3 ? nz : ny;          /* nodes per column */
    const long long stride = s->L.D == 3 ? nx * ny : nx;  /* node step along the column */
    for (long long col = 0; col < ncol; ++col) {
        double h = 0.0;
        for (long long k = 0; k < len; ++k) {
            const long long n = col + k * stride;
            if (is_solid(s, n)) continue;
            double rr = 0.0, rb = 0.0;
            for (int i = 0; i < Q; ++i) {
                rr += F(s, 0, i)[n];
                rb += F(s, 1, i)[n];
            }
            h += 0.5 * (1.0 + (rr - rb) / (rr + rb));
        }
        const double phi = s->hf_phi / (s->hf_K + h / s->hf_hs);
        for (long long k = 0; k < len; ++k) s->phi_field[col + k * stride] = phi;
    }
}

/* Switch the height-dependent flux on (every > 0: refresh the flux field from the current
 * state before every step whose step counter is a multiple of `every`) or off (every <= 0,
 * which keeps the last field). */
int ora_set_height_flux(ora_ctx* s, double phi_s, double K, double h_scale, long long every) {
    if (every > 0 && (!(h_scale > 0.0) || !(K > 0.0) || !isfinite(phi_s) || !isfinite(K)))
        return 1;
    if (every > 0 && !s->phi_field) {
        s->phi_field = (double*)malloc(s->N * sizeof(double));
        if (!s->phi_field) return 1;
        for (long long n = 0; n < s->N; ++n) s->phi_field[n] = s->p.phi;
    }
    s->hf_every = every;
    s->hf_phi = phi_s;
    s->hf_K = K;
    s->hf_hs = h_scale;
    return 0;
}

/* Threads of the per-node loops (>= 1; without OpenMP the loops stay sequential). */
int ora_set_threads(ora_ctx* s, int threads) {
    if (threads < 1) return 1;
    s->threads = threads;
    return 0;
}

/* Advance nsteps.  mask_in (nullable, [nsteps][N]) replaces the site selection
 * (frozen-mask runs); mask_log (nullable, [nsteps][N]) records the sites used. */
int ora_step(ora_ctx* s, long long nsteps, unsigned char* mask_log, const unsigned char* mask_in) {
    for (long long t = 0; t < nsteps; ++t) {
        if (s->hf_every > 0 && s->step % s->hf_every == 0) height_flux(s);
        one_step(s, mask_in ? mask_in + t * s->N : NULL, mask_log ? mask_log + t * s->N : NULL);
    }
    return 0;
}

/* Pressure outlets for the blue component (see outlet_plane): lo, hi switch the planes at
 * the ends of the last lattice axis; rho_out > 0 is the blue density held there. */
int ora_set_outlet(ora_ctx* s, int lo, int hi, double rho_out) {
    if ((lo || hi) && !(rho_out > 0.0 && isfinite(rho_out))) return 1;
    if ((lo || hi) && (s->L.D == 3 ? s->p.nz : s->p.ny) < 3) return 1;
    s->out_lo = lo != 0;
    s->out_hi = hi != 0;
    s->out_rho = rho_out;
    apply_outlets(s);  /* the current state takes the outlet values at once */
    return 0;
}

/* The flux field in use (N doubles), or 1 when none is bound. */
int ora_get_phi_field(const ora_ctx* s, double* out) {
    if (!s->phi_field) return 1;
    memcpy(out, s->phi_field, s->N * sizeof(double));
    return 0;
}

/* ------------------------------------------------------------------ observables */

/* Per-node macroscopic fields of the current state (pre-sink): rho_r, rho_b, u[D][N],
 * rho^N, and the gradient magnitude ||F|| of that phase field.  Any pointer may be NULL. */
int ora_fields(ora_ctx* s, double* rho_r, double* rho_b, double* u, double* rhoN, double* gradmag) {
    int Q = s->L.Q;
    phase_field_fluid(s);
    phase_field_solid(s);
    for (long long n = 0; n < s->N; ++n) {
        double rr = 0.0, rb = 0.0, j[3] = {0.0, 0.0, 0.0};
        if (!is_solid(s, n)) {
            for (int i = 0; i < Q; ++i) {
                double a = F(s, 0, i)[n], b = F(s, 1, i)[n];
                rr += a;
                rb += b;
                for (int d = 0; d < 3; ++d) j[d] += (a + b) * s->L.c[i][d];
            }
        }
        double rho = rr + rb;
        if (rho_r) rho_r[n] = rr;
        if (rho_b) rho_b[n] = rb;
        if (u)
            for (int d = 0; d < s->L.D; ++d) u[d * s->N + n] = rho > 0.0 ? j[d] / rho : 0.0;
        if (rhoN) rhoN[n] = s->rhoN[n];
        if (gradmag) {
            double Fv[3] = {0.0, 0.0, 0.0};
            if (!is_solid(s, n)) colour_gradient(s, n, Fv);
            gradmag[n] = sqrt(Fv[0] * Fv[0] + Fv[1] * Fv[1] + Fv[2] * Fv[2]);
        }
    }
    return 0;
}

/* Reductions over fluid nodes, summed sequentially in node order. */
int ora_observables(ora_ctx* s, ora_obs* o) {
    const int Q = s->L.Q;
    memset(o, 0, sizeof(*o));
    phase_field_fluid(s);
    phase_field_solid(s);
    double max_rr = 0.0, sum_pin = 0.0, sum_pout = 0.0;
    long long n_in = 0, n_out = 0;
    for (long long n = 0; n < s->N; ++n) {
        if (is_solid(s, n)) continue;
        double rr = 0.0, rb = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            double a = F(s, 0, i)[n], b = F(s, 1, i)[n];
            rr += a;
            rb += b;
            /* negative beyond rounding noise: below -1e-6 of the bulk equilibrium value */
            if (a < -1e-6 * s->p.rho_in[0] * rest_weight(&s->L, i, s->alpha[0])) o->n_negative++;
            if (b < -1e-6 * s->p.rho_in[1] * rest_weight(&s->L, i, s->alpha[1])) o->n_negative++;
            for (int d = 0; d < 3; ++d) j[d] += (a + b) * s->L.c[i][d];
        }
        double rho = rr + rb;
        double un = sqrt(j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / rho;
        if (un > o->max_u) o->max_u = un;
        o->mass_r += rr;
        o->mass_b += rb;
        if (rr > max_rr) max_rr = rr;
        /* EOS p = sum_k rho_k zeta (1 - alpha_k)  (Eq. EOS) */
        double p = rr * s->L.zeta * (1.0 - s->alpha[0]) + rb * s->L.zeta * (1.0 - s->alpha[1]);
        double rN = s->rhoN[n];
        if (rN > 0.9) { sum_pin += p; n_in++; }
        if (rN < -0.9) { sum_pout += p; n_out++; }
        double Fv[3];
        colour_gradient(s, n, Fv);
        o->perim_grad += 0.5 * sqrt(Fv[0] * Fv[0] + Fv[1] * Fv[1] + Fv[2] * Fv[2]);
        if (site_of(s, n)) o->n_sites++;
    }
    for (long long n = 0; n < s->N; ++n) {
        if (is_solid(s, n)) continue;
        double rr = 0.0;
        for (int i = 0; i < Q; ++i) rr += F(s, 0, i)[n];
        if (rr > 0.5 * max_rr) o->v_half++;
    }
    o->step = s->step;
    o->site_steps = s->site_steps;
    o->sink_total = s->sink_total;
    o->v_mass = o->mass_r / s->p.rho_in[0];
    o->perim_sites = (double)o->n_sites / s->p.sbar;
    o->p_in = n_in ? sum_pin / n_in : 0.0;
    o->p_out = n_out ? sum_pout / n_out : 0.0;
    o->max_rho_r = max_rr;
    return 0;
}
