/* Host-only driver that runs the FP64 oracle under AddressSanitizer and UBSan: every site rule,
 * walls and a flux field, D2Q9 and D3Q19, small domains with ragged sizes.  Built and run by
 * tests/test_oracle_sanitized.py; exits non-zero on any sanitizer report. */
#include "../../oracle/cg_oracle.c"

#include <stdio.h>

static int run(int Q, int nx, int ny, int nz, int site_rule, int walls, int field) {
    ora_params p = {0};
    p.Q = Q;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.rho_in[0] = 1.0;
    p.rho_in[1] = walls ? 0.1 : 1.0;
    p.tau[0] = 1.0;
    p.tau[1] = walls ? 0.6 : 1.0;
    p.sigma = 4e-4;
    p.beta = 0.7;
    p.phi = 1e-3;
    p.sbar = 3.0;
    p.gamma = site_rule == 1 ? 0.5 : 0.1;
    p.site_rule = site_rule;
    p.kappa = 0.01;
    const long long N = (long long)nx * ny * nz;
    unsigned char* solid = NULL;
    double* phi = NULL;
    double* rr = malloc(sizeof(double) * N);
    double* rb = malloc(sizeof(double) * N);
    if (walls) solid = calloc(N, 1);
    if (field) phi = malloc(sizeof(double) * N);
    for (long long n = 0; n < N; ++n) {
        const int x = (int)(n % nx), y = (int)((n / nx) % ny);
        const double d = 4.0 - sqrt((x - nx / 2.0) * (x - nx / 2.0) + (y - ny / 2.0) * (y - ny / 2.0));
        const double c = 0.5 * (1.0 + tanh(d / 2.0));
        rr[n] = c;
        rb[n] = (1.0 - c) * p.rho_in[1];
        if (walls && (y == 0 || y == ny - 1)) {
            solid[n] = 1;
            rr[n] = rb[n] = 0.0;
        }
        if (field) phi[n] = 1e-3 * (1.0 + 0.1 * (double)(n % 7) / 7.0);
    }
    ora_ctx* s = ora_create(&p, solid, phi);
    if (!s) return 1;
    int rc = ora_init_equilibrium(s, rr, rb, NULL);
    unsigned char* log = malloc((size_t)N * 3);
    if (walls) rc |= ora_set_height_flux(s, 1e-3, 1.0, 4.0, 2);
    rc |= ora_step(s, 3, log, NULL);
    rc |= ora_step(s, 2, NULL, log);
    double* f = malloc(sizeof(double) * 2 * Q * N);
    rc |= ora_get_populations(s, f);
    rc |= ora_set_populations(s, f);
    double* g = malloc(sizeof(double) * N);
    rc |= ora_get_fmag(s, g);
    rc |= ora_set_fmag(s, g);
    ora_recompute_fmag(s);
    double* fl = malloc(sizeof(double) * 8 * N);
    rc |= ora_fields(s, fl, fl + N, fl + 2 * N, fl + 5 * N, fl + 6 * N);
    ora_obs o;
    rc |= ora_observables(s, &o);
    printf("Q=%d %dx%dx%d rule=%d walls=%d field=%d mass_r=%.12g sites=%lld rc=%d\n", Q, nx, ny,
           nz, site_rule, walls, field, o.mass_r, o.n_sites, rc);
    ora_destroy(s);
    free(rr);
    free(rb);
    free(solid);
    free(phi);
    free(log);
    free(f);
    free(g);
    free(fl);
    return rc != 0;
}

int main(void) {
    int bad = 0;
    for (int rule = 0; rule < 3; ++rule) {
        bad |= run(9, 13, 11, 1, rule, 0, 0);
        bad |= run(9, 13, 11, 1, rule, 1, 1);
        bad |= run(19, 7, 6, 5, rule, 0, 1);
        bad |= run(19, 7, 6, 5, rule, 1, 0);
    }
    return bad;
}
