/*
 * Drives the FP64 oracle (oracle/lbmref.c) through every option on tiny
 * lattices, for the AddressSanitizer / UndefinedBehaviorSanitizer build run
 * by tests/test_sanitizers.py: periodic, walls of two materials, pressure
 * faces, the optimised model, hysteresis (both readings), the D3Q19 phase
 * lattice and sub-voxel walls (both upstream readings), with read-out,
 * restore and diagnostics.  Exit status 0 and no sanitizer report = pass.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbmref.h"

static void base_params(lbmref_params *p, int nx, int ny, int nz) {
    memset(p, 0, sizeof(*p));
    p->nx = nx; p->ny = ny; p->nz = nz;
    p->rho_l = 1.0; p->rho_g = 0.001; p->nu_l = 0.01; p->nu_g = 0.1;
    p->sigma = 1e-3; p->W = 4.0; p->M = 1.0 / 6.0;
    p->mobility_corr = 1; p->gamma = -22.5; p->phi_M = 0.8; p->phi_m = 0.2; p->D = 1e-4;
    p->eps = 1e-10; p->mix_phi = 0.1; p->mix_width = 0.001; p->slip_lo = 0.5; p->slip_hi = 0.95;
    p->P_ref = 1.0 / 3.0; p->clamp_a = 1e-12; p->hyst_beta = 0.95; p->q_phase = 7;
    p->slip_factor = 1.0;
    for (int k = 0; k < 16; ++k) p->theta_deg[k] = 90.0;
}

static int run_case(const char *name, int walls, int open_x, int optimised, int hyst, int q,
                    int subvoxel, int same_step) {
    const int nx = 9, ny = 7, nz = 6;
    const long N = (long)nx * ny * nz;
    lbmref_params p;
    base_params(&p, nx, ny, nz);
    p.mix_tanh = optimised; p.interface_slip = optimised;
    p.hysteresis = hyst; p.q_phase = q; p.subvoxel_same_step = same_step;
    p.theta_deg[0] = 55.0; p.theta_deg[1] = 125.0;
    if (open_x) {
        p.face_pressure[0] = p.face_pressure[1] = 1;
        p.face_P[0] = p.P_ref + 2e-4; p.face_ramp[0] = 1e-6; p.face_P[1] = p.P_ref;
    }
    double *phi = malloc(N * sizeof(double)), *u = malloc(3 * N * sizeof(double));
    double *P = malloc(N * sizeof(double)), *sdf = malloc(N * sizeof(double));
    uint8_t *solid = calloc(N, 1);
    for (long n = 0; n < N; ++n) {
        long x = n % nx, y = (n / nx) % ny, z = n / ((long)nx * ny);
        double r = sqrt((x - 4.3) * (x - 4.3) + (y - 3.6) * (y - 3.6) + (z - 2.9) * (z - 2.9));
        phi[n] = 0.5 * (1.0 - tanh((r - 2.2) / 2.0));
        for (int a = 0; a < 3; ++a) u[a * N + n] = 1e-3 * sin(0.7 * n + a);
        P[n] = p.P_ref + 1e-5 * cos(0.3 * n);
        if (walls && (y == 0 || z == 0)) solid[n] = (uint8_t)(y == 0 ? 1 : 2);
        double sy = y - (0.7 + 0.2 * sin(0.9 * x)), sz = z - (0.6 + 0.25 * cos(0.8 * x));
        sdf[n] = sy < sz ? sy : sz;
    }
    lbmref_state *s = lbmref_create(&p, walls ? solid : NULL, (walls && subvoxel) ? sdf : NULL, phi, u, P);
    if (!s) { fprintf(stderr, "%s: create failed\n", name); return 1; }
    lbmref_step(s, 7);
    const int Q = q == 19 ? 19 : 7;
    double *h = malloc((size_t)Q * N * sizeof(double)), *g = malloc(19 * N * sizeof(double));
    lbmref_fields(s, phi, P, u);
    lbmref_pops(s, h, g);
    lbmref_set_pops(s, h, g, lbmref_step_count(s));
    lbmref_step(s, 4);
    lbmref_diag d;
    lbmref_diagnostics(s, &d);
    uint8_t *kind = malloc(N);
    lbmref_kinds(s, kind);
    int bad = !(d.n_nan == 0 && isfinite(d.phi_sum));
    printf("%s: phi_sum %.12f n_nan %ld\n", name, d.phi_sum, d.n_nan);
    lbmref_destroy(s);
    free(phi); free(u); free(P); free(sdf); free(solid); free(h); free(g); free(kind);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= run_case("periodic", 0, 0, 0, 0, 7, 0, 0);
    bad |= run_case("walls", 1, 0, 0, 0, 7, 0, 0);
    bad |= run_case("walls_open_optimised", 1, 1, 1, 0, 7, 0, 0);
    bad |= run_case("hysteresis_1", 1, 1, 1, 1, 7, 0, 0);
    bad |= run_case("hysteresis_2_q19", 1, 1, 1, 2, 19, 0, 0);
    bad |= run_case("subvoxel_lagged", 1, 1, 1, 0, 7, 1, 0);
    bad |= run_case("subvoxel_same_step_q19", 1, 0, 1, 1, 19, 1, 1);
    /* single-node building blocks */
    lbmref_params p;
    base_params(&p, 4, 4, 4);
    double w[3], nw[3] = {0.0, 0.0, 1.0}, g0[3] = {0.1, -0.2, 0.05};
    int c[3] = {1, 0, 1};
    lbmref_wet_direction(nw, g0, 60.0, p.eps, w);
    double ps = lbmref_wet_phi_s(0.7, w, c, p.W, p.clamp_a);
    double dt = lbmref_dtheta(&p, 0.85, 0.03, -1e-3);
    double gin[19], gout[19], uu[3], PP, geq[19], K[19], grad[3] = {0.01, 0.0, -0.02};
    for (int i = 0; i < 19; ++i) gin[i] = 0.05 + 0.001 * i;
    lbmref_collide_g_node(&p, gin, 0.6, grad, 1e-3, gout, uu, &PP);
    lbmref_geq_node(&p, 0.6, uu, PP, grad, 1e-3, geq, K);
    bad |= !(isfinite(ps) && isfinite(dt) && isfinite(gout[7]) && isfinite(geq[3]));
    /* invalid input is rejected, not read past its end */
    lbmref_params q;
    base_params(&q, 0, 4, 4);
    double one = 1.0;
    bad |= lbmref_create(&q, NULL, NULL, &one, NULL, NULL) != NULL;
    printf(bad ? "FAIL\n" : "OK\n");
    return bad;
}
