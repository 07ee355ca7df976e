/*
 * Drives the host-side code of the C-ABI library (parameter validation,
 * node classification, wall and ghost tables, sub-voxel wall fractions,
 * tile tables, arena layout) through lbm_footprint and lbm_create, for the
 * AddressSanitizer / UndefinedBehaviorSanitizer build of the library's host
 * code run by tests/test_sanitizers.py.  Without a GPU, lbm_create stops at
 * its first device call with LBM_E_DEVICE after the host-side layout has
 * run; with one it succeeds and the handle is destroyed.  Exit status 0 and
 * no sanitizer report = pass.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

/* friction model of the next cases */
static int g_friction = LBM_FRICTION_INTERFACE_SLIP;
static double g_slip_factor = 1.0;

static void base(lbm_params *p, int nx, int ny, int nz) {
    memset(p, 0, sizeof(*p));
    p->nx = nx; p->ny = ny; p->nz = nz;
    p->storage = LBM_FP32_SHIFT;
    p->rho_l = 1.0; p->rho_g = 0.001; p->nu_l = 0.01; p->nu_g = 0.1;
    p->sigma = 1e-3; p->W = 4.0; p->M = 1.0 / 6.0;
    p->mobility_corr = 1; p->mc_gamma = -22.5; p->mc_phi_M = 0.8; p->mc_phi_m = 0.2; p->mc_D = 1e-4;
    p->eps = 1e-10; p->mix = LBM_MIX_TANH; p->mix_phi = 0.1; p->mix_width = 0.001;
    p->friction = g_friction; p->slip_factor = g_slip_factor; p->slip_lo = 0.5; p->slip_hi = 0.95;
    p->P_ref = 1.0 / 3.0; p->q_phase = 7; p->hyst_beta = 0.95;
}

static int create_case(const char *name, int nx, int ny, int nz, int walls, int open_x, int q,
                       int hyst, int subvoxel, int storage, int expect_inval) {
    const long N = (long)nx * ny * nz;
    lbm_params p;
    base(&p, nx, ny, nz);
    p.q_phase = q; p.hysteresis = hyst; p.subvoxel = subvoxel; p.storage = storage;
    if (open_x) {
        p.face_bc[0] = p.face_bc[1] = LBM_BC_PRESSURE;
        p.face_P[0] = p.P_ref + 1e-4; p.face_P[1] = p.P_ref;
    }
    uint8_t *solid = calloc(N, 1);
    double *phi = malloc(N * sizeof(double)), *sdf = malloc(N * sizeof(double));
    for (long n = 0; n < N; ++n) {
        long x = n % nx, y = (n / nx) % ny, z = n / ((long)nx * ny);
        phi[n] = 0.5 * (1.0 - tanh((fabs(x - nx / 2.0) - nx / 4.0) / 2.0));
        if (walls && (y == 0 || z == 0 || y == ny - 1)) solid[n] = (uint8_t)(z == 0 ? 2 : 1);
        double sy = fmin(y - 0.6, (ny - 1) - 0.6 - y), sz = z - (0.55 + 0.3 * cos(0.4 * x));
        sdf[n] = sy < sz ? sy : sz;
    }
    lbm_geometry g;
    memset(&g, 0, sizeof(g));
    for (int k = 0; k < 16; ++k) g.theta_deg[k] = 90.0;
    g.theta_deg[0] = 60.0; g.theta_deg[1] = 120.0;
    g.solid = walls ? solid : NULL;
    g.sdf = subvoxel ? sdf : NULL;
    lbm_init in;
    memset(&in, 0, sizeof(in));
    in.kind = LBM_INIT_FIELDS;
    in.phi = phi;
    size_t fp = lbm_footprint(&p);
    lbm_handle *h = NULL;
    int rc = lbm_create(&p, &g, &in, NULL, &h);
    int bad = 0;
    if (expect_inval) bad = rc != LBM_E_INVAL || fp != 0;
    else bad = !(rc == LBM_OK || rc == LBM_E_DEVICE) || fp == 0;
    printf("%s: footprint %zu rc %d %s\n", name, fp, rc, rc ? lbm_last_error() : "");
    if (h) lbm_destroy(h);
    free(solid); free(phi); free(sdf);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= create_case("periodic", 20, 9, 7, 0, 0, 7, 0, 0, LBM_FP32_SHIFT, 0);
    bad |= create_case("walls_open", 70, 13, 9, 1, 1, 7, 0, 0, LBM_FP32_SHIFT, 0);
    bad |= create_case("walls_q19_hyst", 33, 10, 6, 1, 1, 19, 1, 0, LBM_FP64, 0);
    bad |= create_case("subvoxel", 64, 12, 8, 1, 0, 7, 2, 1, LBM_FP16_SHIFT_G, 0);
    bad |= create_case("ragged_tiles", 17, 5, 3, 1, 1, 7, 0, 0, LBM_FP32, 0);
    bad |= create_case("fp16_all", 20, 9, 7, 1, 0, 7, 0, 0, LBM_FP16_SHIFT_ALL, 1);
    bad |= create_case("bad_q", 20, 9, 7, 1, 0, 8, 0, 0, LBM_FP32_SHIFT, 1);
    bad |= create_case("empty", 0, 9, 7, 0, 0, 7, 0, 0, LBM_FP32_SHIFT, 1);
    g_friction = LBM_FRICTION_PARTIAL_SLIP; g_slip_factor = 0.5;
    bad |= create_case("partial_slip", 40, 12, 10, 1, 1, 7, 0, 1, LBM_FP32_SHIFT, 0);
    g_slip_factor = 1.5;
    bad |= create_case("bad_slip_factor", 40, 12, 10, 1, 1, 7, 0, 0, LBM_FP32_SHIFT, 1);
    g_friction = 3; g_slip_factor = 0.5;
    bad |= create_case("bad_friction", 40, 12, 10, 1, 1, 7, 0, 0, LBM_FP32_SHIFT, 1);
    printf(bad ? "FAIL\n" : "OK\n");
    return bad;
}
