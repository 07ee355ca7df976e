/*
 * lbmref.h -- FP64 CPU oracle for the conservative Allen-Cahn phase-field
 * lattice Boltzmann step (Thirumalaisamy et al., "Capillary flow simulation
 * with the phase-field-based lattice Boltzmann solver", Sec. II and III.A).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the GPU path.
 *
 * Scheme: two lattices (read A, write B) with a pull-form streaming step,
 * every quantity in IEEE double.  Node index n = x + nx*(y + ny*z); every
 * per-node input/output array is laid out in that order, vector fields as
 * [3][N] and population arrays as [Q][N].
 *
 * Lattice order (an interface format the GPU library also follows):
 *   0:(0,0,0)  1:(+1,0,0) 2:(-1,0,0) 3:(0,+1,0) 4:(0,-1,0) 5:(0,0,+1) 6:(0,0,-1)
 *   7:(+1,+1,0) 8:(-1,-1,0) 9:(+1,-1,0) 10:(-1,+1,0)
 *   11:(+1,0,+1) 12:(-1,0,-1) 13:(+1,0,-1) 14:(-1,0,+1)
 *   15:(0,+1,+1) 16:(0,-1,-1) 17:(0,+1,-1) 18:(0,-1,+1)
 * The hydrodynamic populations use all 19 (D3Q19, T = 1/3); the phase-field
 * populations use the first 7 (D3Q7, T = 1/4).
 */
#ifndef LBMREF_H
#define LBMREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbmref_params {
    int nx, ny, nz;
    /* fluids: phi = 1 is the heavy (liquid) phase */
    double rho_l, rho_g, nu_l, nu_g;
    double sigma, W, M;
    double F_ex[3];
    /* local mobility correction (Sec. II.A, delta-theta) */
    int mobility_corr;
    double gamma, phi_M, phi_m, D;
    double eps;            /* epsilon in n = grad/(|grad|+eps) and in the sign term */
    /* mixture relaxation: 0 -> F(phi) = phi, 1 -> F = 0.5[tanh((phi-mix_phi)/mix_width)+1] */
    int mix_tanh;
    double mix_phi, mix_width;
    /* friction: 0 -> no-slip bounce-back everywhere,
     *           1 -> free-slip (wall moving with the tangential fluid velocity)
     *                where slip_lo <= phi <= slip_hi */
    int interface_slip;
    double slip_lo, slip_hi;
    double P_ref;
    /* faces 0:x- 1:x+ 2:y- 3:y+ 4:z- 5:z+ ; 0 periodic, 1 pressure */
    int face_pressure[6];
    double face_P[6], face_ramp[6];
    double theta_deg[16];  /* contact angle per solid material */
    double clamp_a;        /* a = 2 phi - 1 is clamped to [-1+clamp_a, 1-clamp_a] */
    /* contact-angle hysteresis (Sec. III.A): each wall link blends its value
     * with one kept from the previous step,
     * phi_s,i = beta * previous + (1 - beta) * phi_s,i (current gradient);
     * 0 off; 1: previous = the blended value that step used (recursive);
     * 2: previous = the value from that step's own gradient */
    int hysteresis;
    double hyst_beta;
    /* phase-field lattice: 7 (D3Q7, T = 1/4) or 19 (D3Q19, T = 1/3, as the
     * paper writes Eqs. 1-4); 0 means 7 */
    int q_phase;
    /* sub-voxel walls, links whose wall lies nearer than half a link (q < 1/2):
     * which upstream value the linear interpolated bounce-back takes.
     * 0: the population that entered the node along the link at this step
     *    (the upstream node's post-collision value of the step before; the
     *    local form an in-place update can evaluate);
     * 1: the upstream node's post-collision value of the same step (the
     *    scheme as published); where that node is solid, the half-way rule. */
    int subvoxel_same_step;
    /* wall velocity in the slip band, as a fraction of the tangential fluid
     * velocity: 1 the free slip of Sec. III.A, 0 no slip, in between a
     * partial slip (read only when interface_slip is set) */
    double slip_factor;
} lbmref_params;

typedef struct lbmref_diag {
    double phi_sum;
    double mom[3];
    double u_max;
    double P_liq_mean, P_gas_mean;   /* mean P over phi > 0.99 / phi < 0.01 */
    long n_nan, n_liq, n_gas;
} lbmref_diag;

typedef struct lbmref_state lbmref_state;

/* solid[n]: 0 = fluid, 1+k = solid of material k (k < 16).  May be NULL.
 * sdf[N]: NULL for voxel walls (half-way bounce-back, normals from the solid
 * links); else sub-voxel walls given by the signed distance to the wall
 * surface (> 0 at fluid nodes next to a wall, <= 0 at their solid
 * neighbours): per-link wall fractions for the interpolated bounce-back of g
 * and wall normals from the distance gradient.
 * phi0[N] required; u0[3][N] and P0[N] may be NULL (0 and P_ref).
 * Returns NULL on invalid input or allocation failure. */
lbmref_state *lbmref_create(const lbmref_params *p, const uint8_t *solid, const double *sdf,
                            const double *phi0, const double *u0, const double *P0);
void lbmref_destroy(lbmref_state *s);
void lbmref_step(lbmref_state *s, long nsteps);
long lbmref_step_count(const lbmref_state *s);
/* node kind: 0 fluid, 1 solid, 2 pressure ghost */
void lbmref_kinds(const lbmref_state *s, uint8_t *kind);
/* phi, P, u at the current step (any may be NULL).  Solid: 0.  Ghost: phi of
 * the owner, P = the face pressure at this step, u = 0. */
void lbmref_fields(lbmref_state *s, double *phi, double *P, double *u);
/* populations f_i(x) entering the collision of the current step, h [Q][N]
 * (Q = 7 or 19, the phase lattice) and g [19][N]; zero at solid and ghost
 * nodes. */
void lbmref_pops(const lbmref_state *s, double *h, double *g);
/* overwrite fluid-node populations (restore); ghosts keep their values */
void lbmref_set_pops(lbmref_state *s, const double *h, const double *g, long step);
void lbmref_diagnostics(lbmref_state *s, lbmref_diag *d);

/* ---- single-node building blocks, exposed for closed-form tests ---- */
/* phi_s,i of the wetting model for one solid link: phi_smpl sampled at the
 * fluid node, w the steepest-variation direction, c the link. */
double lbmref_wet_phi_s(double phi_smpl, const double w[3], const int c[3],
                        double W, double clamp_a);
/* direction w for a wall normal n_w (into the fluid), gradient g0 and angle */
void lbmref_wet_direction(const double n_w[3], const double g0[3], double theta_deg,
                          double eps, double w[3]);
/* delta-theta of the local mobility correction */
double lbmref_dtheta(const lbmref_params *p, double phi, double grad_norm, double lap);
/* D3Q19 collision at one node from its 19 incoming populations, phi, grad phi,
 * laplacian phi.  Writes post-collision populations, u[3] and P. */
void lbmref_collide_g_node(const lbmref_params *p, const double g_in[19], double phi,
                           const double grad[3], double lap, double g_out[19],
                           double u[3], double *P);
/* equilibrium (K_i included) of the hydrodynamic populations */
void lbmref_geq_node(const lbmref_params *p, double phi, const double u[3], double P,
                     const double grad[3], double lap, double geq[19], double K[19]);

#ifdef __cplusplus
}
#endif
#endif
