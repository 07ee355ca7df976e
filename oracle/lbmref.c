/*
 * lbmref.c -- FP64 CPU oracle of the phase-field LB time step.
 *
 * TEST INFRASTRUCTURE ONLY (see lbmref.h).  Plain C99 + OpenMP, two lattices,
 * pull-form streaming, every quantity in double.  Each function names the part
 * of the paper it follows; where the paper is silent the chosen reading is
 * stated next to the code.
 *
 * One time step t -> t+1, in the paper's order:
 *   S1  phi = sum_i h_i                                   (Sec. II.A, after Eq. 4)
 *   S2  neighbour phi, wetting substitute phi_s,i at solid links
 *                                                         (Sec. II.B, Eqs. 17-19)
 *   S3  isotropic gradient / Laplacian                    (Sec. II.A, Eq. 16)
 *   S4  rho, mu, tau_mix                                  (Eqs. 9-12, Sec. III.A)
 *   S5  rho u, u, P                                       (Sec. II.A, after Eq. 15)
 *   S6  filtered D3Q19 collision with forcing K_i         (Eqs. 6-8, 13-15)
 *   S7  D3Q7 phase-field collision, mobility correction   (Eqs. 1-5)
 *   S9  pressure-face ghosts: equilibrium populations from the owner's phi and
 *       u of this step and the face pressure of the next (Dirichlet P, Neumann
 *       u and phi; Sec. III.A)
 *   S8  streaming (pull) with half-way bounce-back at solid links, or with
 *       sub-voxel walls the linearly interpolated bounce-back of g (h keeps
 *       the half-way rule); in the slip band the wall moves with slip_factor
 *       times the tangential fluid velocity (1: the free slip of Sec. III.A);
 *       a ghost source hands over the populations S9 just set (Sec. III.A
 *       friction)
 *   S10 swap lattices, t <- t+1
 * Equation numbers count every numbered display of the paper in order
 * (Eq. 1 the phase-field LB equation ... Eq. 19 the wall value phi_s,i).
 */
#include "lbmref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D3Q19 velocity set and weights; D3Q7 is its first seven vectors. */
static const int CV[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double WG[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                              1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const double WH[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
static const double TG = 1.0 / 3.0; /* lattice temperature of D3Q19 */
static const double TH = 0.25;      /* lattice temperature of D3Q7 */

/* the phase-field lattice: its size, weights and temperature */
static int phase_Q(const lbmref_params *p) { return p->q_phase == 19 ? 19 : 7; }
static const double *phase_w(const lbmref_params *p) { return p->q_phase == 19 ? WG : WH; }
static double phase_T(const lbmref_params *p) { return p->q_phase == 19 ? TG : TH; }

enum { K_FLUID = 0, K_SOLID = 1, K_GHOST = 2 };

static int opposite(int i) {
    /* for every i > 0 the pair (odd, odd+1) holds opposite vectors */
    int o = 0;
    for (int j = 0; j < 19; ++j)
        if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2]) o = j;
    return o;
}

struct lbmref_state {
    lbmref_params p;
    int nx, ny, nz;
    long N;
    uint8_t *kind;   /* K_FLUID / K_SOLID / K_GHOST */
    uint8_t *mat;    /* material of solid nodes */
    int8_t *gface;   /* face of a ghost node */
    long *owner;     /* interior node one step inward from a ghost */
    double *nw;      /* [N*3] unit wall normal into the fluid, 0 without solid links */
    double *hyst;    /* [N*19] wall value each link used last (hysteresis), or NULL */
    double *qw;      /* [N*19] sub-voxel walls: fraction of link i from node n to the
                      * wall (0 < q <= 1), set at solid links only; NULL: voxel walls */
    double *gpre;    /* [N*19] incoming g of the current step (sub-voxel walls only) */
    double *h[2];    /* [N*Q] phase population i of node n at n*Q+i (Q = 7 or 19) */
    double *g[2];    /* [N*19] */
    int cur;
    double *phi, *rho, *u, *P, *grad, *lap, *mu;
    long step;
    int opp[19];
};

/* ---------------------------------------------------------------- indexing */
/* periodic wrap of a coordinate that is at most one period outside [0, n) */
static long wrap1(long v, long n) {
    if (v < 0) v += n;
    if (v >= n) v -= n;
    if (v < 0 || v >= n) { v %= n; if (v < 0) v += n; }
    return v;
}
static long node_of(const lbmref_state *s, long x, long y, long z) {
    x = wrap1(x, s->nx);
    y = wrap1(y, s->ny);
    z = wrap1(z, s->nz);
    return x + (long)s->nx * (y + (long)s->ny * z);
}
static void coords(const lbmref_state *s, long n, long *x, long *y, long *z) {
    long nxy = (long)s->nx * s->ny;
    *z = n / nxy;
    long r = n - *z * nxy;
    *y = r / s->nx;
    *x = r - *y * s->nx;
}
/* neighbour x + sgn*c_i with periodic wrap */
static long neighbour(const lbmref_state *s, long n, int i, int sgn) {
    long x, y, z;
    coords(s, n, &x, &y, &z);
    return node_of(s, x + sgn * CV[i][0], y + sgn * CV[i][1], z + sgn * CV[i][2]);
}

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

static double pressure_at_face(const lbmref_params *p, int f, long t) {
    return p->face_P[f] + p->face_ramp[f] * (double)t;
}

/* ------------------------------------------------ equilibrium building blocks */
/* Second-order Maxwellian weight Gamma_i (Sec. II.A, Eq. 3) for temperature T. */
static double gamma_i(double w, const int c[3], const double u[3], double T) {
    double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return w * (1.0 + cu / T + cu * cu / (2.0 * T * T) - uu / (2.0 * T));
}

static double density(const lbmref_params *p, double phi) {
    /* linear in the clamped order parameter (reading: phi = 1 is the liquid) */
    return p->rho_g + clamp01(phi) * (p->rho_l - p->rho_g);
}

static double chem_potential(const lbmref_params *p, double phi, double lap) {
    /* chemical potential, Eq. 9 */
    return 48.0 * p->sigma / p->W * phi * (phi - 1.0) * (phi - 0.5)
           - 1.5 * p->sigma * p->W * lap;
}

static double tau_mix(const lbmref_params *p, double phi) {
    /* Eqs. 10-12; the optimised model of Sec. III.A swaps F(phi) for a tanh step */
    double pb = clamp01(phi);
    double F = p->mix_tanh ? 0.5 * (tanh((pb - p->mix_phi) / p->mix_width) + 1.0) : pb;
    double tau_w = p->nu_l / TG + 0.5;
    double tau_a = p->nu_g / TG + 0.5;
    return (1.0 - F) * tau_a + F * tau_w;
}

void lbmref_geq_node(const lbmref_params *p, double phi, const double u[3], double P,
                     const double grad[3], double lap, double geq[19], double K[19]) {
    /* Eqs. 7-8: g_eq = rho Gamma + w (P/T - rho) - K/2 */
    double rho = density(p, phi);
    double rdif = p->rho_l - p->rho_g;
    double mu = chem_potential(p, phi, lap);
    for (int i = 0; i < 19; ++i) {
        double G = gamma_i(WG[i], CV[i], u, TG);
        double cg = 0.0, cf = 0.0;
        for (int a = 0; a < 3; ++a) {
            cg += (CV[i][a] - u[a]) * grad[a];
            cf += (CV[i][a] - u[a]) * p->F_ex[a];
        }
        K[i] = ((G - WG[i]) * rdif + G * mu / TG) * cg + G * cf / TG;
        geq[i] = rho * G + WG[i] * (P / TG - rho) - 0.5 * K[i];
    }
}

/* moments of the hydrodynamic populations (Sec. II.A, after Eq. 15): u first,
 * then P, which needs u */
static void hydro_moments(const lbmref_params *p, const double *g, double phi,
                          const double grad[3], double lap, double u[3], double *P) {
    double rho = density(p, phi);
    double mu = chem_potential(p, phi, lap);
    double rdif = p->rho_l - p->rho_g;
    double sum = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
        sum += g[i];
        for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * g[i];
    }
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * (mu * grad[a] + p->F_ex[a])) / rho;
    double ug = u[0] * grad[0] + u[1] * grad[1] + u[2] * grad[2];
    *P = TG * sum + 0.5 * TG * rdif * ug;
}

void lbmref_collide_g_node(const lbmref_params *p, const double g_in[19], double phi,
                           const double grad[3], double lap, double g_out[19],
                           double u[3], double *P) {
    /* S5 moments, then the filtered collision of Eqs. 13-15:
     *   g* = G_eq + (1 - 1/tau) Phi_i : Pi,  G_eq = g_eq + K  (BGK of Eq. 6 with
     *   its non-equilibrium part g - g_eq replaced by its second-order Hermite
     *   projection Phi_i = w_i (c c - T I) / (2 T^2),  Pi = sum c c (g - g_eq)). */
    double geq[19], K[19];
    hydro_moments(p, g_in, phi, grad, lap, u, P);
    lbmref_geq_node(p, phi, u, *P, grad, lap, geq, K);
    double Pi[3][3] = {{0}};
    for (int i = 0; i < 19; ++i) {
        double d = g_in[i] - geq[i];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Pi[a][b] += CV[i][a] * CV[i][b] * d;
    }
    double omega = 1.0 - 1.0 / tau_mix(p, phi);
    for (int i = 0; i < 19; ++i) {
        double contr = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                contr += (CV[i][a] * CV[i][b] - (a == b ? TG : 0.0)) * Pi[a][b];
        double phi_i = WG[i] / (2.0 * TG * TG) * contr;
        g_out[i] = geq[i] + K[i] + omega * phi_i;
    }
}

/* ------------------------------------------------------ mobility correction */
static double fclip(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

double lbmref_dtheta(const lbmref_params *p, double phi, double grad_norm, double lap) {
    /* Sec. II.A, Eq. 5 with Delta phi read as the Laplacian and the sign term
     * s = lap / (|lap| + eps). */
    if (!p->mobility_corr) return 0.0;
    double s = lap / (fabs(lap) + p->eps);
    double Y1 = fmin(fclip((phi - p->phi_M) / p->D), fclip((1.0 - phi) / p->D));
    double Y2 = fmin(fclip(phi / p->D), fclip((p->phi_m - phi) / p->D));
    return p->gamma * p->M / (phase_T(p) * p->W) * grad_norm * ((1.0 + s) * Y1 + (1.0 - s) * Y2);
}

/* ----------------------------------------------------------------- wetting */
void lbmref_wet_direction(const double n_w[3], const double g0[3], double theta_deg,
                          double eps, double w[3]) {
    /* Rotate the wall normal about n x grad(phi) by (pi - theta): the result is
     * -cos(theta) n + sin(theta) t, t the unit tangential part of grad(phi). */
    double th = theta_deg * M_PI / 180.0;
    double ng = n_w[0] * g0[0] + n_w[1] * g0[1] + n_w[2] * g0[2];
    double gt[3], tn = 0.0;
    for (int a = 0; a < 3; ++a) {
        gt[a] = g0[a] - n_w[a] * ng;
        tn += gt[a] * gt[a];
    }
    tn = sqrt(tn);
    for (int a = 0; a < 3; ++a) w[a] = -cos(th) * n_w[a] + sin(th) * gt[a] / (tn + eps);
}

double lbmref_wet_phi_s(double phi_smpl, const double w[3], const int c[3], double W,
                        double clamp_a) {
    /* Eqs. 17-19: invert the tanh profile at the sampled value, move by
     * d_i = w . c_i along the profile and evaluate it again. */
    double a = 2.0 * phi_smpl - 1.0;
    if (a > 1.0 - clamp_a) a = 1.0 - clamp_a;
    if (a < -1.0 + clamp_a) a = -1.0 + clamp_a;
    double x_x0 = 0.5 * W * atanh(a);
    double d = w[0] * c[0] + w[1] * c[1] + w[2] * c[2];
    return 0.5 * (1.0 + tanh((x_x0 + d) / (0.5 * W)));
}

/* S2 + S3 at fluid node n: gradient and Laplacian of phi with the wetting
 * substitute at solid links. */
/* What stencil() does with the hysteresis history of a node's wall links:
 * EVAL blends with it (read-out), STEP blends and stores (a time step), SET
 * stores the unblended value (initial state, restore).  What a step stores
 * is the reading of the blend: the blended value it used (hysteresis = 1,
 * the blend is recursive) or the unblended value from its own gradient
 * (hysteresis = 2, a blend of the current and the previous step's
 * gradient-derived values). */
enum { HYST_EVAL = 0, HYST_STEP = 1, HYST_SET = 2 };

static void stencil(lbmref_state *s, long n, double grad[3], double *lap, int hmode) {
    const lbmref_params *p = &s->p;
    double pc = s->phi[n];
    double ph[19];
    int sol[19];
    int any = 0;
    ph[0] = pc;
    sol[0] = 0;
    for (int i = 1; i < 19; ++i) {
        long m = neighbour(s, n, i, +1);
        sol[i] = (s->kind[m] == K_SOLID);
        ph[i] = sol[i] ? pc : s->phi[m]; /* neutral value for the pre-gradient */
        any |= sol[i];
    }
    if (any) {
        const double *nw = &s->nw[3 * n];
        double g0[3] = {0.0, 0.0, 0.0};
        for (int i = 1; i < 19; ++i)
            for (int a = 0; a < 3; ++a) g0[a] += (ph[i] - ph[s->opp[i]]) * CV[i][a] * WG[i];
        for (int a = 0; a < 3; ++a) g0[a] /= 2.0 * TG;
        for (int i = 1; i < 19; ++i) {
            if (!sol[i]) continue;
            long m = neighbour(s, n, i, +1);
            double w[3];
            lbmref_wet_direction(nw, g0, p->theta_deg[s->mat[m]], p->eps, w);
            ph[i] = lbmref_wet_phi_s(pc, w, CV[i], p->W, p->clamp_a);
            if (p->hysteresis) {
                double *prev = &s->hyst[19 * n + i];
                if (hmode == HYST_SET) {
                    *prev = ph[i];
                } else {
                    const double fresh = ph[i];
                    ph[i] = p->hyst_beta * (*prev) + (1.0 - p->hyst_beta) * fresh;
                    if (hmode == HYST_STEP) *prev = p->hysteresis == 2 ? fresh : ph[i];
                }
            }
        }
    }
    /* Eq. 16 as printed: gradient from the differences phi(x + c_i) - phi(x - c_i)
     * over all i (each +-c pair twice) divided by 2T; Laplacian from
     * phi(x + c_i) - phi(x) */
    double gsum[3] = {0.0, 0.0, 0.0}, l = 0.0;
    for (int i = 1; i < 19; ++i) {
        for (int a = 0; a < 3; ++a) gsum[a] += (ph[i] - ph[s->opp[i]]) * CV[i][a] * WG[i];
        l += (ph[i] - pc) * WG[i];
    }
    for (int a = 0; a < 3; ++a) grad[a] = gsum[a] / (2.0 * TG);
    *lap = 2.0 * l / TG;
}

/* phase-field equilibrium (Eqs. 2-4), theta including the correction of Eq. 5 */
static void heq_node(const lbmref_params *p, double phi, const double u[3],
                     const double grad[3], double lap, double heq[19]) {
    const int Q = phase_Q(p);
    const double *w = phase_w(p), T = phase_T(p);
    double gn = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    double nh[3];
    for (int a = 0; a < 3; ++a) nh[a] = grad[a] / (gn + p->eps);
    double theta = p->M / T * (1.0 - 4.0 * (phi - 0.5) * (phi - 0.5)) / p->W;
    theta += lbmref_dtheta(p, phi, gn, lap);
    for (int i = 0; i < Q; ++i) {
        double cn = CV[i][0] * nh[0] + CV[i][1] * nh[1] + CV[i][2] * nh[2];
        heq[i] = phi * gamma_i(w[i], CV[i], u, T) + theta * w[i] * cn;
    }
}

/* -------------------------------------------------------------- geometry */
static int classify(lbmref_state *s, const uint8_t *solid) {
    const lbmref_params *p = &s->p;
    for (long n = 0; n < s->N; ++n) {
        long x, y, z;
        coords(s, n, &x, &y, &z);
        long c[3] = {x, y, z};
        long dim[3] = {s->nx, s->ny, s->nz};
        s->gface[n] = -1;
        s->owner[n] = -1;
        if (solid && solid[n]) {
            if (solid[n] > 16) return -1;
            s->kind[n] = K_SOLID;
            s->mat[n] = (uint8_t)(solid[n] - 1);
            continue;
        }
        s->kind[n] = K_FLUID;
        s->mat[n] = 0;
        int nfaces = 0;
        for (int f = 0; f < 6; ++f) {
            if (!p->face_pressure[f]) continue;
            int ax = f / 2;
            long layer = (f % 2 == 0) ? 0 : dim[ax] - 1;
            if (c[ax] == layer) {
                ++nfaces;
                s->gface[n] = (int8_t)f;
            }
        }
        if (nfaces > 1) return -1; /* a ghost on two pressure faces has no single owner */
        if (nfaces == 1) s->kind[n] = K_GHOST;
    }
    for (long n = 0; n < s->N; ++n) {
        if (s->kind[n] != K_GHOST) continue;
        int f = s->gface[n];
        int ax = f / 2, sg = (f % 2 == 0) ? +1 : -1;
        long x, y, z;
        coords(s, n, &x, &y, &z);
        long c[3] = {x, y, z};
        c[ax] += sg;
        long o = node_of(s, c[0], c[1], c[2]);
        /* the ghost copies phi and u from its inward neighbour, which must be
         * a fluid node (a face ghost next to a solid node is rejected) */
        if (s->kind[o] != K_FLUID) return -1;
        s->owner[n] = o;
    }
    /* wall normal: -sum of w_i c_i over solid links, normalised (voxel walls) */
    for (long n = 0; n < s->N; ++n) {
        double v[3] = {0.0, 0.0, 0.0};
        if (s->kind[n] == K_FLUID) {
            for (int i = 1; i < 19; ++i) {
                long m = neighbour(s, n, i, +1);
                if (s->kind[m] == K_SOLID)
                    for (int a = 0; a < 3; ++a) v[a] -= WG[i] * CV[i][a];
            }
        }
        double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int a = 0; a < 3; ++a) s->nw[3 * n + a] = nv > 0.0 ? v[a] / nv : 0.0;
    }
    return 0;
}

/* ghost populations: equilibrium at the owner's phi and u and the face
 * pressure, without forcing and without the counter-term */
static void ghost_fill(lbmref_state *s, double *hdst, double *gdst, long t) {
    const lbmref_params *p = &s->p;
#pragma omp parallel for schedule(static) if (s->N >= 16384)
    for (long n = 0; n < s->N; ++n) {
        if (s->kind[n] != K_GHOST) continue;
        const int Q = phase_Q(p);
        const double *w = phase_w(p), T = phase_T(p);
        double *h = &hdst[(long)Q * n], *g = &gdst[19 * n];
        long o = s->owner[n];
        if (o < 0) {
            for (int i = 0; i < Q; ++i) h[i] = 0.0;
            for (int i = 0; i < 19; ++i) g[i] = 0.0;
            continue;
        }
        double ph = s->phi[o];
        const double *u = &s->u[3 * o];
        double rho = density(p, ph);
        double Pb = pressure_at_face(p, s->gface[n], t);
        for (int i = 0; i < Q; ++i) h[i] = ph * gamma_i(w[i], CV[i], u, T);
        for (int i = 0; i < 19; ++i)
            g[i] = rho * gamma_i(WG[i], CV[i], u, TG) + WG[i] * (Pb / TG - rho);
    }
}

/* S1: order parameter on fluid nodes, then Neumann copy to ghosts */
static void phase_moment(lbmref_state *s) {
    const double *h = s->h[s->cur];
    const int Q = phase_Q(&s->p);
#pragma omp parallel for schedule(static) if (s->N >= 16384)
    for (long n = 0; n < s->N; ++n) {
        double v = 0.0;
        if (s->kind[n] == K_FLUID)
            for (int i = 0; i < Q; ++i) v += h[(long)Q * n + i];
        s->phi[n] = v;
    }
#pragma omp parallel for schedule(static) if (s->N >= 16384)
    for (long n = 0; n < s->N; ++n)
        if (s->kind[n] == K_GHOST) s->phi[n] = s->owner[n] >= 0 ? s->phi[s->owner[n]] : 0.0;
}

/* S2-S5 on every fluid node from the current populations (no collision) */
static void macroscopic(lbmref_state *s) {
    const lbmref_params *p = &s->p;
    const double *g = s->g[s->cur];
    phase_moment(s);
#pragma omp parallel for schedule(static) if (s->N >= 16384)
    for (long n = 0; n < s->N; ++n) {
        if (s->kind[n] != K_FLUID) continue;
        double grad[3], lap, u[3], P;
        stencil(s, n, grad, &lap, HYST_EVAL);
        hydro_moments(p, &g[19 * n], s->phi[n], grad, lap, u, &P);
        for (int a = 0; a < 3; ++a) {
            s->u[3 * n + a] = u[a];
            s->grad[3 * n + a] = grad[a];
        }
        s->P[n] = P;
        s->lap[n] = lap;
        s->rho[n] = density(p, s->phi[n]);
    }
}

/* ------------------------------------------------------------------- API */
/* Sub-voxel walls from a signed distance to the wall surface (positive in
 * the fluid, the solid nodes at <= 0).  The link from fluid node x to solid
 * node x + c_i crosses the surface at the fraction
 *     q = sdf(x) / (sdf(x) - sdf(x + c_i))
 * of its length (linear interpolation of the distance along the link), and
 * the wall normal into the fluid is the normalised gradient of sdf by the
 * central differences of Eq. 16.  Invalid (-1): a fluid node with a solid
 * link whose distances do not straddle the surface. */
static int walls_from_sdf(lbmref_state *s, const double *sdf) {
    for (long n = 0; n < s->N; ++n) {
        if (s->kind[n] != K_FLUID) continue;
        int any = 0;
        for (int i = 1; i < 19; ++i) {
            long m = neighbour(s, n, i, +1);
            if (s->kind[m] != K_SOLID) continue;
            any = 1;
            double a = sdf[n], b = sdf[m];
            if (!(a > 0.0) || !(b <= 0.0)) return -1;
            s->qw[19 * n + i] = a / (a - b);
        }
        if (!any) continue;
        double gs[3] = {0.0, 0.0, 0.0};
        for (int i = 1; i < 19; ++i) {
            double d = sdf[neighbour(s, n, i, +1)] - sdf[neighbour(s, n, i, -1)];
            for (int a = 0; a < 3; ++a) gs[a] += d * CV[i][a] * WG[i];
        }
        double gn = sqrt(gs[0] * gs[0] + gs[1] * gs[1] + gs[2] * gs[2]);
        if (gn > 0.0)
            for (int a = 0; a < 3; ++a) s->nw[3 * n + a] = gs[a] / gn;
    }
    return 0;
}

lbmref_state *lbmref_create(const lbmref_params *p, const uint8_t *solid, const double *sdf,
                            const double *phi0, const double *u0, const double *P0) {
    if (!p || !phi0 || p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
    if (p->W <= 0.0 || p->M <= 0.0 || p->rho_l <= 0.0 || p->rho_g <= 0.0) return NULL;
    if (p->nu_l <= 0.0 || p->nu_g <= 0.0) return NULL;
    lbmref_state *s = (lbmref_state *)calloc(1, sizeof(*s));
    if (!s) return NULL;
    s->p = *p;
    s->nx = p->nx; s->ny = p->ny; s->nz = p->nz;
    s->N = (long)p->nx * p->ny * p->nz;
    long N = s->N;
    for (int i = 0; i < 19; ++i) s->opp[i] = opposite(i);
    s->kind = malloc(N); s->mat = malloc(N); s->gface = malloc(N);
    s->owner = malloc(N * sizeof(long));
    s->nw = malloc(3 * N * sizeof(double));
    s->hyst = p->hysteresis ? calloc(19 * N, sizeof(double)) : NULL;
    s->qw = sdf ? calloc(19 * N, sizeof(double)) : NULL;
    s->gpre = sdf ? calloc(19 * N, sizeof(double)) : NULL;
    for (int k = 0; k < 2; ++k) {
        s->h[k] = calloc((long)phase_Q(p) * N, sizeof(double));
        s->g[k] = calloc(19 * N, sizeof(double));
    }
    s->phi = calloc(N, sizeof(double)); s->rho = calloc(N, sizeof(double));
    s->u = calloc(3 * N, sizeof(double)); s->P = calloc(N, sizeof(double));
    s->grad = calloc(3 * N, sizeof(double)); s->lap = calloc(N, sizeof(double));
    s->mu = calloc(N, sizeof(double));
    if (!s->kind || !s->mat || !s->gface || !s->owner || !s->nw || (p->hysteresis && !s->hyst) ||
        (sdf && (!s->qw || !s->gpre)) ||
        !s->h[0] || !s->h[1] ||
        !s->g[0] || !s->g[1] || !s->phi || !s->rho || !s->u || !s->P || !s->grad ||
        !s->lap || !s->mu) {
        lbmref_destroy(s);
        return NULL;
    }
    if (classify(s, solid) != 0 || (sdf && walls_from_sdf(s, sdf) != 0)) {
        lbmref_destroy(s);
        return NULL;
    }
    /* S0: phi0 on fluid nodes, Neumann copy on ghosts; equilibria everywhere */
    for (long n = 0; n < N; ++n) s->phi[n] = (s->kind[n] == K_FLUID) ? phi0[n] : 0.0;
    for (long n = 0; n < N; ++n)
        if (s->kind[n] == K_GHOST && s->owner[n] >= 0) s->phi[n] = s->phi[s->owner[n]];
    double *h = s->h[0], *g = s->g[0];
#pragma omp parallel for schedule(static) if (s->N >= 16384)
    for (long n = 0; n < N; ++n) {
        if (s->kind[n] != K_FLUID) continue;
        double grad[3], lap, u[3], P;
        stencil(s, n, grad, &lap, HYST_SET);
        for (int a = 0; a < 3; ++a) u[a] = u0 ? u0[a * N + n] : 0.0;
        P = P0 ? P0[n] : p->P_ref;
        double heq[19], geq[19], K[19];
        heq_node(p, s->phi[n], u, grad, lap, heq);
        lbmref_geq_node(p, s->phi[n], u, P, grad, lap, geq, K);
        for (int i = 0; i < phase_Q(p); ++i) h[(long)phase_Q(p) * n + i] = heq[i];
        for (int i = 0; i < 19; ++i) g[19 * n + i] = geq[i];
        for (int a = 0; a < 3; ++a) s->u[3 * n + a] = u[a];
    }
    s->cur = 0;
    s->step = 0;
    return s;
}

void lbmref_destroy(lbmref_state *s) {
    if (!s) return;
    free(s->kind); free(s->mat); free(s->gface); free(s->owner); free(s->nw); free(s->hyst);
    free(s->qw); free(s->gpre);
    for (int k = 0; k < 2; ++k) { free(s->h[k]); free(s->g[k]); }
    free(s->phi); free(s->rho); free(s->u); free(s->P); free(s->grad); free(s->lap);
    free(s->mu);
    free(s);
}

long lbmref_step_count(const lbmref_state *s) { return s->step; }

void lbmref_kinds(const lbmref_state *s, uint8_t *kind) { memcpy(kind, s->kind, s->N); }

static void one_step(lbmref_state *s) {
    const lbmref_params *p = &s->p;
    long N = s->N;
    double *hA = s->h[s->cur], *gA = s->g[s->cur];
    double *hB = s->h[1 - s->cur], *gB = s->g[1 - s->cur];
    phase_moment(s); /* S1 */
    if (s->gpre) memcpy(s->gpre, gA, 19 * N * sizeof(double));
    /* S2-S7: collide every fluid node in place in lattice A */
#pragma omp parallel for schedule(static) if (s->N >= 16384)
    for (long n = 0; n < N; ++n) {
        if (s->kind[n] != K_FLUID) continue;
        double grad[3], lap, u[3], P, gout[19], heq[19];
        stencil(s, n, grad, &lap, HYST_STEP);
        double ph = s->phi[n];
        lbmref_collide_g_node(p, &gA[19 * n], ph, grad, lap, gout, u, &P);
        heq_node(p, ph, u, grad, lap, heq);
        const int Q = phase_Q(p);
        double tau_h = p->M / phase_T(p) + 0.5;
        for (int i = 0; i < Q; ++i) hA[(long)Q * n + i] -= (hA[(long)Q * n + i] - heq[i]) / tau_h;
        for (int i = 0; i < 19; ++i) gA[19 * n + i] = gout[i];
        for (int a = 0; a < 3; ++a) s->u[3 * n + a] = u[a];
        s->rho[n] = density(p, ph);
        s->P[n] = P;
    }
    /* S9: ghost populations streaming out at this step: equilibrium at the
     * owners' phi and u of this step and the face pressure of step t+1 (a
     * one-step lag in phi and u; ghosts are never collided) */
    ghost_fill(s, hA, gA, s->step + 1);
    /* S8: pull into lattice B */
    const int Qh = phase_Q(p);
#pragma omp parallel for schedule(static) if (s->N >= 16384)
    for (long y = 0; y < N; ++y) {
        if (s->kind[y] != K_FLUID) continue;
        /* wall velocity seen by the slip bounce-back: the tangential fluid
         * velocity times slip_factor inside the interface band (1: free
         * slip), zero elsewhere */
        double uw[3] = {0.0, 0.0, 0.0};
        double ph = s->phi[y];
        if (p->interface_slip && ph >= p->slip_lo && ph <= p->slip_hi) {
            const double *nw = &s->nw[3 * y], *u = &s->u[3 * y];
            double un = nw[0] * u[0] + nw[1] * u[1] + nw[2] * u[2];
            for (int a = 0; a < 3; ++a) uw[a] = p->slip_factor * (u[a] - nw[a] * un);
        }
        for (int i = 0; i < 19; ++i) {
            long x = neighbour(s, y, i, -1);
            int io = s->opp[i];
            double gv;
            if (s->kind[x] == K_SOLID) {
                /* the population g*_io(y) sent toward the wall comes back as
                 * g_i(y); a wall moving with u_w adds -2 w rho c.u_w / T */
                double cu = CV[io][0] * uw[0] + CV[io][1] * uw[1] + CV[io][2] * uw[2];
                double mw = 2.0 * WG[io] * s->rho[y] * cu / TG;
                if (!s->qw) {
                    gv = gA[19 * y + io] - mw;
                } else {
                    /* linear interpolated bounce-back (Bouzidi, Firdaouss and
                     * Lallemand 2001) with the wall at fraction q of the link.
                     * q >= 1/2: between g*_io(y) and g*_i(y); the moving-wall
                     * term scales by 1/(2q).  q < 1/2: between g*_io(y) and the
                     * population g*_io(y - c_io) one link upstream.  Default:
                     * the one that arrived at y along io at this step stands in
                     * for it (its value a step earlier: exact for a steady
                     * flow, and local).  subvoxel_same_step: the upstream
                     * node's value of this step, or the half-way rule where
                     * that node is solid. */
                    double q = s->qw[19 * y + io];
                    if (q >= 0.5) {
                        gv = gA[19 * y + io] / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * gA[19 * y + i] -
                             mw / (2.0 * q);
                    } else if (p->subvoxel_same_step) {
                        long up = neighbour(s, y, i, +1);
                        if (s->kind[up] == K_SOLID)
                            gv = gA[19 * y + io] - mw;
                        else
                            gv = 2.0 * q * gA[19 * y + io] + (1.0 - 2.0 * q) * gA[19 * up + io] - mw;
                    } else {
                        gv = 2.0 * q * gA[19 * y + io] + (1.0 - 2.0 * q) * s->gpre[19 * y + io] - mw;
                    }
                }
                if (i < Qh) hB[(long)Qh * y + i] = hA[(long)Qh * y + io];
            } else {
                gv = gA[19 * x + i];
                if (i < Qh) hB[(long)Qh * y + i] = hA[(long)Qh * x + i];
            }
            gB[19 * y + i] = gv;
        }
    }
    /* S10 */
    s->cur = 1 - s->cur;
    s->step += 1;
}

void lbmref_step(lbmref_state *s, long nsteps) {
    for (long k = 0; k < nsteps; ++k) one_step(s);
}

void lbmref_fields(lbmref_state *s, double *phi, double *P, double *u) {
    long N = s->N;
    macroscopic(s);
    for (long n = 0; n < N; ++n) {
        int k = s->kind[n];
        double pv = 0.0, Pv = 0.0, uv[3] = {0.0, 0.0, 0.0};
        if (k == K_FLUID) {
            pv = s->phi[n];
            Pv = s->P[n];
            for (int a = 0; a < 3; ++a) uv[a] = s->u[3 * n + a];
        } else if (k == K_GHOST) {
            pv = s->phi[n];
            Pv = pressure_at_face(&s->p, s->gface[n], s->step);
        }
        if (phi) phi[n] = pv;
        if (P) P[n] = Pv;
        if (u)
            for (int a = 0; a < 3; ++a) u[a * N + n] = uv[a];
    }
}

void lbmref_pops(const lbmref_state *s, double *h, double *g) {
    long N = s->N;
    const double *hA = s->h[s->cur], *gA = s->g[s->cur];
    for (long n = 0; n < N; ++n) {
        int fl = (s->kind[n] == K_FLUID);
        if (h)
            for (int i = 0; i < phase_Q(&s->p); ++i) h[i * N + n] = fl ? hA[(long)phase_Q(&s->p) * n + i] : 0.0;
        if (g)
            for (int i = 0; i < 19; ++i) g[i * N + n] = fl ? gA[19 * n + i] : 0.0;
    }
}

void lbmref_set_pops(lbmref_state *s, const double *h, const double *g, long step) {
    long N = s->N;
    double *hA = s->h[s->cur], *gA = s->g[s->cur];
    for (long n = 0; n < N; ++n) {
        if (s->kind[n] != K_FLUID) continue;
        for (int i = 0; i < phase_Q(&s->p); ++i) hA[(long)phase_Q(&s->p) * n + i] = h[i * N + n];
        for (int i = 0; i < 19; ++i) gA[19 * n + i] = g[i * N + n];
    }
    s->step = step;
    if (s->p.hysteresis) {
        /* the history of the wall values restarts from the restored state */
        phase_moment(s);
        for (long n = 0; n < N; ++n) {
            if (s->kind[n] != K_FLUID) continue;
            double grad[3], lap;
            stencil(s, n, grad, &lap, HYST_SET);
        }
    }
}

void lbmref_diagnostics(lbmref_state *s, lbmref_diag *d) {
    long N = s->N;
    macroscopic(s);
    memset(d, 0, sizeof(*d));
    double Pl = 0.0, Pg = 0.0;
    for (long n = 0; n < N; ++n) {
        if (s->kind[n] != K_FLUID) continue;
        double ph = s->phi[n], rho = s->rho[n], P = s->P[n];
        const double *u = &s->u[3 * n];
        double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        if (isnan(ph) || isnan(P) || isnan(um)) { d->n_nan++; continue; }
        d->phi_sum += ph;
        for (int a = 0; a < 3; ++a) d->mom[a] += rho * u[a];
        if (um > d->u_max) d->u_max = um;
        if (ph > 0.99) { Pl += P; d->n_liq++; }
        if (ph < 0.01) { Pg += P; d->n_gas++; }
    }
    d->P_liq_mean = d->n_liq ? Pl / d->n_liq : 0.0;
    d->P_gas_mean = d->n_gas ? Pg / d->n_gas : 0.0;
}
