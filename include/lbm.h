/*
 * lbm.h -- C ABI of the MI355X phase-field lattice Boltzmann library.
 *
 * The library advances the conservative Allen-Cahn phase-field LB method of
 * Thirumalaisamy, Kim, Otomo, Jilesen and Zhang, "Capillary flow simulation
 * with the phase-field-based lattice Boltzmann solver" (AIP accepted
 * manuscript, 2025), on one AMD Instinct MI355X (gfx950):
 *
 *   phase field  h_i  on D3Q7  (T = 1/4): BGK towards phi*Gamma_i + theta w_i c_i.n,
 *                theta with the local mobility correction      (Sec. II.A, Eqs. 1-5)
 *   hydrodynamics g_i on D3Q19 (T = 1/3): filtered collision with the forcing
 *                K_i (phase separation, surface tension, body force)
 *                                                              (Sec. II.A, Eqs. 6-15)
 *   gradient and Laplacian of phi from the 18 nearest neighbours (Eq. 16)
 *   wetting at voxel walls: phi_s,i from the tanh profile along the rotated
 *                normal w                                      (Sec. II.B, Eqs. 17-19)
 *   friction: half-way bounce-back, free slip inside 0.5 <= phi <= 0.95 for
 *                the optimised model, or a partial slip there   (Sec. III.A)
 *   pressure faces: Dirichlet P, Neumann u and phi              (Sec. III.A)
 *
 * Equation numbers count every numbered display of the paper in order.
 *
 * Conventions
 *   Node index n = x + nx*(y + ny*z).  Scalar fields are arrays of N doubles,
 *   vector fields [3][N] (all x components, then y, then z), populations
 *   [Q][N].  Lattice order of the populations (a D3Q7 phase field uses the
 *   first 7):
 *     0:(0,0,0) 1:(+1,0,0) 2:(-1,0,0) 3:(0,+1,0) 4:(0,-1,0) 5:(0,0,+1) 6:(0,0,-1)
 *     7:(+1,+1,0) 8:(-1,-1,0) 9:(+1,-1,0) 10:(-1,+1,0) 11:(+1,0,+1) 12:(-1,0,-1)
 *     13:(+1,0,-1) 14:(-1,0,+1) 15:(0,+1,+1) 16:(0,-1,-1) 17:(0,+1,-1) 18:(0,-1,+1)
 *   phi = 1 is the heavy (liquid) phase.  All coordinates are periodic unless a
 *   face is a pressure face; walls are solid nodes given in the geometry.
 *
 * Errors: every call returns LBM_OK (0) or a negative code; lbm_last_error()
 * returns a thread-local message describing the last failure on the calling
 * thread.  No C++ exception crosses this interface.
 */
#ifndef MI355X_PFLBM_LBM_H
#define MI355X_PFLBM_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_PENDING 1       /* lbm_poll: request not finished yet */
#define LBM_E_INVAL (-1)    /* invalid argument or parameter */
#define LBM_E_NOMEM (-2)    /* device or host allocation failed */
#define LBM_E_DEVICE (-3)   /* HIP runtime error */
#define LBM_E_UNSTABLE (-4) /* NaN or |u| above u_max seen by a diagnostic step */
#define LBM_E_STATE (-5)    /* call not valid in the object's current state */

/* population storage (arithmetic is FP64 for LBM_FP64, FP32 otherwise) */
enum lbm_storage {
    LBM_FP64 = 0,           /* plain doubles */
    LBM_FP32 = 1,           /* plain floats */
    LBM_FP32_SHIFT = 2,     /* floats holding f_i - w_i f_ref */
    LBM_FP16_SHIFT_G = 3,   /* h as shifted floats, g as scaled shifted halves */
    LBM_FP16_SHIFT_ALL = 4  /* h and g as scaled shifted halves: rejected (LBM_E_INVAL).
                               phi = sum h_i carries the rounding of 11-bit h deviations
                               (~1e-4 per step), which the counter-term of Eqs. 2-4 and
                               the mobility correction of Eq. 5 amplify to phi errors of
                               ~1e-1: no error bound can be stated for it */
};

enum lbm_face_bc { LBM_BC_PERIODIC = 0, LBM_BC_PRESSURE = 1 };
enum lbm_mix { LBM_MIX_LINEAR = 0, LBM_MIX_TANH = 1 };
/* friction at walls (Sec. III.A): half-way bounce-back (no slip) everywhere;
 * or inside slip_lo <= phi <= slip_hi a moving-wall bounce-back whose wall
 * velocity is the node's tangential fluid velocity (free slip, the optimised
 * model) or slip_factor times it (partial slip, a variant between the two) */
enum lbm_friction {
    LBM_FRICTION_NOSLIP = 0,
    LBM_FRICTION_INTERFACE_SLIP = 1,
    LBM_FRICTION_PARTIAL_SLIP = 2
};

/* Problem statement (Sec. II, Sec. III.A).  All values in lattice units. */
typedef struct lbm_params {
    int32_t nx, ny, nz;     /* lattice size; each >= 1, N = nx*ny*nz < 2^31 */
    int32_t storage;        /* enum lbm_storage */
    double rho_l, rho_g;    /* densities of the phi = 1 and phi = 0 phases, > 0 */
    double nu_l, nu_g;      /* kinematic viscosities, > 0 (tau = nu/T + 1/2) */
    double sigma;           /* surface tension, >= 0 */
    double W;               /* interface width, > 0 */
    double M;               /* mobility, > 0 */
    double F_ex[3];         /* body force per unit volume */
    int32_t mobility_corr;  /* 1: add delta-theta of Eq. 5 */
    double mc_gamma, mc_phi_M, mc_phi_m, mc_D;
    double eps;             /* epsilon of n = grad/(|grad|+eps) and of the sign term */
    int32_t mix;            /* enum lbm_mix: F(phi) = phi or 0.5[tanh((phi-mix_phi)/mix_width)+1] */
    double mix_phi, mix_width;
    int32_t friction;       /* enum lbm_friction */
    double slip_lo, slip_hi;/* free-slip band of the interface-slip friction */
    double P_ref;           /* reference pressure; shifted storage keeps g_i - w_i P_ref/T */
    int32_t face_bc[6];     /* faces x-, x+, y-, y+, z-, z+; enum lbm_face_bc */
    double face_P[6];       /* pressure face: P(t) = face_P + face_ramp * t */
    double face_ramp[6];
    int32_t diag_every;     /* >0: FP64 diagnostics and the stability check every k steps */
    double u_max;           /* stability limit on |u| (<= 0: NaN check only) */
    int32_t fp16_log2_scale_h; /* unused (h is never stored in FP16); kept for the layout */
    int32_t fp16_log2_scale_g; /* FP16 storage scale 2^k of g deviations (0: default) */
    int32_t hysteresis;     /* contact-angle hysteresis of the optimised model (Sec. III.A):
                               each wall link uses hyst_beta * (a value kept from the
                               previous step) + (1 - hyst_beta) * (the value from the
                               current gradient).  0: off.  1: the kept value is the blended
                               value the previous step used (recursive blend).  2: it is the
                               previous step's unblended, gradient-derived value.  The history
                               starts from the current values at creation and after a
                               restore.  Other values: LBM_E_INVAL */
    double hyst_beta;       /* blend factor in [0, 1) (the paper's 0.95) */
    int32_t q_phase;        /* phase-field lattice: 7 (D3Q7, T = 1/4, the default; 0 means 7)
                               or 19 (D3Q19 with the hydrodynamic weights, T = 1/3, the
                               lattice Sec. II names for Eq. 2); any other value: LBM_E_INVAL */
    int32_t subvoxel;       /* 0: voxel walls, half-way between fluid and solid nodes.
                               1: sub-voxel walls (walls off the lattice, Sec. IV.A offsets
                               and inclined or curved walls) given by lbm_geometry.sdf: g
                               takes the linear interpolated bounce-back at each link's wall
                               fraction and the wall normal is the distance gradient; h keeps
                               the half-way rule (exact phi mass).  Other values: LBM_E_INVAL */
    double slip_factor;     /* friction = LBM_FRICTION_PARTIAL_SLIP only: the wall velocity in
                               the slip band as a fraction of the tangential fluid velocity,
                               in [0, 1] (0: no slip, 1: the free slip); else LBM_E_INVAL.
                               Ignored for the other friction models */
} lbm_params;

/* Geometry.  solid[n] = 0: fluid; 1 + k: solid of material k (< 16).
 * Non-solid nodes on a pressure-face layer become pressure ghosts; a ghost may
 * lie on one pressure face only and its inward neighbour must be fluid.
 * solid may be NULL (no walls). theta_deg[k] in (0, 180): contact angle of
 * material k, measured through the phi = 1 phase (Sec. II.B).
 * sdf[N] (only with lbm_params.subvoxel = 1, else NULL): signed distance to
 * the wall surface, > 0 at every fluid node with a solid neighbour and <= 0
 * at those solid neighbours; the link from fluid x to solid x + c_i crosses
 * the wall at q = sdf(x) / (sdf(x) - sdf(x + c_i)) of its length.  A pair that
 * does not straddle the surface: LBM_E_INVAL.  Host memory, read during
 * lbm_create / lbm_submit only. */
typedef struct lbm_geometry {
    const uint8_t *solid;
    double theta_deg[16];
    const double *sdf;
} lbm_geometry;

enum lbm_init_kind { LBM_INIT_FIELDS = 0, LBM_INIT_POPULATIONS = 1 };

/* Initial state.  FIELDS: phi[N] required, u[3][N] may be NULL (0), P[N] may
 * be NULL (P_ref); populations are set to their equilibria with the wetting
 * stencil applied (h with the counter-term, g with K_i).  POPULATIONS: pops =
 * h[q_phase][N] followed by g[19][N] as returned by lbm_read_fields(LBM_POP_H |
 * LBM_POP_G) and step = the step they belong to (restore). Host memory, read
 * during the call only. */
typedef struct lbm_init {
    int32_t kind;
    const double *phi;
    const double *u;
    const double *P;
    const double *pops;
    int64_t step;
} lbm_init;

/* Device context.  arena: optional caller-owned device memory of
 * arena_bytes >= lbm_footprint(); it must outlive the handle.  NULL: the
 * library allocates.  stream: a hipStream_t the handle's work is queued on
 * (NULL: the null stream).  device: HIP device ordinal. */
typedef struct lbm_device_ctx {
    void *arena;
    size_t arena_bytes;
    void *stream;
    int32_t device;
} lbm_device_ctx;

/* FP64 diagnostics over fluid nodes at the step they were taken. */
typedef struct lbm_diag {
    int64_t step;
    double phi_sum;         /* sum of phi (the conserved mass of Eq. 1) */
    double mom[3];          /* sum of rho u */
    double u_max;           /* max |u| */
    double P_liq_mean;      /* mean P over phi > 0.99 */
    double P_gas_mean;      /* mean P over phi < 0.01 */
    int64_t n_nan, n_liq, n_gas;
} lbm_diag;

typedef struct lbm_handle lbm_handle;

/* Bytes of device memory one lattice needs (populations, phi, flags, tile
 * table, reduction partials and the near-wall arrays).  0 if the parameters
 * are invalid, including a lattice whose populations exceed what 32-bit
 * offsets address: populations are stored in blocks of 64 nodes with rows
 * padded to 64 nodes, in one group of at most 4 GiB while a node's
 * populations take at most 104 bytes, else in two (about 41 M nodes in FP32
 * or FP64 on D3Q7).  The near-wall arrays (and the hysteresis history) are
 * sized as if every node had wall links (the geometry is not known here): an
 * upper bound; lbm_create allocates the exact amount when it allocates
 * itself. */
size_t lbm_footprint(const lbm_params *p);

/* Validate, allocate (or carve the arena), upload geometry and initial state
 * and build the tile table.  Synchronous.  Errors: LBM_E_INVAL (tau <= 1/2,
 * W <= 0, rho <= 0, bad angle, ghost rules, N too large, no fluid node; the
 * geometry is checked before any device call), LBM_E_NOMEM, LBM_E_DEVICE. */
int lbm_create(const lbm_params *p, const lbm_geometry *geo, const lbm_init *init,
               const lbm_device_ctx *ctx, lbm_handle **out);

/* Queue nsteps time steps on the handle's stream and return.  Each step is
 * the phi pass, the wall pass (wetting values and stencil sums of the
 * near-wall nodes, Sec. II.B), the fused stream-collide sweep (Sec. II.A,
 * Eqs. 1-16), the pressure-face ghosts (Sec. III.A) and the step counter.
 * The steps are replayed from HIP graphs captured at the first call (one
 * step per AA parity and diagnostic kind, and 16-step runs without a
 * diagnostic step); while timing is on (lbm_set_timing) every kernel is
 * launched on its own between events instead.  Both give bitwise the same
 * state.  Returns LBM_E_UNSTABLE if a diagnostic taken before this call
 * flagged NaN or |u| > u_max (sticky). */
int lbm_step(lbm_handle *h, int64_t nsteps);

/* Wait for queued work. */
int lbm_sync(lbm_handle *h);

/* Number of steps taken (queued) so far. */
int64_t lbm_step_count(const lbm_handle *h);

#define LBM_PHI 1u
#define LBM_P 2u
#define LBM_U 4u
#define LBM_POP_H 8u
#define LBM_POP_G 16u
/* Synchronous read-back to caller-owned host buffers (NULL skips a field).
 * phi[N], P[N], u[3][N]: macroscopic fields of the current step, evaluated
 * from the populations entering its collision (after the text of Eq. 15).
 * Solid nodes read 0; ghosts read the owner's phi, the face pressure and 0.
 * Allocates device staging for the requested fields for the duration of the
 * call (LBM_E_DEVICE if that fails).
 * pops: h[q_phase][N] (if LBM_POP_H) then g[19][N] (if LBM_POP_G), decoded to double,
 * the value f_i(x) entering the collision; 0 at solid and ghost nodes. */
int lbm_read_fields(lbm_handle *h, uint32_t mask, double *phi, double *P, double *u,
                    double *pops);

/* lbm_read_fields for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same read-back and result, staged through one fixed array
 * of LBM_NOALLOC_MAX_DOUBLES doubles (64 MiB) that the library holds on
 * every GPU it runs on until the process ends, so the call allocates
 * nothing.  The requested fields must fit it: N doubles each for phi and P,
 * 3 N for u, (q_phase + 19) N for pops with LBM_POP_H or LBM_POP_G (all
 * population rows are staged); larger requests return LBM_E_INVAL before
 * any device work.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (from several threads, on any handles) race and must be
 * serialised by the caller.  Synchronous. */
#define LBM_NOALLOC_MAX_DOUBLES (8u << 20)
int lbm_read_fields_noalloc(lbm_handle *h, uint32_t mask, double *phi, double *P, double *u,
                            double *pops);

/* FP64 reduction of the current state (Sigma phi, Sigma rho u, max |u|, mean
 * pressures).  Synchronous. */
int lbm_reduce(lbm_handle *h, lbm_diag *d);

/* Optional per-kernel timing with HIP events on the handle's stream: while on,
 * lbm_step launches each kernel on its own and records events around them;
 * lbm_get_timing returns the accumulated milliseconds of the phi pass with
 * the wall pass, and of the sweep kernel alone (the ghost and step-counter
 * kernels that follow it are not bracketed), and the number of steps timed,
 * and resets them. */
int lbm_set_timing(lbm_handle *h, int32_t on);
int lbm_get_timing(lbm_handle *h, double *phi_ms, double *sweep_ms, int64_t *steps);

/* Free device memory (not a caller arena).  Synchronises first. */
int lbm_destroy(lbm_handle *h);

const char *lbm_last_error(void);

/* Counters describing one lattice, for throughput accounting. */
typedef struct lbm_info {
    int64_t n_nodes, n_fluid, n_ghost, n_solid;
    int64_t n_tiles;
    size_t footprint;
    double bytes_per_fluid_update;   /* population bytes read + written per fluid node */
} lbm_info;
int lbm_get_info(const lbm_handle *h, lbm_info *info);

/* ------------------------------------------------------------------ serving
 * Continuous batching of many independent lattices on one GPU: requests are
 * admitted when their footprint fits the HBM budget and a slot is free, every
 * admitted lattice advances one step per tick in one batched phi pass and one
 * batched sweep over a device table of (lattice, tile) work items, and
 * finished lattices are read back and their memory reused. */
typedef struct lbm_server_cfg {
    size_t hbm_budget;       /* bytes of device memory for lattices (0: 80% of free) */
    int32_t max_slots;       /* lattices resident at once (<= 256) */
    int32_t storage;         /* enum lbm_storage used by every request */
    int32_t device;
    int32_t use_graph;       /* 1: replay each scheduling interval from a captured hipGraph */
    int32_t ticks_per_sync;  /* steps per scheduling interval, rounded up to even (0: 32) */
    int64_t max_resident_nodes; /* admission also waits while the resident lattices hold more
                                   nodes than this, unless none is resident (0: no limit) */
} lbm_server_cfg;

typedef struct lbm_request {
    lbm_params params;       /* storage is overridden by the server's */
    lbm_geometry geometry;
    lbm_init init;           /* LBM_INIT_FIELDS only */
    int64_t nsteps;          /* steps to run, >= 1 */
    double arrival_s;        /* caller timestamp, reported back */
} lbm_request;

typedef struct lbm_result {
    int32_t status;          /* LBM_OK or the request's error */
    int64_t nx, ny, nz;
    double *phi, *P, *u;     /* library-owned host arrays; free with lbm_result_free */
    lbm_diag diag;           /* diagnostics of the final state */
    double t_submit_s, t_admit_s, t_finish_s;  /* library clock (seconds since server creation) */
    int64_t steps;
} lbm_result;

typedef struct lbm_server lbm_server;

int lbm_server_create(const lbm_server_cfg *cfg, lbm_server **out);
/* Copy the request (host arrays are read during the call) and queue it.
 * Thread-safe; returns at once with a ticket.  LBM_E_INVAL if its footprint
 * exceeds the whole budget or its parameters are invalid. */
int lbm_submit(lbm_server *s, const lbm_request *req, uint64_t *ticket);
/* LBM_PENDING until the request has finished, then LBM_OK with *res filled
 * (the request's own error is in res->status).  A ticket is returned once. */
int lbm_poll(lbm_server *s, uint64_t ticket, lbm_result *res);
/* Run the scheduler until every submitted request has finished. */
int lbm_server_drain(lbm_server *s);
/* Current seconds on the server clock. */
double lbm_server_clock(const lbm_server *s);
void lbm_result_free(lbm_result *res);
int lbm_server_destroy(lbm_server *s);

#ifdef __cplusplus
}
#endif
#endif
