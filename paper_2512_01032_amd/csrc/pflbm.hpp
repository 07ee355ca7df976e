// pflbm.hpp -- device-side data layout of the MI355X phase-field LB library.
//
// One lattice lives in HBM as
//   pops        phase-field populations h (D3Q7) and hydrodynamic populations
//               g (D3Q19) in blocks of 64 nodes (pop_layout below)
//   phi [N]     order parameter of the current step (written by the phi pass)
//   flag[N]     node kind / material / face / near-wall / ghost-owner bits
//   link[N]     per-node solid-link mask and owned pressure faces
// and is swept in tiles of TX x TY = 256 columns marching over a z-chunk.
// Several lattices (serving) share one tile table; every tile names its
// lattice, and each lattice's descriptor carries its own parameters, step
// counter and parity.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pflbm {

constexpr int QH = 7;        // D3Q7 phase lattice (the default)
constexpr int QHMAX = 19;    // D3Q19 phase lattice (q_phase = 19)
constexpr int QG = 19;
constexpr int NTHREADS = 256;       // threads per tile / workgroup
constexpr int NPART = 10;           // FP64 diagnostic partials per tile

// flag byte
constexpr uint8_t KIND_FLUID = 0, KIND_SOLID = 1, KIND_GHOST = 2;
constexpr uint8_t F_KIND_MASK = 0x3;
constexpr uint8_t F_NEAR_WALL = 0x40;  // fluid node with at least one solid link
constexpr uint8_t F_OWNER = 0x80;      // fluid node that feeds a pressure ghost
__host__ __device__ inline int flag_kind(uint8_t f) { return f & F_KIND_MASK; }
__host__ __device__ inline int flag_sub(uint8_t f) { return (f >> 2) & 15; }  // material or face
__host__ __device__ inline uint8_t make_flag(int kind, int sub) {
    return (uint8_t)(kind | (sub << 2));
}
// link word: bit i (1..18) = neighbour x + c_i is solid; bit 24+f = this node
// is the owner (inward neighbour) of a ghost on pressure face f
constexpr int LINK_OWNER_SHIFT = 24;

// storage modes (same values as enum lbm_storage)
constexpr int ST_FP64 = 0, ST_FP32 = 1, ST_FP32_SHIFT = 2, ST_FP16_G = 3, ST_FP16_ALL = 4;

constexpr uint32_t SOLID_MASK = 0x7FFFEu;  // link bits 1..18
constexpr int WALL_ROWS = 21;              // sub-voxel wall table: 18 fractions + normal
constexpr int WG_ROWS = 7;                 // wall pass output: gradient and Laplacian
                                           // sums (4), unit wall normal (3)

// ---- population layout: blocked structure of arrays.  Rows are padded to
// nxp = 64 ceil(nx / 64) nodes; node p = x + nxp (y + ny z) of the padded
// lattice lies in block p / 64 at lane p % 64.  The directions h_0 .. h_{QP-1},
// g_0 .. g_18 form G groups of consecutive directions (G = 1 while a node's
// populations take at most 104 bytes, else 2, cut near half the bytes).  A
// group is an array of blocks; a block holds the group's directions one after
// another, 64 lanes each, so the 64 nodes of a wave find all populations of
// a group in one contiguous span.  Both groups use the larger group's block
// size, so a node's byte offset within a group is the same in each.  Every
// group is addressed with 32-bit offsets (at most 4 GiB).
struct PopLayout {
    int G;    // groups (1 or 2)
    int k;    // first direction of group 1 (QP + 19 when G = 1)
    int pb;   // bytes per node in every group (the block holds 64 pb bytes)
};
// bytes per node of the directions before direction u (h first, then g)
__host__ __device__ constexpr int pop_prefix(int u, int qp, int sh, int sg) {
    return u <= qp ? u * sh : qp * sh + (u - qp) * sg;
}
__host__ __device__ constexpr PopLayout pop_layout(int qp, int sh, int sg) {
    const int tot = qp * sh + 19 * sg;
    if (tot <= 104) return PopLayout{1, qp + 19, tot};
    int k = 1;
    while (2 * pop_prefix(k, qp, sh, sg) < tot) ++k;
    const int a = pop_prefix(k, qp, sh, sg);
    return PopLayout{2, k, a > tot - a ? a : tot - a};
}
__host__ __device__ constexpr int pad_row(int nx) { return (nx + 63) / 64 * 64; }

struct alignas(16) Tile {
    int32_t lat;      // lattice index in the descriptor array
    int32_t x0, y0;   // first column of the tile
    int32_t z0, zn;   // z-chunk [z0, z0 + zn)
    int32_t tile_in_lat;  // index of this tile within its lattice (partials slot)
    int32_t pad[2];
};

// per-lattice descriptor, resident in device memory
struct alignas(256) Desc {
    // layout
    int32_t nx, ny, nz, tx;        // tx: tile width (16, 32 or 64); ty = 256 / tx
    int64_t N;
    int32_t storage;
    int32_t ntiles;                // tiles of this lattice
    int32_t q_phase;               // phase lattice: 7 or 19
    int32_t nxp;                   // padded row length of the population layout
    void* pops[2];                 // population groups (pops[1] = pops[0] when G = 1)
    int64_t Np;                    // nodes of the padded lattice, nxp ny nz
    void* phi;
    const uint8_t* flag;
    const uint32_t* link;
    double* partials;              // [ntiles][NPART]
    unsigned int* counter;         // tiles finished in the current sweep
    void* gbuf;                    // [3][face entries] u of each ghost's owner (compute type)
    int64_t gface_base[6];         // first entry of each face plane in gbuf
    int64_t gface_count;           // entries per velocity component
    void* hyst;                    // [18][n_wall] wall values of the last step (compute type)
    const int32_t* wslot;          // [N] slot of a near-wall fluid node (-1: none)
    int64_t n_wall;                // near-wall fluid nodes
    void* wgl;                     // [WG_ROWS][n_wall] (compute type): the wall pass's
                                   // stencil sums with the wetting values and wall normal
    const uint32_t* wmat;          // [3][n_wall]: material of the solid neighbour of link i
                                   // in bits 4 ((i - 1) % 6) of word (i - 1) / 6
    int32_t hysteresis;            // 1, 2: wall values blended with their history (two readings)
    int32_t hyst_reset;            // a read pass records the current wall values instead
    void* wall;                    // sub-voxel walls: [WALL_ROWS][n_wall] (compute type):
                                   // rows 0-17 the wall fraction q of links 1-18, rows
                                   // 18-20 the unit wall normal into the fluid
    int32_t subvoxel;              // 1: interpolated bounce-back of g at the wall fractions
    int32_t pad_sv;
    // time
    int64_t step;                  // advanced on the device after each step's ghost pass
    int64_t t0;                    // step counter value at physical time 0
    int64_t stop_step;             // the sweep leaves the lattice alone from here on
    int64_t diag_every;            // 0: never
    // physics
    double rho_l, rho_g, nu_l, nu_g, sigma, W, M;
    double F[3];
    int32_t mobility_corr, mix, friction, pad0;
    double mc_gamma, mc_phi_M, mc_phi_m, mc_D, eps;
    double mix_phi, mix_width;
    double slip_lo, slip_hi;
    double P_ref;
    int32_t face_bc[6];
    double face_P[6], face_ramp[6];
    double cos_t[16], sin_t[16];
    double clamp_a;
    double href, gref;             // shift references (0 for plain storage)
    double scale_h, scale_g;       // storage scales (1 except FP16)
    double u_max;
    // derived constants in the compute precision (host-computed, read as
    // scalars by the kernels): index names in enum ParamIndex
    float pf[32];
    double pd[32];
    // outputs of the last diagnostic reduction
    double diag[NPART];
    int64_t diag_step;
    int32_t unstable;              // sticky: NaN or |u| > u_max seen
    int32_t pad1;
};

enum ParamIndex {
    PI_RHO_G = 0, PI_RDIF, PI_MU3, PI_MULAP, PI_TAU_G, PI_TAU_L, PI_THETA0, PI_MC_K, PI_MC_INVD,
    PI_MC_PHI_M, PI_MC_PHI_m, PI_EPS, PI_MIX_PHI, PI_MIX_INVW, PI_SLIP_LO, PI_SLIP_HI, PI_CLAMP_A,
    PI_HREF, PI_GREF, PI_SH, PI_SG, PI_INV_SH, PI_INV_SG, PI_ITAU_H, PI_FX, PI_FY, PI_FZ,
    PI_K2W, PI_PREF_DEV, PI_HBETA, PI_HBETA1, PI_SLIP_W6, PI_COUNT
};
static_assert(PI_COUNT <= 32, "parameter block");

// diagnostic partial slots
enum { P_PHI = 0, P_MX, P_MY, P_MZ, P_UMAX, P_NAN, P_PLIQ, P_NLIQ, P_PGAS, P_NGAS };

// kernel modes of the sweep
constexpr int MODE_STEP = 0;   // stream + collide, AA in place
constexpr int MODE_READ = 1;   // macroscopic fields / populations to output buffers
constexpr int MODE_INIT = 2;   // equilibria from (phi, u, P) into even-parity slots
constexpr int MODE_STEP_SV = 3;  // launcher mode: MODE_STEP with sub-voxel walls enabled

struct GhostRef {              // one pressure ghost: lattice and node
    int32_t lat;
    int32_t node;
};

struct WallRef {               // one near-wall fluid node
    int32_t lat;               // lattice
    int32_t node;              // node index (-1: padding, skipped)
    int32_t slot;              // slot in the per-lattice wall arrays
    uint32_t solid;            // solid-link mask (bits 1..18)
};

// entry of a ghost node (x, y, z) on face f in the face buffer
__host__ __device__ inline int64_t ghost_slot(const int64_t* base, int f, int x, int y, int z,
                                              int nx, int ny) {
    const int ax = f >> 1;
    if (ax == 0) return base[f] + y + (int64_t)ny * z;
    if (ax == 1) return base[f] + x + (int64_t)nx * z;
    return base[f] + x + (int64_t)nx * y;
}

struct ReadOut {               // device buffers of MODE_READ (NULL: skip)
    double* phi;
    double* P;
    double* u;                 // [3][N]
    double* pops;              // [26][N]: h then g
};

struct InitIn {                // device inputs of MODE_INIT
    const double* u;           // [3][N] or NULL
    const double* P;           // [N] or NULL
};

// host-side launchers (kernels.hip).  qp: phase-lattice size (7 or 19) of
// every lattice in the table; parity: AA parity of the step every lattice
// in the table is at; tx: tile width of every tile (16, 32 or 64).
// force: run the phi pass even for lattices past their stop step (read-back).
hipError_t launch_phi(int storage, int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                      hipStream_t s, int force = 0);
hipError_t launch_sweep(int storage, int qp, int mode, int tx, int parity, Desc* d, const Tile* tiles,
                        int ntiles, int diag, ReadOut ro, InitIn in, hipStream_t s);
hipError_t launch_restore(int storage, int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                          const double* pops, hipStream_t s);
// step counter of every lattice in the table: t -> t+1 unless stopped
hipError_t launch_advance(Desc* d, int nlat, hipStream_t s);
// the same for the listed slots of a descriptor table only
hipError_t launch_advance_list(Desc* d, const int* slots, int n, hipStream_t s);
// p[0..n) = 0 (device memory)
hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s);
// after a sweep, before the step advances: equilibrium populations of every
// listed pressure ghost for the next step, from its owner's phi and u
hipError_t launch_ghosts(int storage, int qp, const Desc* d, const GhostRef* ghosts, int nghosts,
                         hipStream_t s);
// after the phi pass, before the sweep (mode MODE_STEP, MODE_READ or
// MODE_INIT of the sweep that follows): wetting values, stencil sums and wall
// normal of every listed near-wall fluid node
hipError_t launch_wall(int storage, int mode, const Desc* d, const WallRef* walls, int nwalls,
                       hipStream_t s);

}  // namespace pflbm
