// kernels_impl.hpp -- CDNA4 (gfx950) kernels of the phase-field LB step.
//
// Per time step two launches over a tile table (one lattice, or many lattices
// of a serving batch):
//   phi pass : phi(x) = sum_i h_i(x) read in the current AA parity; a pressure
//              ghost takes its owner's phi (Neumann).     (Sec. II.A, after Eq. 4)
//   sweep    : stages phi and node flags of each z-plane (tile + 1-node halo)
//              in an LDS ring, then per fluid node
//                - neighbour phi, wetting substitute at solid links (Eqs. 17-19)
//                - isotropic gradient / Laplacian (Eq. 16)
//                - rho, mu (Eq. 9), tau_mix (Eqs. 10-12 and the Sec. III.A switch)
//                - rho u, u, P (after Eq. 15)
//                - filtered D3Q19 collision with K_i (Eqs. 6-8, 13-15)
//                - D3Q7 collision with theta and delta-theta (Eqs. 1-5)
//                - AA-pattern write-back with half-way bounce-back and the
//                  free-slip band at solid links (Sec. III.A)
//                - pressure-ghost equilibria written by the ghost's owner
//              FP64 wavefront/LDS reductions of mass, momentum, |u|max and
//              phase pressures on diagnostic steps; the last tile of a lattice
//              reduces the tile partials in a fixed order and advances the
//              lattice's step counter.
//
// AA pattern (one population array, updated in place).  At an even step node
// x reads f_i from slot (x, i) and writes f*_i to (x, opp(i)); at an odd step
// it reads f_i from (x - c_i, opp(i)) and writes f*_i to (x + c_i, i).  When
// x - c_i (x + c_i) is solid the odd-step access goes to the node's own slot
// (x, i) ((x, opp(i))) instead, which realises the half-way bounce-back.  The
// odd-step access to the solid node's slot is still issued (its value is
// replaced or never read): every access then uses a scalar per-direction base
// and wall nodes add a masked access to their own slot, rather than choosing a
// base pointer per lane.  Every live slot is read and written by one node
// only, so the sweep needs no second lattice and no synchronisation between
// tiles.  The parity is a template argument; all lattices of a launch share it.
//
// Arithmetic of the FP32 storage modes is FP32 and written in deviation form:
// with f_i = w_i f_ref + d_i the moments use d_i only (sum_i w_i c_i = 0), so
// shifted storage keeps its precision through the collision.
#pragma once

#include <hip/hip_runtime.h>

#include "pflbm.hpp"

namespace pflbm {

// ----------------------------------------------------------------- lattice
// D3Q19 in the order of the public interface; D3Q7 is the first seven.
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
__host__ __device__ constexpr double wg(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
__host__ __device__ constexpr double wh(int i) { return i == 0 ? 0.25 : 0.125; }
constexpr double TGc = 1.0 / 3.0;  // D3Q19 lattice temperature
constexpr double THc = 0.25;       // D3Q7 lattice temperature
constexpr uint32_t SOLID_MASK = 0x7FFFEu;  // link bits 1..18

constexpr int LDS_PLANE = 400;     // >= (TX + 2) * (TY + 2) for TX in {16, 32, 64}

// ------------------------------------------------------ uniform values
// Values read through the descriptor are the same for every lane of a
// workgroup; readfirstlane keeps them in scalar registers, so that population
// addresses are a scalar base plus one 32-bit vector offset.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline int64_t uni(int64_t v) {
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ inline double uni(double v) { return __builtin_bit_cast(double, uni(__builtin_bit_cast(int64_t, v))); }
__device__ inline float uni(float v) { return __builtin_bit_cast(float, uni(__builtin_bit_cast(int, v))); }
template <typename P> __device__ inline P* unip(P* p) { return (P*)uni((int64_t)(uintptr_t)p); }

__device__ inline Tile load_tile(const Tile* tiles) {
    const Tile t = tiles[blockIdx.x];
    Tile u;
    u.lat = uni(t.lat); u.x0 = uni(t.x0); u.y0 = uni(t.y0); u.z0 = uni(t.z0); u.zn = uni(t.zn);
    u.tile_in_lat = uni(t.tile_in_lat); u.pad[0] = u.pad[1] = 0;
    return u;
}

// --------------------------------------------------------------- storage
// Population array [Q][N] of storage type S behind raw buffer resources: the
// directions [0, QS) share resource r0 and [QS, Q) resource r1; direction q is
// reached with the scalar offset (q - group start) * N * sizeof(S) and the
// per-lane 32-bit byte offset of the node.  Each resource spans at most 4 GiB.
constexpr int BUF_FLAGS = 0x00020000;
constexpr int AUX_NT = 2;      // non-temporal: every population is touched once per step
template <int Q> struct Split { static constexpr int QS = Q > 10 ? 10 : Q; };
template <typename S, int Q> struct PopArray {
    __amdgpu_buffer_rsrc_t r0, r1;
    uint32_t stride;           // N * sizeof(S)
    __device__ __amdgpu_buffer_rsrc_t rs(int q) const { return q < Split<Q>::QS ? r0 : r1; }
    __device__ uint32_t so(int q) const { return (uint32_t)(q < Split<Q>::QS ? q : q - Split<Q>::QS) * stride; }
};
template <typename S> struct Store;
template <> struct Store<double> {
    static constexpr bool scaled = false;
    template <int Q> __device__ static double ld(const PopArray<double, Q>& a, int q, uint32_t n) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(a.rs(q), n * 8u, a.so(q), AUX_NT);
        return __builtin_bit_cast(double, v);
    }
    template <int Q> __device__ static void st(const PopArray<double, Q>& a, int q, uint32_t n, double v) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), a.rs(q), n * 8u, a.so(q), AUX_NT);
    }
};
template <> struct Store<float> {
    static constexpr bool scaled = false;
    template <int Q> __device__ static float ld(const PopArray<float, Q>& a, int q, uint32_t n) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(a.rs(q), n * 4u, a.so(q), AUX_NT));
    }
    template <int Q> __device__ static void st(const PopArray<float, Q>& a, int q, uint32_t n, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), a.rs(q), n * 4u, a.so(q), AUX_NT);
    }
};
template <> struct Store<_Float16> {
    static constexpr bool scaled = true;
    template <int Q> __device__ static float ld(const PopArray<_Float16, Q>& a, int q, uint32_t n) {
        const uint16_t b = __builtin_amdgcn_raw_buffer_load_b16(a.rs(q), n * 2u, a.so(q), AUX_NT);
        return (float)__builtin_bit_cast(_Float16, b);
    }
    template <int Q> __device__ static void st(const PopArray<_Float16, Q>& a, int q, uint32_t n, float v) {
        const _Float16 hv = (_Float16)v;   // round to nearest even
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, hv), a.rs(q), n * 2u, a.so(q), AUX_NT);
    }
};
template <typename S, int Q> __device__ inline PopArray<S, Q> pop_array(void* base, int64_t N) {
    PopArray<S, Q> a;
    char* b = unip((char*)base);
    const uint32_t stride = (uint32_t)uni((int64_t)(N * (int64_t)sizeof(S)));
    constexpr int QS = Split<Q>::QS;
    a.stride = stride;
    a.r0 = __builtin_amdgcn_make_buffer_rsrc(b, (short)0, (int)(stride * (uint32_t)QS), BUF_FLAGS);
    a.r1 = __builtin_amdgcn_make_buffer_rsrc(b + (size_t)QS * stride, (short)0,
                                             (int)(stride * (uint32_t)(Q - QS > 0 ? Q - QS : 1)), BUF_FLAGS);
    return a;
}

// ----------------------------------------------------------- parameters
template <typename T> struct Phys {
    T rho_g, rdif, sigma, W, M, F[3];
    T tau_l, tau_g;
    T mc_gamma, mc_phi_M, mc_phi_m, mc_invD, eps;
    T mix_phi, mix_invw;
    T slip_lo, slip_hi;
    T clamp_a;
    T href, gref, sh, sg, inv_sh, inv_sg;
    int mobility_corr, mix, friction;
    __device__ void load(const Desc* D) {
        rho_g = uni((T)D->rho_g);
        rdif = uni((T)(D->rho_l - D->rho_g));
        sigma = uni((T)D->sigma);
        W = uni((T)D->W);
        M = uni((T)D->M);
        F[0] = uni((T)D->F[0]); F[1] = uni((T)D->F[1]); F[2] = uni((T)D->F[2]);
        tau_l = uni((T)(D->nu_l / TGc + 0.5));
        tau_g = uni((T)(D->nu_g / TGc + 0.5));
        mc_gamma = uni((T)D->mc_gamma);
        mc_phi_M = uni((T)D->mc_phi_M);
        mc_phi_m = uni((T)D->mc_phi_m);
        mc_invD = uni((T)(1.0 / D->mc_D));
        eps = uni((T)D->eps);
        mix_phi = uni((T)D->mix_phi);
        mix_invw = uni((T)(1.0 / D->mix_width));
        slip_lo = uni((T)D->slip_lo);
        slip_hi = uni((T)D->slip_hi);
        clamp_a = uni((T)D->clamp_a);
        href = uni((T)D->href);
        gref = uni((T)D->gref);
        sh = uni((T)D->scale_h);
        sg = uni((T)D->scale_g);
        inv_sh = uni((T)(1.0 / D->scale_h));
        inv_sg = uni((T)(1.0 / D->scale_g));
        mobility_corr = uni(D->mobility_corr);
        mix = uni(D->mix);
        friction = uni(D->friction);
    }
};

template <typename T> __device__ inline T clamp01(T v) { return v < T(0) ? T(0) : (v > T(1) ? T(1) : v); }
__device__ inline double dev_tanh(double v) { return tanh(v); }
__device__ inline float dev_tanh(float v) { return tanhf(v); }
__device__ inline double dev_sqrt(double v) { return sqrt(v); }
__device__ inline float dev_sqrt(float v) { return sqrtf(v); }

__device__ inline int wrapc(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Neighbour node indices of (x, y, z) with periodic wrap:
// at(cx, cy, cz) = X[cx+1] + Y[cy+1] + Z[cz+1].
struct Nbr {
    int X[3], Y[3], Z[3];
    __device__ void init(int x, int y, int z, int nx, int ny, int nz) {
        X[0] = x == 0 ? nx - 1 : x - 1; X[1] = x; X[2] = x == nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
        Y[0] = ym * nx; Y[1] = y * nx; Y[2] = yp * nx;
        const int nxy = nx * ny;
        Z[0] = zm * nxy; Z[1] = z * nxy; Z[2] = zp * nxy;
    }
    __device__ uint32_t at(int cx, int cy, int cz) const {
        return (uint32_t)(X[cx + 1] + Y[cy + 1] + Z[cz + 1]);
    }
};

// ------------------------------------------------------- AA population I/O
// Deviations d_i of the populations f_i(x) entering node n's collision at a
// step of parity PAR.  solid: link bits of solid neighbours.
template <typename T, typename S, int Q, int PAR>
__device__ inline void read_pops(const PopArray<S, Q>& a, uint32_t n, const Nbr& nb,
                                 uint32_t solid, T inv_scale, T* d) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (PAR == 0 || i == 0) d[i] = (T)Store<S>::ld(a, i, n);
        else d[i] = (T)Store<S>::ld(a, OPP[i], nb.at(-CX[i], -CY[i], -CZ[i]));
    }
    if (PAR == 1 && solid) {
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if ((solid >> OPP[i]) & 1u) d[i] = (T)Store<S>::ld(a, i, n);   // x - c_i solid
    }
    if (Store<S>::scaled) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] *= inv_scale;
    }
}

// Post-collision deviations of node n at a step of parity PAR.
template <typename T, typename S, int Q, int PAR>
__device__ inline void write_pops(const PopArray<S, Q>& a, uint32_t n, const Nbr& nb,
                                  uint32_t solid, T scale, const T* d) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T v = Store<S>::scaled ? d[i] * scale : d[i];
        if (PAR == 0 || i == 0) Store<S>::st(a, OPP[i], n, v);
        else Store<S>::st(a, i, nb.at(CX[i], CY[i], CZ[i]), v);
    }
    if (PAR == 1 && solid) {
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if ((solid >> i) & 1u)                                           // x + c_i solid
                Store<S>::st(a, OPP[i], n, Store<S>::scaled ? d[i] * scale : d[i]);
    }
}

// f_i(x) into the slots a step of parity PAR reads (initialisation, restore).
template <typename T, typename S, int Q, int PAR>
__device__ inline void place_pops(const PopArray<S, Q>& a, uint32_t n, const Nbr& nb,
                                  uint32_t solid, T scale, const T* d) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const T v = Store<S>::scaled ? d[i] * scale : d[i];
        if (PAR == 0 || i == 0) Store<S>::st(a, i, n, v);
        else Store<S>::st(a, OPP[i], nb.at(-CX[i], -CY[i], -CZ[i]), v);
    }
    if (PAR == 1 && solid) {
#pragma unroll
        for (int i = 1; i < Q; ++i)
            if ((solid >> OPP[i]) & 1u)
                Store<S>::st(a, i, n, Store<S>::scaled ? d[i] * scale : d[i]);
    }
}

// ------------------------------------------------------------------ phi pass
template <typename T, typename SH, int PAR>
__device__ inline T phase_sum(const PopArray<SH, QH>& h, const uint8_t* flg, const uint32_t* lnk,
                              int n, int x, int y, int z, int nx, int ny, int nz,
                              const Phys<T>& ph) {
    const uint8_t f = flg[n];
    const uint32_t solid = (PAR == 1 && (f & F_NEAR_WALL)) ? (lnk[n] & SOLID_MASK) : 0u;
    Nbr nb;
    nb.init(x, y, z, nx, ny, nz);
    T d[QH];
    read_pops<T, SH, QH, PAR>(h, (uint32_t)n, nb, solid, ph.inv_sh, d);
    T s = T(0);
#pragma unroll
    for (int i = 0; i < QH; ++i) s += d[i];
    return ph.href + s;
}

template <typename T, typename SH, int PAR>
__global__ void __launch_bounds__(NTHREADS)
phi_kernel(const Desc* __restrict__ descs, const Tile* __restrict__ tiles, int force) {
    const Tile tl = load_tile(tiles);
    const Desc* D = descs + tl.lat;
    const int64_t step = uni(D->step);
    if (!force && step >= uni(D->stop_step)) return;
    const int nx = uni(D->nx), ny = uni(D->ny), nz = uni(D->nz), TX = uni(D->tx);
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    if (x >= nx || y >= ny) return;
    Phys<T> ph;
    ph.load(D);
    const PopArray<SH, QH> h = pop_array<SH, QH>(D->h, uni(D->N));
    const uint8_t* __restrict__ flg = unip(D->flag);
    const uint32_t* __restrict__ lnk = unip(D->link);
    T* __restrict__ phi = unip((T*)D->phi);
    for (int k = 0; k < tl.zn; ++k) {
        const int z = tl.z0 + k;
        const int n = x + nx * (y + ny * z);
        const uint8_t f = flg[n];
        const int kind = flag_kind(f);
        T v = T(0);
        if (kind == KIND_FLUID) {
            v = phase_sum<T, SH, PAR>(h, flg, lnk, n, x, y, z, nx, ny, nz, ph);
        } else if (kind == KIND_GHOST) {
            // owner = one step inward along the face normal
            const int face = flag_sub(f);
            const int ax = face >> 1, sg = (face & 1) ? -1 : 1;
            int ox = x, oy = y, oz = z;
            if (ax == 0) ox += sg; else if (ax == 1) oy += sg; else oz += sg;
            const int o = ox + nx * (oy + ny * oz);
            v = phase_sum<T, SH, PAR>(h, flg, lnk, o, ox, oy, oz, nx, ny, nz, ph);
        }
        phi[n] = v;
    }
}

// ------------------------------------------------------------------ sweep
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

#ifndef SWEEP_WAVES_PER_EU
#define SWEEP_WAVES_PER_EU 1
#endif
template <typename T, typename SH, typename SG, int MODE, bool DIAG, int TX, int PAR>
__global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(SWEEP_WAVES_PER_EU)))
sweep_kernel(Desc* __restrict__ descs, const Tile* __restrict__ tiles, ReadOut ro, InitIn in) {
    __shared__ T s_phi[4][LDS_PLANE];
    __shared__ uint8_t s_flag[4][LDS_PLANE];
    __shared__ double s_red[NPART][NTHREADS / 64];
    __shared__ int s_last;

    const Tile tl = load_tile(tiles);
    Desc* D = descs + tl.lat;
    const int64_t step = uni(D->step);
    if (MODE == MODE_STEP && step >= uni(D->stop_step)) return;
    const int64_t time = step - uni(D->t0);
    const int nx = uni(D->nx), ny = uni(D->ny), nz = uni(D->nz);
    constexpr int TY = NTHREADS / TX;
    const int tid = threadIdx.x;
    const int tx = tid & (TX - 1), ty = tid / TX;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    const bool active = (x < nx) && (y < ny);
    const int64_t N = uni(D->N);
    const int64_t dev = uni(D->diag_every);
    const bool diag = DIAG && (MODE == MODE_READ || (dev > 0 && (time % dev) == 0));
    Phys<T> ph;
    ph.load(D);
    const T* __restrict__ phig = unip((const T*)D->phi);
    const uint8_t* __restrict__ flg = unip(D->flag);
    const uint32_t* __restrict__ lnk = unip(D->link);
    const PopArray<SH, QH> hb = pop_array<SH, QH>(D->h, uni(D->N));
    const PopArray<SG, QG> gb = pop_array<SG, QG>(D->g, uni(D->N));
    const T Tg = T(TGc);
    // exact reciprocals of the lattice temperatures: 1/Tg = 3, 1/(2 Tg) = 1.5,
    // 1/(2 Tg^2) = 4.5, 1/Th = 4, 1/(2 Th) = 2, 1/(2 Th^2) = 8
    const T iTg = T(3), i2Tg = T(1.5), i2Tg2 = T(4.5), iTh = T(4), i2Th = T(2), i2Th2 = T(8);

    constexpr int LW = TX + 2, LN = (TX + 2) * (TY + 2);
    static_assert(LN <= LDS_PLANE, "LDS plane too small");
    auto stage = [&](int m, int zp) {
        const int zz = wrapc(zp, nz);
        for (int c = tid; c < LN; c += NTHREADS) {
            const int lx = c % LW, ly = c / LW;
            const int gx = wrapc(tl.x0 - 1 + lx, nx), gy = wrapc(tl.y0 - 1 + ly, ny);
            const int n = gx + nx * (gy + ny * zz);
            s_phi[m & 3][c] = phig[n];
            s_flag[m & 3][c] = flg[n];
        }
    };

    double acc[NPART];
#pragma unroll
    for (int j = 0; j < NPART; ++j) acc[j] = 0.0;

    stage(0, tl.z0 - 1);
    stage(1, tl.z0);
    const int c0 = (ty + 1) * LW + (tx + 1);
    for (int k = 0; k < tl.zn; ++k) {
        const int z = tl.z0 + k;
        // a 4-plane ring needs one barrier per plane: a thread that runs ahead
        // stages plane z+2 into the slot of z-2, which no thread still reads
        stage(k + 2, z + 1);
        __syncthreads();
        if (!active) continue;
        const int sm = k & 3, s0 = (k + 1) & 3, sp = (k + 2) & 3;
        const int n = x + nx * (y + ny * z);
        const uint8_t f = s_flag[s0][c0];
        const int kind = flag_kind(f);
        if (kind != KIND_FLUID) {
            if (MODE == MODE_READ) {
                double pv = 0.0, Pv = 0.0;
                if (kind == KIND_GHOST) {
                    const int face = flag_sub(f);
                    pv = (double)s_phi[s0][c0];
                    Pv = D->face_P[face] + D->face_ramp[face] * (double)time;
                }
                if (ro.phi) ro.phi[n] = pv;
                if (ro.P) ro.P[n] = Pv;
                if (ro.u) { ro.u[n] = 0.0; ro.u[N + n] = 0.0; ro.u[2 * N + n] = 0.0; }
                if (ro.pops)
                    for (int i = 0; i < QH + QG; ++i) ro.pops[(int64_t)i * N + n] = 0.0;
            }
            continue;
        }
        const uint32_t links = (f & (F_NEAR_WALL | F_OWNER)) ? lnk[n] : 0u;
        const uint32_t solid = links & SOLID_MASK;
        Nbr nb;
        nb.init(x, y, z, nx, ny, nz);

        // ---- gradient and Laplacian (Eq. 16) over the 18 neighbours, with
        //      the node's own phi standing in at solid links (pre-gradient)
        const T pc = s_phi[s0][c0];
        T grad[3] = {T(0), T(0), T(0)}, lap = T(0);
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            const int sl = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
            T v = s_phi[sl][c0 + CY[i] * LW + CX[i]];
            v = ((solid >> i) & 1u) ? pc : v;
            grad[0] += T(wg(i) * CX[i]) * v;
            grad[1] += T(wg(i) * CY[i]) * v;
            grad[2] += T(wg(i) * CZ[i]) * v;
            lap += T(wg(i)) * (v - pc);
        }
        grad[0] *= iTg; grad[1] *= iTg; grad[2] *= iTg;
        lap = T(6) * lap;
        T nw[3] = {T(0), T(0), T(0)};
        if (solid) {
            // wetting (Eqs. 17-19): wall normal into the fluid from the solid
            // links, t the unit tangential part of the pre-gradient,
            // w = -cos(theta) n + sin(theta) t, phi_s,i from the tanh profile
            // through phi(x) shifted by d_i = w . c_i; the stencil sums then
            // take phi_s,i - phi(x) at each solid link
#pragma unroll
            for (int i = 1; i < 19; ++i) {
                if ((solid >> i) & 1u) {
                    nw[0] -= T(wg(i) * CX[i]);
                    nw[1] -= T(wg(i) * CY[i]);
                    nw[2] -= T(wg(i) * CZ[i]);
                }
            }
            const T nn = dev_sqrt(nw[0] * nw[0] + nw[1] * nw[1] + nw[2] * nw[2]);
            const T inn = nn > T(0) ? T(1) / nn : T(0);
            nw[0] *= inn; nw[1] *= inn; nw[2] *= inn;
            const T ng = nw[0] * grad[0] + nw[1] * grad[1] + nw[2] * grad[2];
            T gt[3] = {grad[0] - nw[0] * ng, grad[1] - nw[1] * ng, grad[2] - nw[2] * ng};
            const T tn = dev_sqrt(gt[0] * gt[0] + gt[1] * gt[1] + gt[2] * gt[2]);
            const T itn = T(1) / (tn + ph.eps);
            gt[0] *= itn; gt[1] *= itn; gt[2] *= itn;
            T a = T(2) * pc - T(1);
            a = a > T(1) - ph.clamp_a ? T(1) - ph.clamp_a : a;
            a = a < -T(1) + ph.clamp_a ? -T(1) + ph.clamp_a : a;
            const T k2W = T(2) / ph.W;
            T dgx = T(0), dgy = T(0), dgz = T(0), dl = T(0);
            for (int i = 1; i < 19; ++i) {
                if (!((solid >> i) & 1u)) continue;
                const int cx = CX[i], cy = CY[i], cz = CZ[i];
                const int sl = cz < 0 ? sm : (cz > 0 ? sp : s0);
                const int mat = flag_sub(s_flag[sl][c0 + cy * LW + cx]);
                const T ct = (T)D->cos_t[mat], st = (T)D->sin_t[mat];
                const T d = -ct * (nw[0] * T(cx) + nw[1] * T(cy) + nw[2] * T(cz)) +
                            st * (gt[0] * T(cx) + gt[1] * T(cy) + gt[2] * T(cz));
                const T t = dev_tanh(k2W * d);
                // tanh(artanh(a) + 2d/W) by the addition theorem
                const T ps = T(0.5) * (T(1) + (a + t) / (T(1) + a * t));
                const T w = T(wg(i)) * (ps - pc);
                dgx += w * T(cx); dgy += w * T(cy); dgz += w * T(cz);
                dl += w;
            }
            grad[0] += dgx * iTg; grad[1] += dgy * iTg; grad[2] += dgz * iTg;
            lap += T(6) * dl;
        }

        // ---- local scalars (Eq. 9, Eqs. 10-12)
        const T pb = clamp01(pc);
        const T rho = ph.rho_g + pb * ph.rdif;
        const T mu = T(48) * ph.sigma / ph.W * pc * (pc - T(1)) * (pc - T(0.5)) -
                     T(1.5) * ph.sigma * ph.W * lap;

        // ---- moments of the populations entering the collision
        T u[3], pdev;                       // pdev = P/T - gref
        T m[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};   // sum c c d: xx yy zz xy xz yz
        if (MODE == MODE_INIT) {
            const double* ui = in.u;
            u[0] = ui ? (T)ui[n] : T(0);
            u[1] = ui ? (T)ui[N + n] : T(0);
            u[2] = ui ? (T)ui[2 * N + n] : T(0);
            const T P0 = in.P ? (T)in.P[n] : (T)D->P_ref;
            pdev = P0 * iTg - ph.gref;
        } else {
            T dg[QG];
            read_pops<T, SG, QG, PAR>(gb, (uint32_t)n, nb, solid, ph.inv_sg, dg);
            // u first (it needs only g and phi), then P (after Eq. 15)
            T s = T(0), j[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int i = 0; i < QG; ++i) {
                s += dg[i];
                j[0] += T(CX[i]) * dg[i];
                j[1] += T(CY[i]) * dg[i];
                j[2] += T(CZ[i]) * dg[i];
                if (CX[i]) m[0] += dg[i];
                if (CY[i]) m[1] += dg[i];
                if (CZ[i]) m[2] += dg[i];
                if (CX[i] * CY[i]) m[3] += T(CX[i] * CY[i]) * dg[i];
                if (CX[i] * CZ[i]) m[4] += T(CX[i] * CZ[i]) * dg[i];
                if (CY[i] * CZ[i]) m[5] += T(CY[i] * CZ[i]) * dg[i];
            }
            const T irho = T(1) / rho;
            u[0] = (j[0] + T(0.5) * (mu * grad[0] + ph.F[0])) * irho;
            u[1] = (j[1] + T(0.5) * (mu * grad[1] + ph.F[1])) * irho;
            u[2] = (j[2] + T(0.5) * (mu * grad[2] + ph.F[2])) * irho;
            pdev = s + T(0.5) * ph.rdif * (u[0] * grad[0] + u[1] * grad[1] + u[2] * grad[2]);
            if (MODE == MODE_READ && ro.pops) {
                for (int i = 0; i < QG; ++i)
                    ro.pops[(int64_t)(QH + i) * N + n] = (double)(T(wg(i)) * ph.gref + dg[i]);
            }
        }
        const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

        if (MODE == MODE_READ) {
            const T P = Tg * (ph.gref + pdev);
            if (ro.phi) ro.phi[n] = (double)pc;
            if (ro.P) ro.P[n] = (double)P;
            if (ro.u) { ro.u[n] = (double)u[0]; ro.u[N + n] = (double)u[1]; ro.u[2 * N + n] = (double)u[2]; }
            if (ro.pops) {
                T dh[QH];
                read_pops<T, SH, QH, PAR>(hb, (uint32_t)n, nb, solid, ph.inv_sh, dh);
                for (int i = 0; i < QH; ++i)
                    ro.pops[(int64_t)i * N + n] = (double)(T(wh(i)) * ph.href + dh[i]);
            }
        }
        if (DIAG && diag) {
            const double um = sqrt((double)uu);
            const double P = (double)(Tg * (ph.gref + pdev));
            const bool bad = isnan((double)pc) || isnan(um) || isnan(P);
            if (bad) {
                acc[P_NAN] += 1.0;
            } else {
                acc[P_PHI] += (double)pc;
                acc[P_MX] += (double)(rho * u[0]);
                acc[P_MY] += (double)(rho * u[1]);
                acc[P_MZ] += (double)(rho * u[2]);
                acc[P_UMAX] = fmax(acc[P_UMAX], um);
                if (pc > T(0.99)) { acc[P_PLIQ] += P; acc[P_NLIQ] += 1.0; }
                if (pc < T(0.01)) { acc[P_PGAS] += P; acc[P_NGAS] += 1.0; }
            }
        }
        if (MODE == MODE_READ) continue;

        // ---- D3Q19 filtered collision (Eqs. 6-8, 13-15) in moment space.
        // With Gamma_i = w_i (1 + gam_i) and the equilibrium deviation
        //   deq_i = rho w_i gam_i + w_i pdev - K_i / 2,
        // the second moment of deq follows in closed form on D3Q19 (its weights
        // are isotropic to fourth order):
        //   sum_i c c deq_i = rho u u + T pdev I - (1/2) sum_i c c K_i,
        //   sum_i c c K_i = rdif [T (u g + g u) - u u (u.g) + T I (u.g)]
        //                 + (mu/T) [T (u g + g u) - u u (u.g)]
        //                 + (1/T) [T (u F + F u) - u u (u.F)],   g = grad phi,
        // so Pi = sum c c (d - deq) needs only the ten moments of the incoming
        // populations, and every outgoing population is computed and stored
        // on its own:  d*_i = deq_i + K_i + (1 - 1/tau) w_i/(2T^2) (c c - T I):Pi.
        const T ug = u[0] * grad[0] + u[1] * grad[1] + u[2] * grad[2];
        const T uF = u[0] * ph.F[0] + u[1] * ph.F[1] + u[2] * ph.F[2];
        T om = T(0), Pi[6] = {T(0), T(0), T(0), T(0), T(0), T(0)}, trPi = T(0);
        if (MODE == MODE_STEP) {
            const T cg = ph.rdif + mu * iTg;              // coefficient of (u g + g u)
            const T cu3 = (ph.rdif + mu * iTg) * ug + uF * iTg;   // coefficient of -u u
            const T ciso = ph.rdif * Tg * ug;            // coefficient of I
            // sum c c K: symmetric tensor, components xx yy zz xy xz yz
            const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const int al = ia[c], be = ib[c];
                const T ccK = cg * Tg * (u[al] * grad[be] + grad[al] * u[be]) +
                              (u[al] * ph.F[be] + ph.F[al] * u[be]) -
                              u[al] * u[be] * cu3 + (c < 3 ? ciso : T(0));
                const T ccdeq = rho * u[al] * u[be] + (c < 3 ? Tg * pdev : T(0)) - T(0.5) * ccK;
                Pi[c] = m[c] - ccdeq;
            }
            trPi = Tg * (Pi[0] + Pi[1] + Pi[2]);
            T Fm;
            if (ph.mix) Fm = T(0.5) * (dev_tanh((pb - ph.mix_phi) * ph.mix_invw) + T(1));
            else Fm = pb;
            const T tau = (T(1) - Fm) * ph.tau_g + Fm * ph.tau_l;
            om = (T(1) - T(1) / tau) * i2Tg2;
        }
        // bounce-back of the moving-wall kind inside the free-slip band
        // (Sec. III.A): the wall moves with the tangential fluid velocity
        T uw[3] = {T(0), T(0), T(0)};
        if (MODE == MODE_STEP && solid && ph.friction && pc >= ph.slip_lo && pc <= ph.slip_hi) {
            const T un = nw[0] * u[0] + nw[1] * u[1] + nw[2] * u[2];
            uw[0] = u[0] - nw[0] * un;
            uw[1] = u[1] - nw[1] * un;
            uw[2] = u[2] - nw[2] * un;
        }
#pragma unroll
        for (int i = 0; i < QG; ++i) {
            const T w = T(wg(i));
            const T cu = T(CX[i]) * u[0] + T(CY[i]) * u[1] + T(CZ[i]) * u[2];
            const T gam = cu * iTg + cu * cu * i2Tg2 - uu * i2Tg;  // Gamma/w - 1
            const T G = w * (T(1) + gam);
            const T cgr = T(CX[i]) * grad[0] + T(CY[i]) * grad[1] + T(CZ[i]) * grad[2] - ug;
            const T cf = T(CX[i]) * ph.F[0] + T(CY[i]) * ph.F[1] + T(CZ[i]) * ph.F[2] - uF;
            const T K = (w * gam * ph.rdif + G * mu * iTg) * cgr + G * cf * iTg;
            const T base = w * (rho * gam + pdev);
            T v;
            if (MODE == MODE_STEP) {
                const T cPc = T(CX[i] * CX[i]) * Pi[0] + T(CY[i] * CY[i]) * Pi[1] +
                              T(CZ[i] * CZ[i]) * Pi[2] + T(2 * CX[i] * CY[i]) * Pi[3] +
                              T(2 * CX[i] * CZ[i]) * Pi[4] + T(2 * CY[i] * CZ[i]) * Pi[5];
                v = base + T(0.5) * K + om * w * (cPc - trPi);
                const T vs = Store<SG>::scaled ? v * ph.sg : v;
                if (PAR == 0 || i == 0) {
                    T vb = vs;
                    if (i > 0 && ((solid >> i) & 1u)) {
                        const T cuw = T(CX[i]) * uw[0] + T(CY[i]) * uw[1] + T(CZ[i]) * uw[2];
                        const T vw = v - T(6) * w * rho * cuw;
                        vb = Store<SG>::scaled ? vw * ph.sg : vw;
                    }
                    Store<SG>::st(gb, OPP[i], (uint32_t)n, vb);
                } else {
                    Store<SG>::st(gb, i, nb.at(CX[i], CY[i], CZ[i]), vs);
                    if ((solid >> i) & 1u) {
                        const T cuw = T(CX[i]) * uw[0] + T(CY[i]) * uw[1] + T(CZ[i]) * uw[2];
                        const T vw = v - T(6) * w * rho * cuw;
                        Store<SG>::st(gb, OPP[i], (uint32_t)n, Store<SG>::scaled ? vw * ph.sg : vw);
                    }
                }
            } else {
                v = base - T(0.5) * K;    // MODE_INIT: the equilibrium g_eq_i - w_i gref
                const T vs = Store<SG>::scaled ? v * ph.sg : v;
                if (PAR == 0 || i == 0) {
                    Store<SG>::st(gb, i, (uint32_t)n, vs);
                } else {
                    Store<SG>::st(gb, OPP[i], nb.at(-CX[i], -CY[i], -CZ[i]), vs);
                    if ((solid >> OPP[i]) & 1u) Store<SG>::st(gb, i, (uint32_t)n, vs);
                }
            }
        }

        // ---- D3Q7 phase field (Eqs. 1-5)
        {
            const T gnorm = dev_sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
            T theta = ph.M * iTh * (T(1) - T(4) * (pc - T(0.5)) * (pc - T(0.5))) / ph.W;
            if (ph.mobility_corr) {
                const T sgn = lap / (fabs(lap) + ph.eps);
                const T y1a = clamp01((pc - ph.mc_phi_M) * ph.mc_invD);
                const T y1b = clamp01((T(1) - pc) * ph.mc_invD);
                const T y2a = clamp01(pc * ph.mc_invD);
                const T y2b = clamp01((ph.mc_phi_m - pc) * ph.mc_invD);
                const T Y1 = y1a < y1b ? y1a : y1b;
                const T Y2 = y2a < y2b ? y2a : y2b;
                theta += ph.mc_gamma * ph.M * iTh / ph.W * gnorm *
                         ((T(1) + sgn) * Y1 + (T(1) - sgn) * Y2);
            }
            const T ign = theta / (gnorm + ph.eps);   // theta n = theta grad / (|grad| + eps)
            const T tn[3] = {grad[0] * ign, grad[1] * ign, grad[2] * ign};
            const T itau_h = T(1) / (ph.M * iTh + T(0.5));
            T B[QH];
            if (MODE == MODE_STEP) read_pops<T, SH, QH, PAR>(hb, (uint32_t)n, nb, solid, ph.inv_sh, B);
#pragma unroll
            for (int i = 0; i < QH; ++i) {
                const T w = T(wh(i));
                const T cu = T(CX[i]) * u[0] + T(CY[i]) * u[1] + T(CZ[i]) * u[2];
                const T gam = cu * iTh + cu * cu * i2Th2 - uu * i2Th;
                const T cn = T(CX[i]) * tn[0] + T(CY[i]) * tn[1] + T(CZ[i]) * tn[2];
                const T heq = w * ((pc - ph.href) + pc * gam + cn);
                if (MODE == MODE_STEP) B[i] = B[i] - (B[i] - heq) * itau_h;
                else B[i] = heq;
            }
            if (MODE == MODE_STEP) write_pops<T, SH, QH, PAR>(hb, (uint32_t)n, nb, solid, ph.sh, B);
            else place_pops<T, SH, QH, PAR>(hb, (uint32_t)n, nb, solid, ph.sh, B);
        }
        if (MODE == MODE_INIT) continue;

        // ---- pressure ghosts owned by this node: equilibria for step t+1 at
        //      the owner's phi and u and the face pressure of step t+1, into
        //      the slots the next (opposite) parity reads
        if (links >> LINK_OWNER_SHIFT) {
            for (int face = 0; face < 6; ++face) {
                if (!((links >> (LINK_OWNER_SHIFT + face)) & 1u)) continue;
                const int ax = face >> 1, sgn = (face & 1) ? -1 : 1;   // inward normal
                const int nfx = ax == 0 ? sgn : 0, nfy = ax == 1 ? sgn : 0, nfz = ax == 2 ? sgn : 0;
                const uint32_t gidx = nb.at(-nfx, -nfy, -nfz);         // the ghost
                const T Pb = (T)(D->face_P[face] + D->face_ramp[face] * (double)(time + 1));
                const T pdb = Pb * iTg - ph.gref;
#pragma unroll
                for (int i = 1; i < QG; ++i) {
                    if (CX[i] * nfx + CY[i] * nfy + CZ[i] * nfz <= 0) continue;
                    // fluid node y = g + c_i = x + (c_i - n_f), inside the LDS ring
                    const int ex = CX[i] - nfx, ey = CY[i] - nfy, ez = CZ[i] - nfz;
                    const int sl = ez < 0 ? sm : (ez > 0 ? sp : s0);
                    if (flag_kind(s_flag[sl][c0 + ey * LW + ex]) != KIND_FLUID) continue;
                    const T cu = T(CX[i]) * u[0] + T(CY[i]) * u[1] + T(CZ[i]) * u[2];
                    const uint32_t dst = PAR ? nb.at(ex, ey, ez) : gidx;
                    const int slot = PAR ? i : OPP[i];
                    {
                        const T gam = cu * iTg + cu * cu * i2Tg2 - uu * i2Tg;
                        const T v = T(wg(i)) * (rho * gam + pdb);
                        Store<SG>::st(gb, slot, dst, Store<SG>::scaled ? v * ph.sg : v);
                    }
                    if (i < QH) {
                        const T gam = cu * iTh + cu * cu * i2Th2 - uu * i2Th;
                        const T v = T(wh(i)) * ((pc - ph.href) + pc * gam);
                        Store<SH>::st(hb, slot, dst, Store<SH>::scaled ? v * ph.sh : v);
                    }
                }
            }
        }
    }

    if (MODE == MODE_INIT) return;

    // ---- per-tile FP64 partials (wavefront shuffle -> LDS), then the last
    //      tile of the lattice reduces them in a fixed order
    if (DIAG && diag) {
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int j = 0; j < NPART; ++j) {
            const double v = (j == P_UMAX) ? wave_max(acc[j]) : wave_sum(acc[j]);
            if (lane == 0) s_red[j][wv] = v;
        }
        __syncthreads();
        if (tid < NPART) {
            double v = s_red[tid][0];
            for (int w = 1; w < NTHREADS / 64; ++w)
                v = (tid == P_UMAX) ? fmax(v, s_red[tid][w]) : v + s_red[tid][w];
            D->partials[(int64_t)tl.tile_in_lat * NPART + tid] = v;
        }
    }
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        const unsigned old = __hip_atomic_fetch_add(D->counter, 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        s_last = (old == (unsigned)uni(D->ntiles) - 1u);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (DIAG && diag) {
        // fixed-order reduction: thread t sums tiles t, t+256, ... then a tree
        const int nt = uni(D->ntiles);
        for (int j = 0; j < NPART; ++j) {
            double v = 0.0;
            for (int t = tid; t < nt; t += NTHREADS) {
                const double p = __hip_atomic_load(&D->partials[(int64_t)t * NPART + j],
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v = (j == P_UMAX) ? fmax(v, p) : v + p;
            }
            v = (j == P_UMAX) ? wave_max(v) : wave_sum(v);
            if ((tid & 63) == 0) s_red[j][tid >> 6] = v;
        }
        __syncthreads();
        if (tid < NPART) {
            double v = s_red[tid][0];
            for (int w = 1; w < NTHREADS / 64; ++w)
                v = (tid == P_UMAX) ? fmax(v, s_red[tid][w]) : v + s_red[tid][w];
            D->diag[tid] = v;
        }
        __syncthreads();
        if (tid == 0) {
            D->diag_step = step;
            const bool nan = D->diag[P_NAN] > 0.0;
            const bool fast = D->u_max > 0.0 && D->diag[P_UMAX] > D->u_max;
            if (nan || fast) D->unstable = 1;
        }
    }
    if (tid == 0) {
        if (MODE == MODE_STEP) D->step = step + 1;
        __hip_atomic_store(D->counter, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// --------------------------------------------------------------- restore
// Populations f_i(x) of a step of parity PAR (canonical [26][N] doubles) into
// the AA slots that step reads.
template <typename T, typename SH, typename SG, int PAR>
__global__ void __launch_bounds__(NTHREADS)
restore_kernel(const Desc* __restrict__ descs, const Tile* __restrict__ tiles,
               const double* __restrict__ pops) {
    const Tile tl = load_tile(tiles);
    const Desc* D = descs + tl.lat;
    const int nx = uni(D->nx), ny = uni(D->ny), nz = uni(D->nz), TX = uni(D->tx);
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    if (x >= nx || y >= ny) return;
    Phys<T> ph;
    ph.load(D);
    const int64_t N = uni(D->N);
    const PopArray<SH, QH> hb = pop_array<SH, QH>(D->h, uni(D->N));
    const PopArray<SG, QG> gb = pop_array<SG, QG>(D->g, uni(D->N));
    const uint8_t* __restrict__ flg = unip(D->flag);
    const uint32_t* __restrict__ lnk = unip(D->link);
    for (int k = 0; k < tl.zn; ++k) {
        const int z = tl.z0 + k;
        const int n = x + nx * (y + ny * z);
        const uint8_t f = flg[n];
        if (flag_kind(f) != KIND_FLUID) continue;
        const uint32_t solid = (f & F_NEAR_WALL) ? (lnk[n] & SOLID_MASK) : 0u;
        Nbr nb;
        nb.init(x, y, z, nx, ny, nz);
        T dh[QH], dg[QG];
        for (int i = 0; i < QH; ++i) dh[i] = (T)(pops[(int64_t)i * N + n] - wh(i) * D->href);
        for (int i = 0; i < QG; ++i) dg[i] = (T)(pops[(int64_t)(QH + i) * N + n] - wg(i) * D->gref);
        place_pops<T, SH, QH, PAR>(hb, (uint32_t)n, nb, solid, ph.sh, dh);
        place_pops<T, SG, QG, PAR>(gb, (uint32_t)n, nb, solid, ph.sg, dg);
    }
}

// -------------------------------------------------------------- launchers
template <typename T, typename SH, typename SG, int TX, int PAR>
hipError_t launch_sweep_tp(int mode, Desc* d, const Tile* tiles, int ntiles, int diag,
                           ReadOut ro, InitIn in, hipStream_t s) {
    dim3 grid(ntiles), block(NTHREADS);
    switch (mode) {
        case MODE_STEP:
            if (diag) sweep_kernel<T, SH, SG, MODE_STEP, true, TX, PAR><<<grid, block, 0, s>>>(d, tiles, ro, in);
            else sweep_kernel<T, SH, SG, MODE_STEP, false, TX, PAR><<<grid, block, 0, s>>>(d, tiles, ro, in);
            break;
        case MODE_READ:
            sweep_kernel<T, SH, SG, MODE_READ, true, TX, PAR><<<grid, block, 0, s>>>(d, tiles, ro, in);
            break;
        case MODE_INIT:
            sweep_kernel<T, SH, SG, MODE_INIT, false, TX, PAR><<<grid, block, 0, s>>>(d, tiles, ro, in);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, typename SH, typename SG>
hipError_t launch_sweep_storage(int mode, int tx, int parity, Desc* d, const Tile* tiles,
                                int ntiles, int diag, ReadOut ro, InitIn in, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    const int key = tx * 2 + (parity & 1);
    switch (key) {
        case 128: return launch_sweep_tp<T, SH, SG, 64, 0>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 129: return launch_sweep_tp<T, SH, SG, 64, 1>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 64: return launch_sweep_tp<T, SH, SG, 32, 0>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 65: return launch_sweep_tp<T, SH, SG, 32, 1>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 32: return launch_sweep_tp<T, SH, SG, 16, 0>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 33: return launch_sweep_tp<T, SH, SG, 16, 1>(mode, d, tiles, ntiles, diag, ro, in, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, typename SH>
hipError_t launch_phi_storage(int parity, const Desc* d, const Tile* tiles, int ntiles,
                              hipStream_t s, int force) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(NTHREADS);
    if (parity & 1) phi_kernel<T, SH, 1><<<grid, block, 0, s>>>(d, tiles, force);
    else phi_kernel<T, SH, 0><<<grid, block, 0, s>>>(d, tiles, force);
    return hipGetLastError();
}

template <typename T, typename SH, typename SG>
hipError_t launch_restore_storage(int parity, const Desc* d, const Tile* tiles, int ntiles,
                                  const double* pops, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(NTHREADS);
    if (parity & 1) restore_kernel<T, SH, SG, 1><<<grid, block, 0, s>>>(d, tiles, pops);
    else restore_kernel<T, SH, SG, 0><<<grid, block, 0, s>>>(d, tiles, pops);
    return hipGetLastError();
}

}  // namespace pflbm
