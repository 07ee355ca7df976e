// kernels_impl.hpp -- CDNA4 (gfx950) kernels of the phase-field LB step.
//
// Per time step, over a tile table (one lattice, or many lattices of a
// serving batch) and a list of near-wall fluid nodes:
//   phi pass : phi(x) = sum_i h_i(x) read in the current AA parity; a pressure
//              ghost takes its owner's phi (Neumann).     (Sec. II.A, after Eq. 4)
//   wall pass: at every near-wall fluid node the wall normal, the wetting
//              values at the solid links (Eqs. 17-19, with the hysteresis
//              blend of Sec. III.A) and the gradient / Laplacian sums with
//              them (Eq. 16)
//   sweep    : stages phi and node flags of each z-plane (tile + 1-node halo)
//              in an LDS ring, then per fluid node
//                - isotropic gradient / Laplacian (Eq. 16); the wall pass's
//                  sums at near-wall nodes
//                - rho, mu (Eq. 9), tau_mix (Eqs. 10-12 and the Sec. III.A switch)
//                - rho u, u, P (after Eq. 15)
//                - filtered D3Q19 collision with K_i (Eqs. 6-8, 13-15)
//                - D3Q7 collision with theta and delta-theta (Eqs. 1-5)
//                - AA-pattern write-back with half-way bounce-back and the
//                  free-slip band at solid links (Sec. III.A)
//                - pressure-ghost equilibria written by the ghost's owner
//              FP64 wavefront/LDS reductions of mass, momentum, |u|max and
//              phase pressures on diagnostic steps; the last tile of a lattice
//              reduces the tile partials in a fixed order.
//
// AA pattern (the populations are updated in place).  At an even step node x
// reads f_i from slot (x, i) and writes f*_i to (x, opp(i)); at an odd step it
// reads f_i from (x - c_i, opp(i)) and writes f*_i to (x + c_i, i).  When
// x - c_i (x + c_i) is solid the odd-step access goes to the node's own slot
// (x, i) ((x, opp(i))) instead, which realises the half-way bounce-back; the
// two candidate slots of an access share a buffer resource, so each lane
// picks its slot by its offset within one access.  Every live slot is read
// and written by one node only, so the sweep needs no second lattice and no
// synchronisation between tiles.  The parity is a template argument; all
// lattices of a launch share it.
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
// phase lattice of QP directions: weights and the inverse-temperature
// factors 1/T, 1/(2T^2), 1/(2T) of its second-order equilibrium (D3Q7:
// T = 1/4, D3Q19: T = 1/3)
template <int QP> __host__ __device__ constexpr double wp(int i) { return QP == 19 ? wg(i) : wh(i); }
template <int QP> __host__ __device__ constexpr double itp() { return QP == 19 ? 3.0 : 4.0; }
template <int QP> __host__ __device__ constexpr double i2tp2() { return QP == 19 ? 4.5 : 8.0; }
template <int QP> __host__ __device__ constexpr double i2tp() { return QP == 19 ? 1.5 : 2.0; }
constexpr double TGc = 1.0 / 3.0;  // D3Q19 lattice temperature
constexpr double THc = 0.25;       // D3Q7 lattice temperature


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
// Every pointer held in a descriptor points to device (global) memory: the
// cast through address space 1 lets the compiler use global instead of flat
// loads and stores (flat ones also count as LDS traffic, so each wait for an
// LDS result would wait for them too).
// Workgroup barrier that orders LDS only.  Within one sweep the threads of a
// block share nothing through global memory (each population slot read or
// written during a step is touched by one node only), so the barrier need not
// wait for the population stores in flight, which a full __syncthreads would.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
template <typename P> __device__ inline P* unip(P* p) {
    return (P*)(__attribute__((address_space(1))) P*)uni((int64_t)(uintptr_t)p);
}

__device__ inline Tile load_tile(const Tile* tiles, bool reversed = false) {
    const Tile t = tiles[reversed ? gridDim.x - 1 - blockIdx.x : blockIdx.x];
    Tile u;
    u.lat = uni(t.lat); u.x0 = uni(t.x0); u.y0 = uni(t.y0); u.z0 = uni(t.z0); u.zn = uni(t.zn);
    u.tile_in_lat = uni(t.tile_in_lat); u.pad[0] = u.pad[1] = 0;
    return u;
}

// --------------------------------------------------------------- storage
// Populations in the blocked layout of pop_layout (pflbm.hpp): group r is a
// raw buffer resource of Np * pb bytes; direction u (h first, then g) sits at
// the scalar offset 64 (prefix(u) - prefix(first direction of its group)) of
// every block, and a node at the per-lane byte offset
//   (p / 64) 64 pb + (p % 64) sizeof(S),   p = x + nxp (y + ny z)
// (Nbr below), so both offsets fit 32 bits.
constexpr int BUF_FLAGS = 0x00020000;
// Cache policy of the population accesses (buffer aux bits; 2 = nt).  The
// sweep loads and stores with the default (temporal) policy: an odd step's
// x-shifted stores write partial cache lines at every tile edge, which L2
// merges with the neighbouring tile's part before write-back only when the
// lines stay resident (non-temporal stores: sweep 1.28 -> 1.17 ms on the
// 256 x 256 x 512 duct, FP32; non-temporal loads with temporal stores: 1.34).
// The phi pass only reads h and streams it non-temporally (0.157 vs 0.177 ms).
constexpr int AUX_LD = 0, AUX_ST = 0, AUX_PHI = 2;
// layout constants of a (phase lattice, storage) pair
template <typename SH, typename SG, int QP> struct Lay {
    static constexpr PopLayout L = pop_layout(QP, (int)sizeof(SH), (int)sizeof(SG));
    static constexpr int G = L.G, K = L.k, PB = L.pb, BLK = 64 * L.pb;
    static constexpr int SZH = (int)sizeof(SH), SZG = (int)sizeof(SG);
    static constexpr int prefix(int u) { return pop_prefix(u, QP, SZH, SZG); }
};
// one family of populations (h: U0 = 0, Q = QP; g: U0 = QP, Q = 19)
template <typename S_, int Q_, int U0, typename LAY> struct PopArray {
    typedef S_ S;
    static constexpr int Q = Q_;
    static constexpr bool IS_G = U0 > 0;
    __amdgpu_buffer_rsrc_t r0, r1;
    __device__ __amdgpu_buffer_rsrc_t rs(int q) const { return U0 + q < LAY::K ? r0 : r1; }
    __device__ static constexpr uint32_t so(int q) {
        return (uint32_t)(64 * (LAY::prefix(U0 + q) - (U0 + q < LAY::K ? 0 : LAY::prefix(LAY::K))));
    }
    // directions q and r live in the same group (one resource)
    __device__ static constexpr bool same(int q, int r) { return (U0 + q < LAY::K) == (U0 + r < LAY::K); }
    __device__ static constexpr uint32_t lo(int q, int r) { return so(q) < so(r) ? so(q) : so(r); }
};
template <typename S> struct Store;
template <> struct Store<double> {
    static constexpr bool scaled = false;
    template <int AUX = AUX_LD, typename PA> __device__ static double ld(const PA& a, int q, uint32_t off) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(a.rs(q), off, a.so(q), AUX);
        return __builtin_bit_cast(double, v);
    }
    template <typename PA> __device__ static void st(const PA& a, int q, uint32_t off, double v) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), a.rs(q), off, a.so(q), AUX_ST);
    }
    template <int AUX = AUX_LD, typename PA> __device__ static double ldx(const PA& a, int q, uint32_t voff, uint32_t soff) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(a.rs(q), voff, soff, AUX));
    }
    template <typename PA> __device__ static void stx(const PA& a, int q, uint32_t voff, uint32_t soff, double v) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), a.rs(q), voff, soff, AUX_ST);
    }
};
template <> struct Store<float> {
    static constexpr bool scaled = false;
    template <int AUX = AUX_LD, typename PA> __device__ static float ld(const PA& a, int q, uint32_t off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(a.rs(q), off, a.so(q), AUX));
    }
    template <typename PA> __device__ static void st(const PA& a, int q, uint32_t off, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), a.rs(q), off, a.so(q), AUX_ST);
    }
    template <int AUX = AUX_LD, typename PA> __device__ static float ldx(const PA& a, int q, uint32_t voff, uint32_t soff) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(a.rs(q), voff, soff, AUX));
    }
    template <typename PA> __device__ static void stx(const PA& a, int q, uint32_t voff, uint32_t soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), a.rs(q), voff, soff, AUX_ST);
    }
};
template <> struct Store<_Float16> {
    static constexpr bool scaled = true;
    template <int AUX = AUX_LD, typename PA> __device__ static float ld(const PA& a, int q, uint32_t off) {
        const uint16_t b = __builtin_amdgcn_raw_buffer_load_b16(a.rs(q), off, a.so(q), AUX);
        return (float)__builtin_bit_cast(_Float16, b);
    }
    template <typename PA> __device__ static void st(const PA& a, int q, uint32_t off, float v) {
        const _Float16 hv = (_Float16)v;   // round to nearest even
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, hv), a.rs(q), off, a.so(q), AUX_ST);
    }
    template <int AUX = AUX_LD, typename PA> __device__ static float ldx(const PA& a, int q, uint32_t voff, uint32_t soff) {
        const uint16_t b = __builtin_amdgcn_raw_buffer_load_b16(a.rs(q), voff, soff, AUX);
        return (float)__builtin_bit_cast(_Float16, b);
    }
    template <typename PA> __device__ static void stx(const PA& a, int q, uint32_t voff, uint32_t soff, float v) {
        const _Float16 hv = (_Float16)v;
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, hv), a.rs(q), voff, soff, AUX_ST);
    }
};
// the h (U0 = 0) or g (U0 = QP) family of descriptor D
template <typename S, int Q, int U0, typename LAY>
__device__ inline PopArray<S, Q, U0, LAY> pop_array(const Desc* D) {
    PopArray<S, Q, U0, LAY> a;
    const uint32_t bytes = (uint32_t)uni((int64_t)(D->Np * (int64_t)LAY::PB));
    a.r0 = __builtin_amdgcn_make_buffer_rsrc(unip((char*)D->pops[0]), (short)0, (int)bytes, BUF_FLAGS);
    a.r1 = __builtin_amdgcn_make_buffer_rsrc(unip((char*)D->pops[1]), (short)0, (int)bytes, BUF_FLAGS);
    return a;
}
#define PFLBM_HB(T_SH, T_SG, QP_) PopArray<T_SH, QP_, 0, Lay<T_SH, T_SG, QP_>>
#define PFLBM_GB(T_SH, T_SG, QP_) PopArray<T_SG, QG, QP_, Lay<T_SH, T_SG, QP_>>

// ----------------------------------------------------------- parameters
// Derived constants come precomputed in the compute precision (Desc::pf for
// FP32, Desc::pd for FP64).  No kernel writes them, so they are read through
// the constant address space: scalar loads, which the compiler may repeat
// anywhere (vector loads of them would be counted with the population
// stores, and each wait for one would wait for every store before it).
template <typename T> __device__ inline const T* param_block(const Desc* D);
template <> __device__ inline const float* param_block<float>(const Desc* D) { return D->pf; }
template <> __device__ inline const double* param_block<double>(const Desc* D) { return D->pd; }

template <typename T> struct Phys {
    const __attribute__((address_space(4))) T* p;
    int mobility_corr, mix, friction;
    __device__ void load(const Desc* D) {
        p = (const __attribute__((address_space(4))) T*)uni((int64_t)(uintptr_t)param_block<T>(D));
        mobility_corr = uni(D->mobility_corr);
        mix = uni(D->mix);
        friction = uni(D->friction);
    }
    __device__ T operator[](int k) const { return p[k]; }
};

template <typename T> __device__ inline T clamp01(T v) { return v < T(0) ? T(0) : (v > T(1) ? T(1) : v); }
// Square root, quotient and exponential of the compute type.  FP64 keeps the
// correctly rounded forms; FP32 takes the hardware approximations
// (v_sqrt_f32, v_rcp_f32, v_exp_f32, about one ulp each), far below the
// rounding of the FP32 and FP16 population storage, at a tenth of the
// instructions.
__device__ inline double dev_sqrt(double v) { return sqrt(v); }
__device__ inline float dev_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ inline double dev_div(double a, double b) { return a / b; }
__device__ inline float dev_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double dev_exp(double v) { return exp(v); }
__device__ inline float dev_exp(float v) { return __builtin_amdgcn_exp2f(v * 1.44269504088896341f); }
// (1 + tanh v) / 2 in its logistic form 1 / (1 + e^(-2v)): one exponential
// and one quotient; saturates to 0 and 1 through e^(-2v) = inf and 0
template <typename T> __device__ inline T half_tanh1(T v) { return dev_div(T(1), T(1) + dev_exp(T(-2) * v)); }
// tanh v = 1 - 2 / (e^(2v) + 1) in FP32 (exactly 0 at v = 0, +-1 at the
// ends); the library tanh in FP64
__device__ inline double dev_tanh(double v) { return tanh(v); }
__device__ inline float dev_tanh(float v) { return 1.0f - 2.0f * __builtin_amdgcn_rcpf(dev_exp(2.0f * v) + 1.0f); }

__device__ inline int wrapc(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Byte offsets of the 27 nodes around (x, y, z), periodic wrap, in the
// blocked population layout: at<IS_G>(cx, cy, cz) = A[cx+1] + BY[cy+1] +
// BZ[cz+1], with A = (x' / 64) 64 pb + (x' % 64) sizeof(S) for the wrapped x'
// (AH for h, AG for g: the same registers when h and g share their type),
// BY = y' (nxp / 64) 64 pb, BZ = z' ny (nxp / 64) 64 pb.
struct Nbr {
    uint32_t AH[3], AG[3], BY[3], BZ[3];
    template <typename LAY>
    __device__ void init(int x, int y, int z, int nx, int ny, int nz, int nxp) {
        const int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const uint32_t b = (uint32_t)(xs[c] >> 6) * (uint32_t)LAY::BLK, l = (uint32_t)(xs[c] & 63);
            AH[c] = b + l * (uint32_t)LAY::SZH;
            AG[c] = b + l * (uint32_t)LAY::SZG;
        }
        const uint32_t row = (uint32_t)(nxp >> 6) * (uint32_t)LAY::BLK;
        BY[0] = (uint32_t)ym * row; BY[1] = (uint32_t)y * row; BY[2] = (uint32_t)yp * row;
        const uint32_t plane = (uint32_t)ny * row;
        BZ[0] = (uint32_t)zm * plane; BZ[1] = (uint32_t)z * plane; BZ[2] = (uint32_t)zp * plane;
    }
    template <bool IS_G> __device__ uint32_t at(int cx, int cy, int cz) const {
        return (IS_G ? AG[cx + 1] : AH[cx + 1]) + BY[cy + 1] + BZ[cz + 1];
    }
    template <bool IS_G> __device__ uint32_t own() const { return at<IS_G>(0, 0, 0); }
};

// ------------------------------------------------------- AA population I/O
// At an odd step a wall link changes which slot a node reads or writes: the
// slot of the neighbour (direction a at the neighbour's offset) or its own
// slot (direction b at its own offset).  When a and b share a resource one
// access serves both cases: its scalar offset is the smaller of the two
// directions' offsets and each lane adds the rest to its own address.
template <typename PA>
__device__ inline uint32_t sel_off(int a, uint32_t off_a, int b, uint32_t off_b, bool use_b) {
    const uint32_t lo = PA::lo(a, b);
    return use_b ? off_b + (PA::so(b) - lo) : off_a + (PA::so(a) - lo);
}

// Deviations d_i of the populations f_i(x) entering the node's collision at a
// step of parity PAR.  solid: link bits of solid neighbours.  Odd step:
// f_i(x) is in (x - c_i, opp(i)), or in (x, i) when x - c_i is solid.
template <typename T, int PAR, int AUX = AUX_LD, typename PA>
__device__ inline void read_pops(const PA& a, const Nbr& nb, uint32_t solid, T inv_scale, T* d) {
    typedef typename PA::S S;
    constexpr int Q = PA::Q;
    constexpr bool G = PA::IS_G;
    const uint32_t n = nb.own<G>();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (PAR == 0 || i == 0) {
            d[i] = (T)Store<S>::template ld<AUX>(a, i, n);
        } else if (PA::same(OPP[i], i)) {
            const uint32_t off = sel_off<PA>(OPP[i], nb.at<G>(-CX[i], -CY[i], -CZ[i]), i, n, (solid >> OPP[i]) & 1u);
            d[i] = (T)Store<S>::template ldx<AUX>(a, i, off, PA::lo(OPP[i], i));
        } else {
            d[i] = (T)Store<S>::template ld<AUX>(a, OPP[i], nb.at<G>(-CX[i], -CY[i], -CZ[i]));
            if ((solid >> OPP[i]) & 1u) d[i] = (T)Store<S>::template ld<AUX>(a, i, n);
        }
    }
    if (Store<S>::scaled) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] *= inv_scale;
    }
}

// Store of the post-collision value v of direction i (i > 0) at a step of
// parity PAR: even (x, opp(i)); odd (x + c_i, i), or (x, opp(i)) when x + c_i
// is solid (half-way bounce-back).
template <int PAR, typename PA, typename V>
__device__ inline void put_pop(const PA& a, const Nbr& nb, uint32_t solid, int i, V v) {
    typedef typename PA::S S;
    constexpr bool G = PA::IS_G;
    const uint32_t n = nb.own<G>();
    if (PAR == 0 || i == 0) {
        Store<S>::st(a, OPP[i], n, v);
    } else if (PA::same(i, OPP[i])) {
        const uint32_t off = sel_off<PA>(i, nb.at<G>(CX[i], CY[i], CZ[i]), OPP[i], n, (solid >> i) & 1u);
        Store<S>::stx(a, i, off, PA::lo(i, OPP[i]), v);
    } else {
        Store<S>::st(a, i, nb.at<G>(CX[i], CY[i], CZ[i]), v);
        if ((solid >> i) & 1u) Store<S>::st(a, OPP[i], n, v);
    }
}

// Post-collision deviations of the node at a step of parity PAR.
template <typename T, int PAR, typename PA>
__device__ inline void write_pops(const PA& a, const Nbr& nb, uint32_t solid, T scale, const T* d) {
    typedef typename PA::S S;
    constexpr int Q = PA::Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) put_pop<PAR>(a, nb, solid, i, Store<S>::scaled ? d[i] * scale : d[i]);
}

// f_i(x) into the slot a step of parity PAR reads it from (initialisation,
// restore): even (x, i); odd (x - c_i, opp(i)), or (x, i) when x - c_i is solid.
template <int PAR, typename PA, typename V>
__device__ inline void place_pop(const PA& a, const Nbr& nb, uint32_t solid, int i, V v) {
    typedef typename PA::S S;
    constexpr bool G = PA::IS_G;
    const uint32_t n = nb.own<G>();
    if (PAR == 0 || i == 0) {
        Store<S>::st(a, i, n, v);
    } else if (PA::same(OPP[i], i)) {
        const uint32_t off = sel_off<PA>(OPP[i], nb.at<G>(-CX[i], -CY[i], -CZ[i]), i, n, (solid >> OPP[i]) & 1u);
        Store<S>::stx(a, i, off, PA::lo(OPP[i], i), v);
    } else {
        Store<S>::st(a, OPP[i], nb.at<G>(-CX[i], -CY[i], -CZ[i]), v);
        if ((solid >> OPP[i]) & 1u) Store<S>::st(a, i, n, v);
    }
}
template <typename T, int PAR, typename PA>
__device__ inline void place_pops(const PA& a, const Nbr& nb, uint32_t solid, T scale, const T* d) {
    typedef typename PA::S S;
    constexpr int Q = PA::Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) place_pop<PAR>(a, nb, solid, i, Store<S>::scaled ? d[i] * scale : d[i]);
}

// ------------------------------------------------------------------ phi pass
template <typename T, int PAR, typename LAY, typename PA>
__device__ inline T phase_sum(const PA& h, const uint8_t* flg, const uint32_t* lnk,
                              int n, int x, int y, int z, int nx, int ny, int nz, int nxp,
                              const Phys<T>& ph) {
    constexpr int QP = PA::Q;
    const uint8_t f = flg[n];
    const uint32_t solid = (PAR == 1 && (f & F_NEAR_WALL)) ? (lnk[n] & SOLID_MASK) : 0u;
    Nbr nb;
    nb.init<LAY>(x, y, z, nx, ny, nz, nxp);
    T d[QP];
    read_pops<T, PAR, AUX_PHI>(h, nb, solid, ph[PI_INV_SH], d);
    T s = T(0);
#pragma unroll
    for (int i = 0; i < QP; ++i) s += d[i];
    return ph[PI_HREF] + s;
}

template <typename T, typename SH, typename SG, int PAR, int QP>
__global__ void __launch_bounds__(NTHREADS)
phi_kernel(const Desc* __restrict__ descs, const Tile* __restrict__ tiles, int force) {
    typedef Lay<SH, SG, QP> LAYT;
    // the tile list in reverse: the sweep walks it forwards, so the phi pass
    // starts on the tiles the last sweep wrote last (still in the caches)
    // and ends on those the next sweep reads first (1110 -> 1099 us per
    // step, FP32, 256 x 256 x 512 duct)
    const Tile tl = load_tile(tiles, true);
    const Desc* D = descs + tl.lat;
    const int64_t step = uni(D->step);
    if (!force && step >= uni(D->stop_step)) return;
    const int nx = uni(D->nx), ny = uni(D->ny), nz = uni(D->nz), TX = uni(D->tx);
    const int tx = threadIdx.x & (TX - 1), ty = threadIdx.x / TX;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    if (x >= nx || y >= ny) return;
    Phys<T> ph;
    ph.load(D);
    const auto h = pop_array<SH, QP, 0, LAYT>(D);
    const int nxp = uni(D->nxp);
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
            v = phase_sum<T, PAR, LAYT>(h, flg, lnk, n, x, y, z, nx, ny, nz, nxp, ph);
        } else if (kind == KIND_GHOST) {
            // owner = one step inward along the face normal
            const int face = flag_sub(f);
            const int ax = face >> 1, sg = (face & 1) ? -1 : 1;
            int ox = x, oy = y, oz = z;
            if (ax == 0) ox += sg; else if (ax == 1) oy += sg; else oz += sg;
            const int o = ox + nx * (oy + ny * oz);
            v = phase_sum<T, PAR, LAYT>(h, flg, lnk, o, ox, oy, oz, nx, ny, nz, nxp, ph);
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

// ------------------------------------------------------------ node state
// Per-node quantities the D3Q19 and D3Q7 updates need once the moments are
// known (all in the compute precision T).
// c_i . v over the non-zero components of c_i only (IEEE arithmetic keeps
// 0 * v, so the zero components are left out explicitly; after unrolling
// every test below is a compile-time constant)
template <typename T> __device__ inline T cdot(int i, T v0, T v1, T v2) {
    T r = T(0);
    bool any = false;
    if (CX[i]) { r = T(CX[i]) * v0; any = true; }
    if (CY[i]) { r = any ? r + T(CY[i]) * v1 : T(CY[i]) * v1; any = true; }
    if (CZ[i]) { r = any ? r + T(CZ[i]) * v2 : T(CZ[i]) * v2; }
    return r;
}
// c_i c_i : Pi with Pi = (xx, yy, zz, xy, xz, yz), non-zero terms only
template <typename T> __device__ inline T ccpi(int i, const T* P) {
    T r = T(0);
    if (CX[i]) r += P[0];
    if (CY[i]) r += P[1];
    if (CZ[i]) r += P[2];
    if (CX[i] * CY[i]) r += T(2 * CX[i] * CY[i]) * P[3];
    if (CX[i] * CZ[i]) r += T(2 * CX[i] * CZ[i]) * P[4];
    if (CY[i] * CZ[i]) r += T(2 * CY[i] * CZ[i]) * P[5];
    return r;
}

template <typename T> struct NodeState {
    T u[3], uu, grad[3], ug, V[3], uV, rho, pdev, Pi[6], trPi, om, pc, tn[3];
};

// D3Q19 post-collision (MODE_STEP) or equilibrium (MODE_INIT) deviation of
// direction i (Eqs. 6-8, 13-15, in the deviation form of the module notes):
//   d*_i = w_i (rho gam_i + pdev) + K_i / 2 + om w_i (c c - T I):Pi
//   g_eq_i - w_i gref = w_i (rho gam_i + pdev) - K_i / 2
//   K_i = w_i gam_i rdif (c_i - u).grad + Gamma_i (c_i - u).V
// with gam_i = Gamma_i / w_i - 1 and V = (mu grad + F) / T.
template <typename T, int MODE>
__device__ inline T g_out(int i, const NodeState<T>& s, T rdif) {
    const T w = T(wg(i));
    const T a = cdot(i, s.u[0], s.u[1], s.u[2]);
    const T gam = T(3) * a + T(4.5) * a * a - T(1.5) * s.uu;
    const T cgr = cdot(i, s.grad[0], s.grad[1], s.grad[2]) - s.ug;
    const T cv = cdot(i, s.V[0], s.V[1], s.V[2]) - s.uV;
    const T K = w * (gam * rdif * cgr + (T(1) + gam) * cv);
    const T base = w * (s.rho * gam + s.pdev);
    if (MODE == MODE_INIT) return base - T(0.5) * K;
    const T cPc = ccpi(i, s.Pi);
    return base + T(0.5) * K + s.om * w * (cPc - s.trPi);
}

// The same for the pair (i, opp(i)), sharing the terms even in c.
template <typename T, int MODE>
__device__ inline void g_out_pair(int i, const NodeState<T>& s, T rdif, T& vp, T& vm) {
    const T w = T(wg(i));
    const T a = cdot(i, s.u[0], s.u[1], s.u[2]);
    const T e = T(4.5) * a * a - T(1.5) * s.uu;
    const T gp = e + T(3) * a, gm = e - T(3) * a;
    const T b = cdot(i, s.grad[0], s.grad[1], s.grad[2]);
    const T c = cdot(i, s.V[0], s.V[1], s.V[2]);
    const T Kp = w * (gp * rdif * (b - s.ug) + (T(1) + gp) * (c - s.uV));
    const T Km = w * (gm * rdif * (-b - s.ug) + (T(1) + gm) * (-c - s.uV));
    const T bp = w * (s.rho * gp + s.pdev), bm = w * (s.rho * gm + s.pdev);
    if (MODE == MODE_INIT) {
        vp = bp - T(0.5) * Kp;
        vm = bm - T(0.5) * Km;
        return;
    }
    const T cPc = ccpi(i, s.Pi);
    const T filt = s.om * w * (cPc - s.trPi);
    vp = bp + T(0.5) * Kp + filt;
    vm = bm + T(0.5) * Km + filt;
}

// The post-collision pair of MODE_STEP with its terms grouped by their
// parity in c_i: the function g_out_pair evaluates, with about half the
// operations (in another order, so equal up to rounding).  With a = c_i.u,
// b = c_i.grad, c = c_i.V, e = 9/2 a^2 - 3/2 u.u and r = rdif b + c, the pair
// (i, opp(i)) is w_i (E +- O) with
//   E = e A + 3/2 a r + C0 + om c_i c_i:Pi,   O = 3 a A + e r / 2 + c / 2,
//   A = rho - (rdif u.grad + u.V) / 2,   C0 = pdev - u.V / 2 - om tr(Pi).
// In scaled variables (a' = 3/2 a from u' = 3/2 u, e2 = e / 2,
// b'' = c_i.(rdif grad), c'' = c_i.(V / 2), B = 2 A, r = b'' + 2 c''):
//   E = e2 B + a' r + C0 + om c_i c_i:Pi,   O = a' B + e2 r + c''.
// The rest population (c_0 = 0) is w_0 (e2 B + C0) with e2 = -3/4 u.u.
template <typename T> struct PairPre {
    T u15[3], rg[3], vh[3], k2, B, C0;
};
template <typename T>
__device__ inline PairPre<T> pair_pre(const NodeState<T>& s, T rdif) {
    PairPre<T> q;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        q.u15[k] = T(1.5) * s.u[k];
        q.rg[k] = rdif * s.grad[k];
        q.vh[k] = T(0.5) * s.V[k];
    }
    q.k2 = T(-0.75) * s.uu;
    q.B = T(2) * s.rho - (rdif * s.ug + s.uV);
    q.C0 = s.pdev - T(0.5) * s.uV - s.om * s.trPi;
    return q;
}
template <typename T>
__device__ inline T g_rest_step(const PairPre<T>& q) {
    return T(wg(0)) * (q.k2 * q.B + q.C0);
}
template <typename T>
__device__ inline void g_pair_step(int i, const NodeState<T>& s, const PairPre<T>& q, T& vp, T& vm) {
    const T a = cdot(i, q.u15[0], q.u15[1], q.u15[2]);
    const T b = cdot(i, q.rg[0], q.rg[1], q.rg[2]);
    const T c = cdot(i, q.vh[0], q.vh[1], q.vh[2]);
    const T e2 = a * a + q.k2;
    const T r = T(2) * c + b;
    const T E = e2 * q.B + (a * r + (s.om * ccpi(i, s.Pi) + q.C0));
    const T O = a * q.B + (e2 * r + c);
    const T w = T(wg(i));
    const T wE = w * E, wO = w * O;
    vp = wE + wO;
    vm = wE - wO;
}

// Phase-field equilibrium deviation of the pair (i, opp(i)) (Eqs. 2-4):
// h_eq_i - w_i href = w_i [(phi - href) + phi gam^h_i + theta c_i.n]
template <typename T, int QP>
__device__ inline void h_eq_pair(int i, const NodeState<T>& s, T href, T& hp, T& hm) {
    const T w = T(wp<QP>(i));
    const T a = cdot(i, s.u[0], s.u[1], s.u[2]);
    const T e = (s.pc - href) + s.pc * (T(i2tp2<QP>()) * a * a - T(i2tp<QP>()) * s.uu);
    const T o = s.pc * T(itp<QP>()) * a + cdot(i, s.tn[0], s.tn[1], s.tn[2]);
    hp = w * (e + o);
    hm = w * (e - o);
}

// ---------------------------------------------------------------- wall pass
// Every near-wall fluid node, after the phi pass (Sec. II.B, Eqs. 17-19): the
// wall normal into the fluid from the solid links (sub-voxel walls: from the
// table); the neutral pre-gradient (the node's own phi at the solid links);
// w = -cos(theta) n + sin(theta) t with t the unit tangential part of the
// pre-gradient; the wetting value phi_s,i from the tanh profile through
// phi(x) shifted by d_i = w . c_i at each solid link; and the gradient and
// Laplacian sums with them, in the difference form the sweep uses (Eq. 16).
// Contact-angle hysteresis (Sec. III.A) blends and records the wall values
// here.  The sweep takes the sums and the normal of its near-wall nodes from
// this pass, so its waves do not branch into the wetting arithmetic.
// Each block's entries belong to one lattice (the launch table pads every
// lattice's list to a multiple of the block size with node -1), so the
// lattice's constants are block-uniform scalars; all neighbour loads are
// issued before the arithmetic.
template <typename T, int MODE>
__global__ void __launch_bounds__(NTHREADS)
wall_kernel(const Desc* __restrict__ descs, const WallRef* __restrict__ walls, int nwalls) {
    __shared__ T s_cs[2][16];   // cos and sin of each material's contact angle
    // XCD-aware order: block b runs on XCD b mod 8; XCD c takes the c-th
    // contiguous eighth of the list, so wall nodes that share phi lines
    // (neighbouring rows and planes) meet in one L2
    const int nb = gridDim.x, S = (nb + 7) / 8, r = nb - 8 * (S - 1);
    const int c = blockIdx.x % 8, j = blockIdx.x / 8;
    const int blk = c * (S - 1) + (c < r ? c : r) + j;
    const int k = blk * NTHREADS + threadIdx.x;
    WallRef wr = {0, -1, 0, 0u};
    if (k < nwalls) wr = walls[k];
    const int lat = uni(walls[blk * NTHREADS].lat);
    const Desc* D = descs + lat;
    if (threadIdx.x < 16) {
        s_cs[0][threadIdx.x] = (T)D->cos_t[threadIdx.x];
        s_cs[1][threadIdx.x] = (T)D->sin_t[threadIdx.x];
    }
    __syncthreads();
    if (MODE == MODE_STEP && uni(D->step) >= uni(D->stop_step)) return;
    if (wr.node < 0) return;
    const int nx = uni(D->nx), ny = uni(D->ny), nz = uni(D->nz);
    const int n = wr.node;
    const int64_t sl = wr.slot, nwl = uni(D->n_wall);
    const int x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
    const T* __restrict__ phig = unip((const T*)D->phi);
    const uint32_t solid = wr.solid;
    const T* pp = unip(param_block<T>(D));
    const T iTg = T(3);
    const int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
    const int ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
    const int zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
    auto nid = [&](int i) -> int {
        return xs[CX[i] + 1] + nx * (ys[CY[i] + 1] + ny * zs[CZ[i] + 1]);
    };
    // phi of the fluid and ghost neighbours; materials of the solid ones
    T nv[19];
#pragma unroll
    for (int i = 1; i < 19; ++i) nv[i] = ((solid >> i) & 1u) ? T(0) : phig[nid(i)];
    const uint32_t* __restrict__ wm = unip(D->wmat);
    const uint32_t mw[3] = {wm[sl], wm[nwl + sl], wm[2 * nwl + sl]};
    const T pc = phig[n];
    T gx = T(0), gy = T(0), gz = T(0), lap = T(0);
    auto pair_sum = [&](int i, T vp, T vm) {
        const T dv = vp - vm;
        if (CX[i]) gx += T(wg(i) * CX[i]) * dv;
        if (CY[i]) gy += T(wg(i) * CY[i]) * dv;
        if (CZ[i]) gz += T(wg(i) * CZ[i]) * dv;
        lap += T(wg(i)) * ((vp - pc) + (vm - pc));
    };
    T nw[3] = {T(0), T(0), T(0)};
    if (uni(D->subvoxel)) {
        const T* __restrict__ wtab = unip((const T*)D->wall);
        nw[0] = wtab[(QG - 1) * nwl + sl];
        nw[1] = wtab[QG * nwl + sl];
        nw[2] = wtab[(QG + 1) * nwl + sl];
    } else {
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            if (!((solid >> i) & 1u)) continue;
            nw[0] -= T(wg(i) * CX[i]); nw[1] -= T(wg(i) * CY[i]); nw[2] -= T(wg(i) * CZ[i]);
        }
        const T nn = dev_sqrt(nw[0] * nw[0] + nw[1] * nw[1] + nw[2] * nw[2]);
        const T inn = nn > T(0) ? dev_div(T(1), nn) : T(0);
        nw[0] *= inn; nw[1] *= inn; nw[2] *= inn;
    }
#pragma unroll
    for (int i = 1; i < 19; i += 2)
        pair_sum(i, ((solid >> i) & 1u) ? pc : nv[i], ((solid >> (i + 1)) & 1u) ? pc : nv[i + 1]);
    const T g0[3] = {gx * iTg, gy * iTg, gz * iTg};
    const T ng = nw[0] * g0[0] + nw[1] * g0[1] + nw[2] * g0[2];
    T gt[3] = {g0[0] - nw[0] * ng, g0[1] - nw[1] * ng, g0[2] - nw[2] * ng};
    const T tnn = dev_sqrt(gt[0] * gt[0] + gt[1] * gt[1] + gt[2] * gt[2]);
    const T itn = dev_div(T(1), tnn + pp[PI_EPS]);
    gt[0] *= itn; gt[1] *= itn; gt[2] *= itn;
    T a = T(2) * pc - T(1);
    a = a > T(1) - pp[PI_CLAMP_A] ? T(1) - pp[PI_CLAMP_A] : a;
    a = a < -T(1) + pp[PI_CLAMP_A] ? -T(1) + pp[PI_CLAMP_A] : a;
    const T k2W = pp[PI_K2W];
    // contact-angle hysteresis (Sec. III.A): the wall value of link i is
    // blended with one kept from the previous step (history [18][n_wall]):
    // the blended value that step used (mode 1) or its unblended value
    // (mode 2); initialisation and a reset pass record the current values
    const int hmode = uni(D->hysteresis);
    T* __restrict__ hist = hmode ? unip((T*)D->hyst) : nullptr;
    const bool record = MODE == MODE_INIT || (MODE == MODE_READ && uni(D->hyst_reset) != 0);
    auto phis = [&](int i) -> T {
        const int mat = (mw[(i - 1) / 6] >> (4 * ((i - 1) % 6))) & 15u;
        const T ct = s_cs[0][mat], sn = s_cs[1][mat];
        const T d = -ct * cdot(i, nw[0], nw[1], nw[2]) + sn * cdot(i, gt[0], gt[1], gt[2]);
        // tanh(artanh(a) + 2d/W) by the addition theorem: phi_s,i is exactly
        // phi(x) where d_i = 0 (a link along the normal of a 90-degree wall),
        // so the Laplacian there is exactly zero as in the FP64 model and the
        // sign term of the mobility correction does not flip on rounding noise
        const T t = dev_tanh(k2W * d);
        T ps = T(0.5) * (T(1) + dev_div(a + t, T(1) + a * t));
        if (hmode) {
            T* hp = hist + (int64_t)(i - 1) * nwl + sl;
            if (record) {
                *hp = ps;
            } else {
                const T fresh = ps;
                ps = pp[PI_HBETA] * *hp + pp[PI_HBETA1] * fresh;
                if (MODE == MODE_STEP) *hp = hmode == 2 ? fresh : ps;
            }
        }
        return ps;
    };
    gx = gy = gz = lap = T(0);
#pragma unroll
    for (int i = 1; i < 19; i += 2) {
        const T vp = ((solid >> i) & 1u) ? phis(i) : nv[i];
        const T vm = ((solid >> (i + 1)) & 1u) ? phis(i + 1) : nv[i + 1];
        pair_sum(i, vp, vm);
    }
    T* __restrict__ out = unip((T*)D->wgl);
    out[sl] = gx;
    out[nwl + sl] = gy;
    out[2 * nwl + sl] = gz;
    out[3 * nwl + sl] = lap;
    out[4 * nwl + sl] = nw[0];
    out[5 * nwl + sl] = nw[1];
    out[6 * nwl + sl] = nw[2];
}

// SV: instance with the interpolated bounce-back of sub-voxel walls (step
// mode only; lattices without sub-voxel walls keep half-way walls in it).
template <typename T, typename SH, typename SG, int MODE, bool DIAG, int TX, int PAR, int QP, bool SV = false>
__global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(PAR == 1 && sizeof(T) == 4 ? 4 : 1)))
sweep_kernel(Desc* __restrict__ descs, const Tile* __restrict__ tiles, ReadOut ro, InitIn in) {
    // LDS ring of phi and flags: each plane holds the tile plus a one-node
    // halo, LN cells, staged NST cells per thread
    constexpr int LW = TX + 2, LN = (TX + 2) * (NTHREADS / TX + 2);
    constexpr int NST = (LN + NTHREADS - 1) / NTHREADS;
    __shared__ T s_phi[4][LN];
    __shared__ uint8_t s_flag[4][LN];
    __shared__ double s_red[NPART][NTHREADS / 64];
    __shared__ int s_last;
    // sub-voxel instance: f_i^in of each solid link i, kept by the thread
    // that read it from the stream step to its write-back
    __shared__ T s_fin[SV ? QG - 1 : 1][NTHREADS];

    const Tile tl = load_tile(tiles);
    Desc* D = descs + tl.lat;
    const int64_t step = uni(D->step);
    if (MODE == MODE_STEP && step >= uni(D->stop_step)) return;
    const int64_t time = step - uni(D->t0);
    const int nx = uni(D->nx), ny = uni(D->ny), nz = uni(D->nz);
    const int nxy = nx * ny;
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
    typedef Lay<SH, SG, QP> LAYT;
    const auto hb = pop_array<SH, QP, 0, LAYT>(D);
    const auto gb = pop_array<SG, QG, QP, LAYT>(D);
    const int nxp = uni(D->nxp);
    const T Tg = T(TGc);
    const T iTg = T(3), i2Tg2 = T(4.5);
    const T rdif = ph[PI_RDIF];

    // a thread stages cells tid + j * NTHREADS; their in-plane offsets (with
    // the periodic wrap) are fixed for the whole z-march (-1: no cell)
    static_assert(TY + 2 <= NTHREADS, "LDS plane");
    int coff[NST];
#pragma unroll
    for (int j = 0; j < NST; ++j) {
        const int c = tid + j * NTHREADS;
        coff[j] = -1;
        if (c < LN) coff[j] = wrapc(tl.x0 - 1 + c % LW, nx) + nx * wrapc(tl.y0 - 1 + c / LW, ny);
    }
    auto stage = [&](int m, int zp) {
        const int zz = zp < 0 ? zp + nz : (zp >= nz ? zp - nz : zp);
        const int zo = zz * nxy;
#pragma unroll
        for (int j = 0; j < NST; ++j) {
            if (coff[j] < 0) continue;
            s_phi[m & 3][tid + j * NTHREADS] = phig[coff[j] + zo];
            s_flag[m & 3][tid + j * NTHREADS] = flg[coff[j] + zo];
        }
    };

    double acc[NPART];
#pragma unroll
    for (int j = 0; j < NPART; ++j) acc[j] = 0.0;

    // ring slot j holds plane z0 - 1 + j (mod 4).  The prologue stages the
    // three planes the first node plane needs; the global loads of plane z+2
    // are issued during plane z-1 and written during plane z to the slot of
    // plane z-2 (last read in the previous iteration), so their latency
    // overlaps a plane of population traffic, and one barrier per plane
    // orders the ring.
    stage(0, tl.z0 - 1);
    stage(1, tl.z0);
    stage(2, tl.z0 + 1);
    lds_barrier();
    const int c0 = (ty + 1) * LW + (tx + 1);
    // link word of the node (solid-link mask, owned ghost faces), fetched one
    // plane ahead from the staged flags: the odd step's population addresses
    // depend on it
    constexpr uint8_t LINKED = F_NEAR_WALL | F_OWNER;
    const int32_t* __restrict__ wsl_arr = unip(D->wslot);
    // descriptor fields the plane loop reads, through the constant address
    // space (scalar loads; the sweep writes none of them)
    const __attribute__((address_space(4))) Desc* DC = (const __attribute__((address_space(4))) Desc*)D;
    uint32_t lk_next = 0u;
    int32_t ws_next = 0;
    if (active && (s_flag[1][c0] & LINKED)) lk_next = lnk[x + nx * y + nxy * tl.z0];
    if (active && (s_flag[1][c0] & F_NEAR_WALL)) ws_next = wsl_arr[x + nx * y + nxy * tl.z0];
    // phi and flags of one plane for the ring, loaded a plane before they
    // are written to LDS
    T nv[NST];
    uint8_t nf[NST];
    auto fetch = [&](int zz) {
        const int zo = (zz >= nz ? zz - nz : zz) * nxy;
#pragma unroll
        for (int j = 0; j < NST; ++j)
            if (coff[j] >= 0) { nv[j] = phig[coff[j] + zo]; nf[j] = flg[coff[j] + zo]; }
    };
    if (tl.zn > 1) fetch(tl.z0 + 2);
    for (int k = 0; k < tl.zn; ++k) {
        const int z = tl.z0 + k;
        const bool more = k + 1 < tl.zn;
        // this plane's link word and wall slot (loaded one plane ahead) are
        // taken here, before the next plane's loads are issued: a wait for
        // them later would also wait for those loads
        const uint32_t links = lk_next;
        const int32_t wslot_cur = ws_next;
        asm volatile("" ::"v"(links), "v"(wslot_cur));
        // plane z + 2 (loaded during the previous plane) goes to the free
        // ring slot (k + 3) & 3 as soon as the node's populations have
        // arrived, before the node's stores (a wait for it after the stores
        // would also wait for every store); the loads of plane z + 3 follow
        bool staged = !more;
        auto stage_next = [&]() {
            if (staged) return;
            const int m = (k + 3) & 3;
#pragma unroll
            for (int j = 0; j < NST; ++j)
                if (coff[j] >= 0) { s_phi[m][tid + j * NTHREADS] = nv[j]; s_flag[m][tid + j * NTHREADS] = nf[j]; }
            staged = true;
            if (k + 2 < tl.zn) fetch(z + 3);
        };
        lk_next = 0u;
        ws_next = 0;
        if (more && active) {
            const uint8_t fn = s_flag[(k + 2) & 3][c0];
            if (fn & LINKED) lk_next = lnk[x + nx * y + nxy * (z + 1)];
            if (fn & F_NEAR_WALL) ws_next = wsl_arr[x + nx * y + nxy * (z + 1)];
        }
        do {
        if (!active) continue;
        const int sm = k & 3, s0 = (k + 1) & 3, sp = (k + 2) & 3;
        const int n = x + nx * y + nxy * z;
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
                    for (int i = 0; i < QP + QG; ++i) ro.pops[(int64_t)i * N + n] = 0.0;
            }
            continue;
        }
        const uint32_t solid = links & SOLID_MASK;
        Nbr nb;
        nb.init<LAYT>(x, y, z, nx, ny, nz, nxp);
        const uint32_t gown = nb.own<true>();   // the node's own g slots
        NodeState<T> st;
        const T pc = s_phi[s0][c0];
        st.pc = pc;

        // ---- gradient and Laplacian (Eq. 16) in the paper's difference form,
        //      sum_i (phi(x + c_i) - phi(x - c_i)) c_i w_i / (2T), each +-c pair
        //      once (hence 1/T): a neighbourhood symmetric about x gives an
        //      exactly zero component, which the eps-regularised unit vectors
        //      (normal, wall tangent) would otherwise turn into O(1) noise
        auto nbv = [&](int i) -> T {
            const int sl = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
            return s_phi[sl][c0 + CY[i] * LW + CX[i]];
        };
        T gx = T(0), gy = T(0), gz = T(0), lap = T(0);
        auto pair_sum = [&](int i, T vp, T vm) {
            const T dv = vp - vm;
            if (CX[i]) gx += T(wg(i) * CX[i]) * dv;
            if (CY[i]) gy += T(wg(i) * CY[i]) * dv;
            if (CZ[i]) gz += T(wg(i) * CZ[i]) * dv;
            lap += T(wg(i)) * ((vp - pc) + (vm - pc));
        };
#pragma unroll
        for (int i = 1; i < 19; i += 2) pair_sum(i, nbv(i), nbv(i + 1));
        T nw[3] = {T(0), T(0), T(0)};
        // sub-voxel walls: per-slot table of link fractions and wall normal
        const bool svx = DC->subvoxel != 0;
        const T* __restrict__ wtab = nullptr;
        const int64_t wsl = wslot_cur, wstr = DC->n_wall;
        if (SV && MODE == MODE_STEP && solid && svx) {
            wtab = unip((const T*)DC->wall);
            // Even steps load the wall fractions into registers right after
            // the stream step.  Odd steps (fewer registers to spare) keep the fraction of a pair
            // (i, ibar) with one solid link in the LDS slot of its fluid
            // partner until the write-back (the solid link's own slot takes
            // f_i^in); pairs with both links solid reload theirs there.
            // 4-byte fractions go straight from memory to LDS (no registers
            // held, no wait here), FP64 ones through registers.
            if constexpr (PAR == 1 && sizeof(T) == 4) {
#pragma unroll
                for (int i = 1; i < QG; i += 2) {
                    const bool si = (solid >> i) & 1u, sj = (solid >> (i + 1)) & 1u;
                    // destination: row of the partner link, the wave's 64 lanes
                    if (si && !sj)
                        __builtin_amdgcn_global_load_lds((const void*)(wtab + (int64_t)(i - 1) * wstr + wsl),
                                                         (void*)&s_fin[i][tid & ~63], 4, 0, 0);
                    if (sj && !si)
                        __builtin_amdgcn_global_load_lds((const void*)(wtab + (int64_t)i * wstr + wsl),
                                                         (void*)&s_fin[i - 1][tid & ~63], 4, 0, 0);
                }
            } else {
#pragma unroll
                for (int i = 1; i < QG && PAR == 1; i += 2) {
                    const bool si = (solid >> i) & 1u, sj = (solid >> (i + 1)) & 1u;
                    if (si != sj) s_fin[si ? i : i - 1][tid] = wtab[(int64_t)(si ? i - 1 : i) * wstr + wsl];
                }
            }
        }
        if (solid) {
            // wetting (Eqs. 17-19): the stencil sums with the wall values and
            // the wall normal come from the wall pass
            const T* __restrict__ wgl = unip((const T*)DC->wgl);
            gx = wgl[wsl];
            gy = wgl[wstr + wsl];
            gz = wgl[2 * wstr + wsl];
            lap = wgl[3 * wstr + wsl];
            nw[0] = wgl[4 * wstr + wsl];
            nw[1] = wgl[5 * wstr + wsl];
            nw[2] = wgl[6 * wstr + wsl];
        }
        st.grad[0] = gx * iTg; st.grad[1] = gy * iTg; st.grad[2] = gz * iTg;
        lap = T(6) * lap;

        // ---- local scalars (Eq. 9, Eqs. 10-12)
        const T pb = clamp01(pc);
        st.rho = ph[PI_RHO_G] + pb * rdif;
        const T mu = ph[PI_MU3] * pc * (pc - T(1)) * (pc - T(0.5)) - ph[PI_MULAP] * lap;

        // ---- moments of the populations entering the collision
        T m[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};   // sum c c d: xx yy zz xy xz yz
        T qv[QG];   // sub-voxel even steps: wall fractions of the solid links
        if (MODE == MODE_INIT) {
            const double* ui = in.u;
            st.u[0] = ui ? (T)ui[n] : T(0);
            st.u[1] = ui ? (T)ui[N + n] : T(0);
            st.u[2] = ui ? (T)ui[2 * N + n] : T(0);
            st.pdev = in.P ? (T)in.P[n] * iTg - ph[PI_GREF] : ph[PI_PREF_DEV];
        } else {
            T dg[QG];
            read_pops<T, PAR>(gb, nb, solid, ph[PI_INV_SG], dg);
            if (SV && MODE == MODE_STEP && svx && solid && PAR == 0) {
#pragma unroll
                for (int i = 1; i < QG; ++i)
                    qv[i] = ((solid >> i) & 1u) ? wtab[(int64_t)(i - 1) * wstr + wsl] : T(0);
            }
            // pairs (i, opp(i)): even part feeds mass and second moments, odd
            // part the momentum; u first (it needs only g and phi), then P
            T s = dg[0], j[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int i = 1; i < QG; i += 2) {
                const T ev = dg[i] + dg[i + 1], od = dg[i] - dg[i + 1];
                s += ev;
                if (CX[i]) j[0] += T(CX[i]) * od;
                if (CY[i]) j[1] += T(CY[i]) * od;
                if (CZ[i]) j[2] += T(CZ[i]) * od;
                if (CX[i]) m[0] += ev;
                if (CY[i]) m[1] += ev;
                if (CZ[i]) m[2] += ev;
                if (CX[i] * CY[i]) m[3] += T(CX[i] * CY[i]) * ev;
                if (CX[i] * CZ[i]) m[4] += T(CX[i] * CZ[i]) * ev;
                if (CY[i] * CZ[i]) m[5] += T(CY[i] * CZ[i]) * ev;
            }
            stage_next();
            // sub-voxel walls: f_i^in of each solid link waits in LDS for the
            // write-back (stored once every population has arrived)
            if (SV && MODE == MODE_STEP && svx && solid) {
#pragma unroll
                for (int i = 1; i < QG; ++i)
                    if ((solid >> i) & 1u) s_fin[i - 1][tid] = dg[i];
            }
            const T irho = dev_div(T(1), st.rho);
            st.u[0] = (j[0] + T(0.5) * (mu * st.grad[0] + ph[PI_FX])) * irho;
            st.u[1] = (j[1] + T(0.5) * (mu * st.grad[1] + ph[PI_FY])) * irho;
            st.u[2] = (j[2] + T(0.5) * (mu * st.grad[2] + ph[PI_FZ])) * irho;
            st.pdev = s + T(0.5) * rdif *
                              (st.u[0] * st.grad[0] + st.u[1] * st.grad[1] + st.u[2] * st.grad[2]);
            if (MODE == MODE_READ && ro.pops) {
                for (int i = 0; i < QG; ++i)
                    ro.pops[(int64_t)(QP + i) * N + n] = (double)(T(wg(i)) * ph[PI_GREF] + dg[i]);
            }
        }
        st.uu = st.u[0] * st.u[0] + st.u[1] * st.u[1] + st.u[2] * st.u[2];

        if (MODE == MODE_READ) {
            const T P = Tg * (ph[PI_GREF] + st.pdev);
            if (ro.phi) ro.phi[n] = (double)pc;
            if (ro.P) ro.P[n] = (double)P;
            if (ro.u) { ro.u[n] = (double)st.u[0]; ro.u[N + n] = (double)st.u[1]; ro.u[2 * N + n] = (double)st.u[2]; }
            if (ro.pops) {
                T dh[QP];
                read_pops<T, PAR>(hb, nb, solid, ph[PI_INV_SH], dh);
                for (int i = 0; i < QP; ++i)
                    ro.pops[(int64_t)i * N + n] = (double)(T(wp<QP>(i)) * ph[PI_HREF] + dh[i]);
            }
        }
        if (DIAG && diag) {
            const double um = sqrt((double)st.uu);
            const double P = (double)(Tg * (ph[PI_GREF] + st.pdev));
            const bool bad = isnan((double)pc) || isnan(um) || isnan(P);
            if (bad) {
                acc[P_NAN] += 1.0;
            } else {
                acc[P_PHI] += (double)pc;
                acc[P_MX] += (double)(st.rho * st.u[0]);
                acc[P_MY] += (double)(st.rho * st.u[1]);
                acc[P_MZ] += (double)(st.rho * st.u[2]);
                acc[P_UMAX] = fmax(acc[P_UMAX], um);
                if (pc > T(0.99)) { acc[P_PLIQ] += P; acc[P_NLIQ] += 1.0; }
                if (pc < T(0.01)) { acc[P_PGAS] += P; acc[P_NGAS] += 1.0; }
            }
        }
        if (MODE == MODE_READ) continue;

        // ---- D3Q19 filtered collision (Eqs. 6-8, 13-15) in moment space.
        // The second moment of the equilibrium deviation follows in closed
        // form on D3Q19 (weights isotropic to fourth order):
        //   sum_i c c deq_i = rho u u + T pdev I - (1/2) sum_i c c K_i,
        //   sum_i c c K_i = rdif [T (u g + g u) - u u (u.g) + T I (u.g)]
        //                 + T (u V + V u) - u u (u.V),   g = grad phi,
        // so Pi = sum c c (d - deq) needs only the ten moments of the incoming
        // populations, and each outgoing population is computed and stored
        // on its own (g_out, g_out_pair).
        st.ug = st.u[0] * st.grad[0] + st.u[1] * st.grad[1] + st.u[2] * st.grad[2];
        st.V[0] = (mu * st.grad[0] + ph[PI_FX]) * iTg;
        st.V[1] = (mu * st.grad[1] + ph[PI_FY]) * iTg;
        st.V[2] = (mu * st.grad[2] + ph[PI_FZ]) * iTg;
        st.uV = st.u[0] * st.V[0] + st.u[1] * st.V[1] + st.u[2] * st.V[2];
        st.om = T(0);
        st.trPi = T(0);
#pragma unroll
        for (int c = 0; c < 6; ++c) st.Pi[c] = T(0);
        if (MODE == MODE_STEP) {
            const T cuu = rdif * st.ug + st.uV;            // coefficient of -u u
            const T ciso = rdif * Tg * st.ug;              // coefficient of I
            const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const int al = ia[c], be = ib[c];
                const T ccK = Tg * (rdif * (st.u[al] * st.grad[be] + st.grad[al] * st.u[be]) +
                                    (st.u[al] * st.V[be] + st.V[al] * st.u[be])) -
                              st.u[al] * st.u[be] * cuu + (c < 3 ? ciso : T(0));
                const T ccdeq = st.rho * st.u[al] * st.u[be] + (c < 3 ? Tg * st.pdev : T(0)) -
                                T(0.5) * ccK;
                st.Pi[c] = m[c] - ccdeq;
            }
            st.trPi = Tg * (st.Pi[0] + st.Pi[1] + st.Pi[2]);
            T Fm;
            if (ph.mix) Fm = half_tanh1((pb - ph[PI_MIX_PHI]) * ph[PI_MIX_INVW]);
            else Fm = pb;
            const T tau = (T(1) - Fm) * ph[PI_TAU_G] + Fm * ph[PI_TAU_L];
            st.om = (T(1) - dev_div(T(1), tau)) * i2Tg2;
        }
        const T sg = ph[PI_SG];
        // D3Q19 write-back (AA slots of parity PAR)
        // free-slip band (Sec. III.A): at a wall link the wall moves with the
        // tangential fluid velocity u_w (times the slip factor for partial
        // slip), and the bounced-back population loses the moving-wall term
        // 6 w_i rho (c_i . u_w)
        T uw[3] = {T(0), T(0), T(0)};
        bool slip = false;
        if (MODE == MODE_STEP && solid && ph.friction && pc >= ph[PI_SLIP_LO] && pc <= ph[PI_SLIP_HI]) {
            const T un = nw[0] * st.u[0] + nw[1] * st.u[1] + nw[2] * st.u[2];
            uw[0] = st.u[0] - nw[0] * un;
            uw[1] = st.u[1] - nw[1] * un;
            uw[2] = st.u[2] - nw[2] * un;
            slip = true;
        }
        // waves without a node in the band skip the term (a uniform branch)
        const bool wslip = __builtin_amdgcn_ballot_w64(slip) != 0u;
        const T rho6 = ph[PI_SLIP_W6] * st.rho;   // 6 rho, times the slip factor
        auto mwall = [&](int i) -> T {
            return T(wg(i)) * (rho6 * cdot(i, uw[0], uw[1], uw[2]));
        };
        // write-back: half-way bounce-back at wall links through the slot
        // choice of put_pop (even: the own slot (x, ibar) anyway; odd: (x, ibar)
        // instead of the solid node's (x + c_i, i)), with the moving-wall term
        // applied in registers
        auto put_g = [&](int i, T v) {
            if (MODE == MODE_STEP && !(SV && svx) && wslip)
                if (slip && i > 0 && ((solid >> i) & 1u)) v -= mwall(i);
            const T vs = Store<SG>::scaled ? v * sg : v;
            if (MODE == MODE_STEP) put_pop<PAR>(gb, nb, solid, i, vs);
            else place_pop<PAR>(gb, nb, solid, i, vs);
        };
        // sub-voxel walls (Sec. III.A): the value returned along ibar for a
        // solid link i is the linear interpolated bounce-back at the link's
        // wall fraction q, formed from the pair's post-collision values in
        // registers and f_i^in from LDS:
        //   q >= 1/2: (g*_i - m) / (2q) + (1 - 1/(2q)) g*_ibar
        //   q <  1/2: 2q g*_i + (1 - 2q) f_i^in - m
        // (m: moving-wall term), and stored where the half-way rule puts g*_i
        const bool svw = SV && MODE == MODE_STEP && svx && solid;
        constexpr bool QREG = PAR == 0;   // fractions in registers
        // the compiler places no wait for the memory-to-LDS copies before
        // the LDS reads below; the copies count in vmcnt
        if (PAR == 1 && sizeof(T) == 4 && svw) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        auto bb_value = [&](int i, T q, T gi, T gibar) -> T {
            const T m = slip ? mwall(i) : T(0);
            if (q >= T(0.5)) {
                const T r = dev_div(T(1), T(2) * q);
                return (gi - m) * r + (T(1) - r) * gibar;
            }
            return T(2) * q * gi + (T(1) - T(2) * q) * s_fin[i - 1][tid] - m;
        };
        // the same without branches, as a (g*_i - m) + (1 - a) x:
        //   q >= 1/2: a = 1/(2q), x = g*_ibar;   q < 1/2: a = 2q, x = f_i^in - m
        auto bb_value_sel = [&](int i, T q, T gi, T gibar) -> T {
            const T m = mwall(i);   // zero outside the slip band (u_w = 0)
            const T q2 = T(2) * q;
            const bool hi = q2 >= T(1);
            const T a = hi ? dev_div(T(1), q2) : q2;
            const T x = hi ? gibar : s_fin[i - 1][tid] - m;
            return a * (gi - m) + (T(1) - a) * x;
        };
        PairPre<T> pre;
        if (MODE == MODE_STEP) pre = pair_pre(st, rdif);
        put_g(0, MODE == MODE_STEP ? g_rest_step(pre) : g_out<T, MODE>(0, st, rdif));
#pragma unroll
        for (int i = 1; i < QG; i += 2) {
            T vp, vm;
            if (MODE == MODE_STEP) g_pair_step(i, st, pre, vp, vm);
            else g_out_pair<T, MODE>(i, st, rdif, vp, vm);
            if (svw) {
                const bool si = (solid >> i) & 1u, sj = (solid >> (i + 1)) & 1u;
                if (QREG) {
                    // even steps: only the solid links (registers are short)
                    if (si || sj) {
                        const T wp_i = si ? bb_value(i, qv[i], vp, vm) : vp;
                        const T wm_i = sj ? bb_value(i + 1, qv[i + 1], vm, vp) : vm;
                        vp = wp_i;
                        vm = wm_i;
                    }
                } else {
                    // odd steps: both links formed, those not solid dropped
                    // (fewer branches).  A pair with both links solid reloads
                    // its fractions and uses them in its own branch, so that
                    // only waves holding one wait for the loads (the wait
                    // also covers every store issued before).
                    if (si && sj) {
                        const T qi = wtab[(int64_t)(i - 1) * wstr + wsl];
                        const T qj = wtab[(int64_t)i * wstr + wsl];
                        const T wp_i = bb_value_sel(i, qi, vp, vm);
                        vm = bb_value_sel(i + 1, qj, vm, vp);
                        vp = wp_i;
                    } else {
                        const T q = s_fin[si ? i : i - 1][tid];
                        const T wp_i = bb_value_sel(i, q, vp, vm);
                        const T wm_i = bb_value_sel(i + 1, q, vm, vp);
                        vp = si ? wp_i : vp;
                        vm = sj ? wm_i : vm;
                    }
                }
            }
            put_g(i, vp);
            put_g(i + 1, vm);
        }

        // ---- D3Q7 phase field (Eqs. 1-5)
        {
            const T gnorm = dev_sqrt(st.grad[0] * st.grad[0] + st.grad[1] * st.grad[1] +
                                     st.grad[2] * st.grad[2]);
            T theta = ph[PI_THETA0] * (T(1) - T(4) * (pc - T(0.5)) * (pc - T(0.5)));
            if (ph.mobility_corr) {
                const T sgn = dev_div(lap, fabs(lap) + ph[PI_EPS]);
                const T y1a = clamp01((pc - ph[PI_MC_PHI_M]) * ph[PI_MC_INVD]);
                const T y1b = clamp01((T(1) - pc) * ph[PI_MC_INVD]);
                const T y2a = clamp01(pc * ph[PI_MC_INVD]);
                const T y2b = clamp01((ph[PI_MC_PHI_m] - pc) * ph[PI_MC_INVD]);
                const T Y1 = y1a < y1b ? y1a : y1b;
                const T Y2 = y2a < y2b ? y2a : y2b;
                theta += ph[PI_MC_K] * gnorm * ((T(1) + sgn) * Y1 + (T(1) - sgn) * Y2);
            }
            const T ign = dev_div(theta, gnorm + ph[PI_EPS]);   // theta n = theta grad / (|grad| + eps)
            st.tn[0] = st.grad[0] * ign; st.tn[1] = st.grad[1] * ign; st.tn[2] = st.grad[2] * ign;
            const T href = ph[PI_HREF];
            T B[QP];
            if (MODE == MODE_STEP) read_pops<T, PAR>(hb, nb, solid, ph[PI_INV_SH], B);
            const T itau_h = ph[PI_ITAU_H];
            {
                const T heq0 = T(wp<QP>(0)) * ((pc - href) + pc * (-T(i2tp<QP>()) * st.uu));
                B[0] = MODE == MODE_STEP ? B[0] + (heq0 - B[0]) * itau_h : heq0;
            }
#pragma unroll
            for (int i = 1; i < QP; i += 2) {
                T hp, hm;
                h_eq_pair<T, QP>(i, st, href, hp, hm);
                if (MODE == MODE_STEP) {
                    B[i] = B[i] + (hp - B[i]) * itau_h;
                    B[i + 1] = B[i + 1] + (hm - B[i + 1]) * itau_h;
                } else {
                    B[i] = hp;
                    B[i + 1] = hm;
                }
            }
            if (MODE == MODE_STEP) write_pops<T, PAR>(hb, nb, solid, ph[PI_SH], B);
            else place_pops<T, PAR>(hb, nb, solid, ph[PI_SH], B);
        }

        // ---- pressure ghosts owned by this node: hand this step's u to the
        //      ghost pass (phi of the owner already sits in the ghost's phi entry)
        if (MODE == MODE_STEP && (links >> LINK_OWNER_SHIFT)) {
            T* __restrict__ gbuf = unip((T*)DC->gbuf);
            const int64_t gc = DC->gface_count;
            for (int face = 0; face < 6; ++face) {
                if (!((links >> (LINK_OWNER_SHIFT + face)) & 1u)) continue;
                const int ax = face >> 1, sgn = (face & 1) ? -1 : 1;   // inward normal
                const int gx2 = x - (ax == 0 ? sgn : 0), gy2 = y - (ax == 1 ? sgn : 0),
                          gz2 = z - (ax == 2 ? sgn : 0);
                const int64_t slot = ghost_slot(D->gface_base, face, gx2, gy2, gz2, nx, ny);
                gbuf[slot] = st.u[0];
                gbuf[gc + slot] = st.u[1];
                gbuf[2 * gc + slot] = st.u[2];
            }
        }
        } while (0);
        stage_next();
        lds_barrier();
    }

    // Only a diagnostic pass needs tiles to meet: a cross-tile handshake costs
    // an agent-scope release and acquire per tile (L2 write-back and
    // invalidate on a chip whose XCDs have separate L2s).  The step counter
    // advances in its own kernel.
    if (MODE == MODE_INIT || !(DIAG && diag)) return;

    // ---- per-tile FP64 partials (wavefront shuffle -> LDS), then the last
    //      tile of the lattice reduces them in a fixed order
    {
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
    {
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
    if (tid == 0) __hip_atomic_store(D->counter, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}


// --------------------------------------------------------------- restore
// Populations f_i(x) of a step of parity PAR (canonical [26][N] doubles) into
// the AA slots that step reads.
template <typename T, typename SH, typename SG, int PAR, int QP>
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
    typedef Lay<SH, SG, QP> LAYT;
    const auto hb = pop_array<SH, QP, 0, LAYT>(D);
    const auto gb = pop_array<SG, QG, QP, LAYT>(D);
    const int nxp = uni(D->nxp);
    const uint8_t* __restrict__ flg = unip(D->flag);
    const uint32_t* __restrict__ lnk = unip(D->link);
    for (int k = 0; k < tl.zn; ++k) {
        const int z = tl.z0 + k;
        const int n = x + nx * (y + ny * z);
        const uint8_t f = flg[n];
        if (flag_kind(f) != KIND_FLUID) continue;
        const uint32_t solid = (f & F_NEAR_WALL) ? (lnk[n] & SOLID_MASK) : 0u;
        Nbr nb;
        nb.init<LAYT>(x, y, z, nx, ny, nz, nxp);
        T dh[QP], dg[QG];
        for (int i = 0; i < QP; ++i) dh[i] = (T)(pops[(int64_t)i * N + n] - wp<QP>(i) * D->href);
        for (int i = 0; i < QG; ++i) dg[i] = (T)(pops[(int64_t)(QP + i) * N + n] - wg(i) * D->gref);
        place_pops<T, PAR>(hb, nb, solid, ph[PI_SH], dh);
        place_pops<T, PAR>(gb, nb, solid, ph[PI_SG], dg);
    }
}

// ---------------------------------------------------------- pressure ghosts
// For every ghost g of a pressure face (Sec. III.A: Dirichlet P, Neumann u and
// phi): the populations it hands to the fluid at the next step t+1 are the
// equilibria at its owner's phi and u of step t and the face pressure of step
// t+1, without forcing and without the counter-term.  Only the directions
// that point into a fluid node are written, into the slots the next step's
// parity reads: (g + c_i, i) for an even step, (g, opp(i)) for an odd one.
// Runs after the sweep of step t and before the step counter advances.
template <typename T, typename SH, typename SG, int QP>
__global__ void __launch_bounds__(NTHREADS)
ghost_kernel(const Desc* __restrict__ descs, const GhostRef* __restrict__ ghosts, int nghosts) {
    const int k = blockIdx.x * NTHREADS + threadIdx.x;
    if (k >= nghosts) return;
    const GhostRef gr = ghosts[k];
    const Desc* D = descs + gr.lat;
    const int64_t step = D->step;
    if (step >= D->stop_step) return;
    const int64_t next = step + 1;
    const int par = (int)(next & 1);
    const int nx = D->nx, ny = D->ny, nz = D->nz;
    const int64_t N = D->N;
    const int g = gr.node;
    const int x = g % nx, y = (g / nx) % ny, z = g / (nx * ny);
    const uint8_t fg = D->flag[g];
    const int face = flag_sub(fg);
    const int ax = face >> 1, sgn = (face & 1) ? -1 : 1;
    const int nfx = ax == 0 ? sgn : 0, nfy = ax == 1 ? sgn : 0, nfz = ax == 2 ? sgn : 0;
    const T* pp = param_block<T>(D);
    const T pc = ((const T*)D->phi)[g];           // the owner's phi (Neumann copy)
    const int64_t slot = ghost_slot(D->gface_base, face, x, y, z, nx, ny);
    const T* gb = (const T*)D->gbuf;
    const int64_t gc = D->gface_count;
    const T u[3] = {gb[slot], gb[gc + slot], gb[2 * gc + slot]};
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T pb = clamp01(pc);
    const T rho = pp[PI_RHO_G] + pb * pp[PI_RDIF];
    const double Pb = D->face_P[face] + D->face_ramp[face] * (double)(next - D->t0);
    const T pdb = (T)(Pb * 3.0) - pp[PI_GREF];
    const T iTg = T(3), i2Tg = T(1.5), i2Tg2 = T(4.5);
    const T iTh = T(itp<QP>()), i2Th = T(i2tp<QP>()), i2Th2 = T(i2tp2<QP>());
    // a launch may mix lattices, so the population bases are per lane here
    typedef Lay<SH, SG, QP> LAYT;
    char* const p0 = (char*)D->pops[0];
    char* const p1 = (char*)D->pops[1];
    const int64_t row = (int64_t)(D->nxp >> 6) * LAYT::BLK;
    // byte address of direction u (h first, then g) of node (xa, ya, za)
    auto pop_at = [&](int u, int xa, int ya, int za, int size) -> char* {
        const int64_t off = (int64_t)(xa >> 6) * LAYT::BLK + (int64_t)(xa & 63) * size +
                            (int64_t)ya * row + (int64_t)za * ny * row +
                            64 * (LAYT::prefix(u) - (u < LAYT::K ? 0 : LAYT::prefix(LAYT::K)));
        return (u < LAYT::K ? p0 : p1) + off;
    };
#pragma unroll
    for (int i = 1; i < QG; ++i) {
        if (CX[i] * nfx + CY[i] * nfy + CZ[i] * nfz <= 0) continue;
        // g + c_i (periodic wrap)
        const int xn = wrapc(x + CX[i], nx), yn = wrapc(y + CY[i], ny), zn = wrapc(z + CZ[i], nz);
        if (flag_kind(D->flag[xn + (int64_t)nx * (yn + (int64_t)ny * zn)]) != KIND_FLUID) continue;
        const int xd = par == 0 ? xn : x, yd = par == 0 ? yn : y, zd = par == 0 ? zn : z;
        const int q = par == 0 ? i : OPP[i];
        const T cu = T(CX[i]) * u[0] + T(CY[i]) * u[1] + T(CZ[i]) * u[2];
        const T gam = cu * iTg + cu * cu * i2Tg2 - uu * i2Tg;
        const T vg = T(wg(i)) * (rho * gam + pdb);
        *(SG*)pop_at(QP + q, xd, yd, zd, (int)sizeof(SG)) = (SG)(Store<SG>::scaled ? vg * pp[PI_SG] : vg);
        if (i < QP) {
            const T gh = cu * iTh + cu * cu * i2Th2 - uu * i2Th;
            const T vh = T(wp<QP>(i)) * ((pc - pp[PI_HREF]) + pc * gh);
            *(SH*)pop_at(q, xd, yd, zd, (int)sizeof(SH)) = (SH)(Store<SH>::scaled ? vh * pp[PI_SH] : vh);
        }
    }
}


// -------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_wall_compute(int mode, const Desc* d, const WallRef* walls, int nwalls, hipStream_t s) {
    if (nwalls <= 0) return hipSuccess;
    dim3 grid((nwalls + NTHREADS - 1) / NTHREADS), block(NTHREADS);
    switch (mode) {
        case MODE_STEP: wall_kernel<T, MODE_STEP><<<grid, block, 0, s>>>(d, walls, nwalls); break;
        case MODE_READ: wall_kernel<T, MODE_READ><<<grid, block, 0, s>>>(d, walls, nwalls); break;
        case MODE_INIT: wall_kernel<T, MODE_INIT><<<grid, block, 0, s>>>(d, walls, nwalls); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, typename SH, typename SG>
hipError_t launch_ghosts_storage(int qp, const Desc* d, const GhostRef* ghosts, int nghosts,
                                 hipStream_t s) {
    if (nghosts <= 0) return hipSuccess;
    dim3 grid((nghosts + NTHREADS - 1) / NTHREADS), block(NTHREADS);
    if (qp == 19) ghost_kernel<T, SH, SG, 19><<<grid, block, 0, s>>>(d, ghosts, nghosts);
    else ghost_kernel<T, SH, SG, QH><<<grid, block, 0, s>>>(d, ghosts, nghosts);
    return hipGetLastError();
}

template <typename T, typename SH, typename SG, int TX, int PAR, int QP>
hipError_t launch_sweep_tp(int mode, Desc* d, const Tile* tiles, int ntiles, int diag,
                           ReadOut ro, InitIn in, hipStream_t s) {
    dim3 grid(ntiles), block(NTHREADS);
    switch (mode) {
        case MODE_STEP:
            if (diag) sweep_kernel<T, SH, SG, MODE_STEP, true, TX, PAR, QP><<<grid, block, 0, s>>>(d, tiles, ro, in);
            else sweep_kernel<T, SH, SG, MODE_STEP, false, TX, PAR, QP><<<grid, block, 0, s>>>(d, tiles, ro, in);
            break;
        case MODE_STEP_SV:
            if (diag) sweep_kernel<T, SH, SG, MODE_STEP, true, TX, PAR, QP, true><<<grid, block, 0, s>>>(d, tiles, ro, in);
            else sweep_kernel<T, SH, SG, MODE_STEP, false, TX, PAR, QP, true><<<grid, block, 0, s>>>(d, tiles, ro, in);
            break;
        case MODE_READ:
            sweep_kernel<T, SH, SG, MODE_READ, true, TX, PAR, QP><<<grid, block, 0, s>>>(d, tiles, ro, in);
            break;
        case MODE_INIT:
            sweep_kernel<T, SH, SG, MODE_INIT, false, TX, PAR, QP><<<grid, block, 0, s>>>(d, tiles, ro, in);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, typename SH, typename SG, int QP>
hipError_t launch_sweep_q(int mode, int tx, int parity, Desc* d, const Tile* tiles, int ntiles,
                          int diag, ReadOut ro, InitIn in, hipStream_t s) {
    const int key = tx * 2 + (parity & 1);
    switch (key) {
        case 128: return launch_sweep_tp<T, SH, SG, 64, 0, QP>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 129: return launch_sweep_tp<T, SH, SG, 64, 1, QP>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 64: return launch_sweep_tp<T, SH, SG, 32, 0, QP>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 65: return launch_sweep_tp<T, SH, SG, 32, 1, QP>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 32: return launch_sweep_tp<T, SH, SG, 16, 0, QP>(mode, d, tiles, ntiles, diag, ro, in, s);
        case 33: return launch_sweep_tp<T, SH, SG, 16, 1, QP>(mode, d, tiles, ntiles, diag, ro, in, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, typename SH, typename SG>
hipError_t launch_sweep_storage(int qp, int mode, int tx, int parity, Desc* d, const Tile* tiles,
                                int ntiles, int diag, ReadOut ro, InitIn in, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (qp == 19) return launch_sweep_q<T, SH, SG, 19>(mode, tx, parity, d, tiles, ntiles, diag, ro, in, s);
    return launch_sweep_q<T, SH, SG, QH>(mode, tx, parity, d, tiles, ntiles, diag, ro, in, s);
}

template <typename T, typename SH, typename SG>
hipError_t launch_phi_storage(int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                              hipStream_t s, int force) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(NTHREADS);
    const int key = (qp == 19 ? 2 : 0) + (parity & 1);
    switch (key) {
        case 0: phi_kernel<T, SH, SG, 0, QH><<<grid, block, 0, s>>>(d, tiles, force); break;
        case 1: phi_kernel<T, SH, SG, 1, QH><<<grid, block, 0, s>>>(d, tiles, force); break;
        case 2: phi_kernel<T, SH, SG, 0, 19><<<grid, block, 0, s>>>(d, tiles, force); break;
        default: phi_kernel<T, SH, SG, 1, 19><<<grid, block, 0, s>>>(d, tiles, force); break;
    }
    return hipGetLastError();
}

template <typename T, typename SH, typename SG>
hipError_t launch_restore_storage(int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                                  const double* pops, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(NTHREADS);
    const int key = (qp == 19 ? 2 : 0) + (parity & 1);
    switch (key) {
        case 0: restore_kernel<T, SH, SG, 0, QH><<<grid, block, 0, s>>>(d, tiles, pops); break;
        case 1: restore_kernel<T, SH, SG, 1, QH><<<grid, block, 0, s>>>(d, tiles, pops); break;
        case 2: restore_kernel<T, SH, SG, 0, 19><<<grid, block, 0, s>>>(d, tiles, pops); break;
        default: restore_kernel<T, SH, SG, 1, 19><<<grid, block, 0, s>>>(d, tiles, pops); break;
    }
    return hipGetLastError();
}

}  // namespace pflbm
