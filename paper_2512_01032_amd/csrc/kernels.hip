// kernels.hip -- storage-mode dispatch of the kernel launchers.  The kernels
// themselves live in kernels_impl.hpp; one translation unit per storage mode
// (k_fp64, k_fp32, k_fp16g) instantiates them.  Storage with both h and g in
// FP16 is rejected when a lattice is created and has no kernels.
#include "pflbm.hpp"

namespace pflbm {

// Step counter of every lattice in a descriptor table: t -> t+1 unless the
// lattice has reached its stop step.  Launched once per time step, after the
// ghost pass (the phi, sweep and ghost kernels all read the counter).
__global__ void __launch_bounds__(NTHREADS) advance_kernel(Desc* __restrict__ descs, int nlat) {
    const int k = blockIdx.x * NTHREADS + threadIdx.x;
    if (k >= nlat) return;
    Desc* D = descs + k;
    const int64_t step = D->step;
    if (step < D->stop_step) D->step = step + 1;
}

// The same over a list of descriptor slots (a batch whose other slots are
// being filled or read back meanwhile on another stream: only the listed
// descriptors are touched).
__global__ void __launch_bounds__(NTHREADS) advance_list_kernel(Desc* __restrict__ descs,
                                                                const int* __restrict__ slots, int n) {
    const int k = blockIdx.x * NTHREADS + threadIdx.x;
    if (k >= n) return;
    Desc* D = descs + slots[k];
    const int64_t step = D->step;
    if (step < D->stop_step) D->step = step + 1;
}

hipError_t launch_advance_list(Desc* d, const int* slots, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    advance_list_kernel<<<dim3((n + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), 0, s>>>(d, slots, n);
    return hipGetLastError();
}

// Zero n doubles: read-back staging, whose nodes in dropped all-solid tiles
// no read kernel writes.  A kernel rather than a memset node, so the call is
// safe inside a captured stream as well.
__global__ void __launch_bounds__(NTHREADS) fill_zero_kernel(double* __restrict__ p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * NTHREADS;
    for (int64_t k = (int64_t)blockIdx.x * NTHREADS + threadIdx.x; k < n; k += stride) p[k] = 0.0;
}

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t want = (n + NTHREADS - 1) / NTHREADS;
    const int blocks = (int)(want < 4096 ? want : 4096);
    fill_zero_kernel<<<dim3(blocks), dim3(NTHREADS), 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_advance(Desc* d, int nlat, hipStream_t s) {
    if (nlat <= 0) return hipSuccess;
    advance_kernel<<<dim3((nlat + NTHREADS - 1) / NTHREADS), dim3(NTHREADS), 0, s>>>(d, nlat);
    return hipGetLastError();
}

hipError_t launch_sweep_fp64(int, int, int, int, Desc*, const Tile*, int, int, ReadOut, InitIn, hipStream_t);
hipError_t launch_phi_fp64(int, int, const Desc*, const Tile*, int, hipStream_t, int);
hipError_t launch_restore_fp64(int, int, const Desc*, const Tile*, int, const double*, hipStream_t);
hipError_t launch_ghosts_fp64(int, const Desc*, const GhostRef*, int, hipStream_t);
hipError_t launch_sweep_fp32(int, int, int, int, Desc*, const Tile*, int, int, ReadOut, InitIn, hipStream_t);
hipError_t launch_phi_fp32(int, int, const Desc*, const Tile*, int, hipStream_t, int);
hipError_t launch_restore_fp32(int, int, const Desc*, const Tile*, int, const double*, hipStream_t);
hipError_t launch_ghosts_fp32(int, const Desc*, const GhostRef*, int, hipStream_t);
hipError_t launch_sweep_fp16g(int, int, int, int, Desc*, const Tile*, int, int, ReadOut, InitIn, hipStream_t);
hipError_t launch_phi_fp16g(int, int, const Desc*, const Tile*, int, hipStream_t, int);
hipError_t launch_restore_fp16g(int, int, const Desc*, const Tile*, int, const double*, hipStream_t);
hipError_t launch_ghosts_fp16g(int, const Desc*, const GhostRef*, int, hipStream_t);
hipError_t launch_wall_fp64(int, const Desc*, const WallRef*, int, hipStream_t);
hipError_t launch_wall_fp32(int, const Desc*, const WallRef*, int, hipStream_t);

// the wall pass depends only on the compute type
hipError_t launch_wall(int storage, int mode, const Desc* d, const WallRef* walls, int nwalls,
                       hipStream_t s) {
    if (storage == ST_FP64) return launch_wall_fp64(mode, d, walls, nwalls, s);
    return launch_wall_fp32(mode, d, walls, nwalls, s);
}

hipError_t launch_sweep(int storage, int qp, int mode, int tx, int parity, Desc* d, const Tile* tiles,
                        int ntiles, int diag, ReadOut ro, InitIn in, hipStream_t s) {
    switch (storage) {
        case ST_FP64: return launch_sweep_fp64(qp, mode, tx, parity, d, tiles, ntiles, diag, ro, in, s);
        case ST_FP32:
        case ST_FP32_SHIFT: return launch_sweep_fp32(qp, mode, tx, parity, d, tiles, ntiles, diag, ro, in, s);
        case ST_FP16_G: return launch_sweep_fp16g(qp, mode, tx, parity, d, tiles, ntiles, diag, ro, in, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_phi(int storage, int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                      hipStream_t s, int force) {
    switch (storage) {
        case ST_FP64: return launch_phi_fp64(qp, parity, d, tiles, ntiles, s, force);
        case ST_FP32:
        case ST_FP32_SHIFT: return launch_phi_fp32(qp, parity, d, tiles, ntiles, s, force);
        case ST_FP16_G: return launch_phi_fp16g(qp, parity, d, tiles, ntiles, s, force);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_restore(int storage, int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                          const double* pops, hipStream_t s) {
    switch (storage) {
        case ST_FP64: return launch_restore_fp64(qp, parity, d, tiles, ntiles, pops, s);
        case ST_FP32:
        case ST_FP32_SHIFT: return launch_restore_fp32(qp, parity, d, tiles, ntiles, pops, s);
        case ST_FP16_G: return launch_restore_fp16g(qp, parity, d, tiles, ntiles, pops, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ghosts(int storage, int qp, const Desc* d, const GhostRef* ghosts, int nghosts,
                         hipStream_t s) {
    switch (storage) {
        case ST_FP64: return launch_ghosts_fp64(qp, d, ghosts, nghosts, s);
        case ST_FP32:
        case ST_FP32_SHIFT: return launch_ghosts_fp32(qp, d, ghosts, nghosts, s);
        case ST_FP16_G: return launch_ghosts_fp16g(qp, d, ghosts, nghosts, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace pflbm
