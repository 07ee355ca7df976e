// k_fp16a.hip -- kernel instantiations for one storage mode
// (compute float, h stored as _Float16, g stored as _Float16).
#include "kernels_impl.hpp"

namespace pflbm {

hipError_t launch_sweep_fp16a(int qp, int mode, int tx, int parity, Desc* d, const Tile* tiles,
                          int ntiles, int diag, ReadOut ro, InitIn in, hipStream_t s) {
    return launch_sweep_storage<float, _Float16, _Float16>(qp, mode, tx, parity, d, tiles, ntiles, diag, ro, in, s);
}

hipError_t launch_phi_fp16a(int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                        hipStream_t s, int force) {
    return launch_phi_storage<float, _Float16, _Float16>(qp, parity, d, tiles, ntiles, s, force);
}

hipError_t launch_restore_fp16a(int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                            const double* pops, hipStream_t s) {
    return launch_restore_storage<float, _Float16, _Float16>(qp, parity, d, tiles, ntiles, pops, s);
}

hipError_t launch_ghosts_fp16a(int qp, const Desc* d, const GhostRef* ghosts, int nghosts,
                           hipStream_t s) {
    return launch_ghosts_storage<float, _Float16, _Float16>(qp, d, ghosts, nghosts, s);
}

}  // namespace pflbm
