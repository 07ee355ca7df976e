// k_fp32.hip -- kernel instantiations for one storage mode
// (compute float, h stored as float, g stored as float).
#include "kernels_impl.hpp"

namespace pflbm {

hipError_t launch_sweep_fp32(int qp, int mode, int tx, int parity, Desc* d, const Tile* tiles,
                          int ntiles, int diag, ReadOut ro, InitIn in, hipStream_t s) {
    return launch_sweep_storage<float, float, float>(qp, mode, tx, parity, d, tiles, ntiles, diag, ro, in, s);
}

hipError_t launch_phi_fp32(int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                        hipStream_t s, int force) {
    return launch_phi_storage<float, float, float>(qp, parity, d, tiles, ntiles, s, force);
}

hipError_t launch_restore_fp32(int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                            const double* pops, hipStream_t s) {
    return launch_restore_storage<float, float, float>(qp, parity, d, tiles, ntiles, pops, s);
}

hipError_t launch_ghosts_fp32(int qp, const Desc* d, const GhostRef* ghosts, int nghosts,
                           hipStream_t s) {
    return launch_ghosts_storage<float, float, float>(qp, d, ghosts, nghosts, s);
}

hipError_t launch_wall_fp32(int mode, const Desc* d, const WallRef* walls, int nwalls, hipStream_t s) {
    return launch_wall_compute<float>(mode, d, walls, nwalls, s);
}

}  // namespace pflbm
