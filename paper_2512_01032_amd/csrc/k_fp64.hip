// k_fp64.hip -- kernel instantiations for one storage mode
// (compute double, h stored as double, g stored as double).
#include "kernels_impl.hpp"

namespace pflbm {

hipError_t launch_sweep_fp64(int qp, int mode, int tx, int parity, Desc* d, const Tile* tiles,
                          int ntiles, int diag, ReadOut ro, InitIn in, hipStream_t s) {
    return launch_sweep_storage<double, double, double>(qp, mode, tx, parity, d, tiles, ntiles, diag, ro, in, s);
}

hipError_t launch_phi_fp64(int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                        hipStream_t s, int force) {
    return launch_phi_storage<double, double, double>(qp, parity, d, tiles, ntiles, s, force);
}

hipError_t launch_restore_fp64(int qp, int parity, const Desc* d, const Tile* tiles, int ntiles,
                            const double* pops, hipStream_t s) {
    return launch_restore_storage<double, double, double>(qp, parity, d, tiles, ntiles, pops, s);
}

hipError_t launch_ghosts_fp64(int qp, const Desc* d, const GhostRef* ghosts, int nghosts,
                           hipStream_t s) {
    return launch_ghosts_storage<double, double, double>(qp, d, ghosts, nghosts, s);
}

hipError_t launch_wall_fp64(int mode, const Desc* d, const WallRef* walls, int nwalls, hipStream_t s) {
    return launch_wall_compute<double>(mode, d, walls, nwalls, s);
}

}  // namespace pflbm
