// Stand-ins for the kernel launchers of the HIP library, for the host-only
// sanitizer build of its host code (tests/test_sanitizers.py): that build
// compiles no device code, and its driver stops at the first device call.
// Every launcher reports that no device is present.
#include "../../paper_2512_01032_amd/csrc/pflbm.hpp"

namespace pflbm {

hipError_t launch_phi(int, int, int, const Desc*, const Tile*, int, hipStream_t, int) { return hipErrorNoDevice; }
hipError_t launch_sweep(int, int, int, int, int, Desc*, const Tile*, int, int, ReadOut, InitIn, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_restore(int, int, int, const Desc*, const Tile*, int, const double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_advance(Desc*, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_advance_list(Desc*, const int*, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_fill_zero(double*, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_ghosts(int, int, const Desc*, const GhostRef*, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_wall(int, int, const Desc*, const WallRef*, int, hipStream_t) { return hipErrorNoDevice; }

}  // namespace pflbm
