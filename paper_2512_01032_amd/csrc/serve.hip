// serve.hip -- continuous-batching server (placeholder until the batched
// scheduler lands): every entry point reports LBM_E_STATE.
#include "../../include/lbm.h"
#include "lattice_host.hpp"

using namespace pflbm;

extern "C" int lbm_server_create(const lbm_server_cfg*, lbm_server** out) {
    if (out) *out = nullptr;
    set_error("serving is not available in this build");
    return LBM_E_STATE;
}
extern "C" int lbm_submit(lbm_server*, const lbm_request*, uint64_t*) {
    set_error("serving is not available in this build");
    return LBM_E_STATE;
}
extern "C" int lbm_poll(lbm_server*, uint64_t, lbm_result*) {
    set_error("serving is not available in this build");
    return LBM_E_STATE;
}
extern "C" int lbm_server_drain(lbm_server*) { return LBM_E_STATE; }
extern "C" double lbm_server_clock(const lbm_server*) { return 0.0; }
extern "C" void lbm_result_free(lbm_result*) {}
extern "C" int lbm_server_destroy(lbm_server*) { return LBM_OK; }
