// handle.hpp -- the single-lattice handle behind the opaque lbm_handle of
// include/lbm.h, shared by the sources that implement its entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/lbm.h"
#include "lattice_host.hpp"
#include "pflbm.hpp"

struct lbm_handle {
    lbm_params p;
    lbm_geometry geo;
    int device = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;        // device arena
    bool own_arena = false;
    pflbm::LatticeLayout L;
    pflbm::Desc hdesc;           // host copy of the descriptor at creation
    pflbm::Desc* ddesc = nullptr;
    pflbm::Tile* dtiles = nullptr;
    int ntiles = 0;
    pflbm::GhostRef* dghosts = nullptr;
    int nghosts = 0;
    pflbm::WallRef* dwalls = nullptr;  // near-wall fluid nodes (wall pass)
    int nwalls = 0;
    int64_t step = 0;            // steps queued so far
    // stability flag copied back asynchronously after each lbm_step
    int* h_unstable = nullptr;   // pinned
    hipEvent_t unstable_ev = nullptr;
    bool unstable_pending = false;
    bool unstable = false;
    // per-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double phi_ms = 0.0, sweep_ms = 0.0;
    int64_t steps_timed = 0;
    // replayed step sequences (captured on a private stream at the first
    // untimed lbm_step): one step by [parity][diagnostic], and GRAPH_CHUNK
    // steps without a diagnostic step by starting parity
    hipStream_t cap_stream = nullptr;
    bool graphs_ready = false;
    hipGraphExec_t one[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipGraphExec_t chunk[2] = {nullptr, nullptr};
};

// steps per replay of a chunk graph (even, so a chunk ends at the parity it
// started from)
constexpr int64_t GRAPH_CHUNK = 16;
