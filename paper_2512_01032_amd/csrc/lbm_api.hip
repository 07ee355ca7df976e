// lbm_api.hip -- single-lattice C ABI (include/lbm.h).
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lattice_host.hpp"
#include "pflbm.hpp"

using namespace pflbm;

struct lbm_handle {
    lbm_params p;
    lbm_geometry geo;
    int device = 0;
    hipStream_t stream = nullptr;
    char* base = nullptr;        // device arena
    bool own_arena = false;
    LatticeLayout L;
    Desc hdesc;                  // host copy of the descriptor at creation
    Desc* ddesc = nullptr;
    Tile* dtiles = nullptr;
    int ntiles = 0;
    GhostRef* dghosts = nullptr;
    int nghosts = 0;
    WallRef* dwalls = nullptr;   // near-wall fluid nodes (wall pass)
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
};

#define HIPRET(expr)                                                              \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            set_error("%s: %s", #expr, hipGetErrorString(e_));                    \
            return LBM_E_DEVICE;                                                  \
        }                                                                         \
    } while (0)

extern "C" size_t lbm_footprint(const lbm_params* p) { return footprint_bytes(p); }

static void free_handle(lbm_handle* h) {
    if (!h) return;
    if (h->base && h->own_arena) hipFree(h->base);
    if (h->h_unstable) hipHostFree(h->h_unstable);
    if (h->unstable_ev) hipEventDestroy(h->unstable_ev);
    for (hipEvent_t e : h->ev_pool) hipEventDestroy(e);
    delete h;
}

extern "C" int lbm_create(const lbm_params* p, const lbm_geometry* geo, const lbm_init* init,
                          const lbm_device_ctx* ctx, lbm_handle** out) {
    if (!out) { set_error("out is NULL"); return LBM_E_INVAL; }
    *out = nullptr;
    if (!init) { set_error("init is NULL"); return LBM_E_INVAL; }
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) { set_error("host allocation failed"); return LBM_E_NOMEM; }
    h->p = *p;
    if (geo) h->geo = *geo;
    else {
        memset(&h->geo, 0, sizeof(h->geo));
        for (int k = 0; k < 16; ++k) h->geo.theta_deg[k] = 90.0;
    }
    int rc = build_layout(p, &h->geo, 0, &h->L);
    if (rc != LBM_OK) { free_handle(h); return rc; }
    h->device = ctx ? ctx->device : 0;
    h->stream = ctx ? (hipStream_t)ctx->stream : nullptr;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) { set_error("hipSetDevice(%d): %s", h->device, hipGetErrorString(e)); free_handle(h); return LBM_E_DEVICE; }
    if (ctx && ctx->arena) {
        if (ctx->arena_bytes < h->L.total) {
            set_error("arena of %zu bytes is smaller than the footprint %zu", ctx->arena_bytes, h->L.total);
            free_handle(h);
            return LBM_E_INVAL;
        }
        if (((uintptr_t)ctx->arena) & 255u) {
            set_error("arena must be 256-byte aligned");
            free_handle(h);
            return LBM_E_INVAL;
        }
        h->base = (char*)ctx->arena;
    } else {
        e = hipMalloc((void**)&h->base, h->L.total);
        if (e != hipSuccess) {
            set_error("hipMalloc(%zu): %s", h->L.total, hipGetErrorString(e));
            free_handle(h);
            return LBM_E_NOMEM;
        }
        h->own_arena = true;
    }
    e = hipHostMalloc((void**)&h->h_unstable, sizeof(int), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->unstable_ev, hipEventDisableTiming);
    if (e != hipSuccess) { set_error("pinned flag: %s", hipGetErrorString(e)); free_handle(h); return LBM_E_DEVICE; }
    *h->h_unstable = 0;
    rc = upload_and_init(&h->p, &h->geo, init, h->L, h->base, &h->hdesc, h->stream);
    if (rc != LBM_OK) { free_handle(h); return rc; }
    h->ddesc = (Desc*)(h->base + h->L.off_desc);
    h->dtiles = (Tile*)(h->base + h->L.off_tiles);
    h->ntiles = (int)h->L.tiles.size();
    h->dghosts = (GhostRef*)(h->base + h->L.off_ghosts);
    h->nghosts = (int)h->L.ghosts.size();
    h->dwalls = (WallRef*)(h->base + h->L.off_wrefs);
    h->nwalls = (int)h->L.n_wall;
    h->step = h->hdesc.step;
    // the host copies of flags and links are no longer needed
    std::vector<uint8_t>().swap(h->L.flag);
    std::vector<uint32_t>().swap(h->L.link);
    *out = h;
    return LBM_OK;
}

static hipEvent_t next_event(lbm_handle* h) {
    if (h->ev_used == h->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->ev_pool.push_back(e);
    }
    return h->ev_pool[h->ev_used++];
}

static int poll_unstable(lbm_handle* h, bool wait) {
    if (h->unstable_pending) {
        hipError_t q = wait ? hipEventSynchronize(h->unstable_ev) : hipEventQuery(h->unstable_ev);
        if (q == hipSuccess) {
            h->unstable_pending = false;
            if (*h->h_unstable) h->unstable = true;
        } else if (q != hipErrorNotReady) {
            set_error("stability flag: %s", hipGetErrorString(q));
            return LBM_E_DEVICE;
        }
    }
    if (h->unstable) {
        set_error("diagnostic step saw NaN or |u| above u_max");
        return LBM_E_UNSTABLE;
    }
    return LBM_OK;
}

extern "C" int lbm_step(lbm_handle* h, int64_t nsteps) {
    if (!h) { set_error("handle is NULL"); return LBM_E_INVAL; }
    if (nsteps < 0) { set_error("nsteps < 0"); return LBM_E_INVAL; }
    int rc = poll_unstable(h, false);
    if (rc != LBM_OK) return rc;
    HIPRET(hipSetDevice(h->device));
    const int storage = h->p.storage;
    const int qp = phase_q(&h->p);
    const ReadOut ro = {nullptr, nullptr, nullptr, nullptr};
    const InitIn in = {nullptr, nullptr};
    const int64_t de = h->p.diag_every > 0 ? h->p.diag_every : 0;
    bool any_diag = false;
    for (int64_t k = 0; k < nsteps; ++k) {
        const int64_t t = h->step + k;
        const int diag = de > 0 && (t % de) == 0;
        any_diag |= (diag != 0);
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
        if (h->timing) {
            e0 = next_event(h); e1 = next_event(h); e2 = next_event(h);
            if (!e0 || !e1 || !e2) { set_error("event pool"); return LBM_E_DEVICE; }
            HIPRET(hipEventRecord(e0, h->stream));
        }
        const int par = (int)(t & 1);
        HIPRET(launch_phi(storage, qp, par, h->ddesc, h->dtiles, h->ntiles, h->stream));
        if (h->nwalls) HIPRET(launch_wall(storage, MODE_STEP, h->ddesc, h->dwalls, h->nwalls, h->stream));
        if (h->timing) HIPRET(hipEventRecord(e1, h->stream));
        HIPRET(launch_sweep(storage, qp, h->p.subvoxel ? MODE_STEP_SV : MODE_STEP, h->L.tx, par, h->ddesc, h->dtiles, h->ntiles, diag, ro, in,
                            h->stream));
        if (h->nghosts)
            HIPRET(launch_ghosts(storage, qp, h->ddesc, h->dghosts, h->nghosts, h->stream));
        HIPRET(launch_advance(h->ddesc, 1, h->stream));
        if (h->timing) HIPRET(hipEventRecord(e2, h->stream));
    }
    h->step += nsteps;
    if (any_diag && !h->unstable_pending) {
        HIPRET(hipMemcpyAsync(h->h_unstable, &h->ddesc->unstable, sizeof(int),
                              hipMemcpyDeviceToHost, h->stream));
        HIPRET(hipEventRecord(h->unstable_ev, h->stream));
        h->unstable_pending = true;
    }
    return LBM_OK;
}

extern "C" int lbm_sync(lbm_handle* h) {
    if (!h) { set_error("handle is NULL"); return LBM_E_INVAL; }
    HIPRET(hipSetDevice(h->device));
    HIPRET(hipStreamSynchronize(h->stream));
    return poll_unstable(h, true);
}

extern "C" int64_t lbm_step_count(const lbm_handle* h) { return h ? h->step : -1; }

extern "C" int lbm_read_fields(lbm_handle* h, uint32_t mask, double* phi, double* P, double* u,
                               double* pops) {
    if (!h) { set_error("handle is NULL"); return LBM_E_INVAL; }
    HIPRET(hipSetDevice(h->device));
    HIPRET(hipStreamSynchronize(h->stream));
    return read_lattice(h->p.storage, h->hdesc, (int)(h->step & 1), h->ddesc, h->dtiles, h->ntiles,
                        h->dwalls, h->nwalls, mask, phi, P, u, pops, h->stream);
}

extern "C" int lbm_reduce(lbm_handle* h, lbm_diag* d) {
    if (!h || !d) { set_error("NULL argument"); return LBM_E_INVAL; }
    HIPRET(hipSetDevice(h->device));
    int rc = read_lattice(h->p.storage, h->hdesc, (int)(h->step & 1), h->ddesc, h->dtiles,
                          h->ntiles, h->dwalls, h->nwalls, 0, nullptr, nullptr, nullptr, nullptr, h->stream);
    if (rc != LBM_OK) return rc;
    double v[NPART];
    HIPRET(hipMemcpy(v, h->ddesc->diag, sizeof(v), hipMemcpyDeviceToHost));
    d->step = h->step;
    d->phi_sum = v[P_PHI];
    d->mom[0] = v[P_MX]; d->mom[1] = v[P_MY]; d->mom[2] = v[P_MZ];
    d->u_max = v[P_UMAX];
    d->n_nan = (int64_t)v[P_NAN];
    d->n_liq = (int64_t)v[P_NLIQ];
    d->n_gas = (int64_t)v[P_NGAS];
    d->P_liq_mean = d->n_liq ? v[P_PLIQ] / (double)d->n_liq : 0.0;
    d->P_gas_mean = d->n_gas ? v[P_PGAS] / (double)d->n_gas : 0.0;
    return LBM_OK;
}

extern "C" int lbm_set_timing(lbm_handle* h, int32_t on) {
    if (!h) { set_error("handle is NULL"); return LBM_E_INVAL; }
    h->timing = on != 0;
    return LBM_OK;
}

extern "C" int lbm_get_timing(lbm_handle* h, double* phi_ms, double* sweep_ms, int64_t* steps) {
    if (!h) { set_error("handle is NULL"); return LBM_E_INVAL; }
    HIPRET(hipSetDevice(h->device));
    HIPRET(hipStreamSynchronize(h->stream));
    for (size_t k = 0; k + 2 < h->ev_used; k += 3) {
        float a = 0.f, b = 0.f;
        HIPRET(hipEventElapsedTime(&a, h->ev_pool[k], h->ev_pool[k + 1]));
        HIPRET(hipEventElapsedTime(&b, h->ev_pool[k + 1], h->ev_pool[k + 2]));
        h->phi_ms += a;
        h->sweep_ms += b;
        h->steps_timed += 1;
    }
    h->ev_used = 0;
    if (phi_ms) *phi_ms = h->phi_ms;
    if (sweep_ms) *sweep_ms = h->sweep_ms;
    if (steps) *steps = h->steps_timed;
    h->phi_ms = h->sweep_ms = 0.0;
    h->steps_timed = 0;
    return LBM_OK;
}

extern "C" int lbm_destroy(lbm_handle* h) {
    if (!h) return LBM_OK;
    hipSetDevice(h->device);
    hipStreamSynchronize(h->stream);
    free_handle(h);
    return LBM_OK;
}

extern "C" int lbm_get_info(const lbm_handle* h, lbm_info* info) {
    if (!h || !info) { set_error("NULL argument"); return LBM_E_INVAL; }
    info->n_nodes = h->L.N;
    info->n_fluid = h->L.n_fluid;
    info->n_ghost = h->L.n_ghost;
    info->n_solid = h->L.n_solid;
    info->n_tiles = h->ntiles;
    info->footprint = h->L.total;
    int sh, sg, sphi;
    storage_sizes(h->p.storage, &sh, &sg, &sphi);
    info->bytes_per_fluid_update = 2.0 * (phase_q(&h->p) * sh + QG * sg);
    return LBM_OK;
}
