// lbm_api.hip -- single-lattice C ABI (include/lbm.h).
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "handle.hpp"
#include "lattice_host.hpp"
#include "pflbm.hpp"

using namespace pflbm;


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
    for (int a = 0; a < 2; ++a) {
        for (int b = 0; b < 2; ++b)
            if (h->one[a][b]) hipGraphExecDestroy(h->one[a][b]);
        if (h->chunk[a]) hipGraphExecDestroy(h->chunk[a]);
    }
    if (h->cap_stream) hipStreamDestroy(h->cap_stream);
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

static bool diag_step(const lbm_handle* h, int64_t t) {
    const int64_t de = h->p.diag_every > 0 ? h->p.diag_every : 0;
    return de > 0 && (t % de) == 0;
}

// Queue the kernels of steps t0 .. t0+n-1 on stream s: per step the phi pass,
// the wall pass, the sweep (its AA parity and diagnostic instance chosen by
// the step), the pressure ghosts and the step counter.  With events (timed
// runs) the phi + wall passes and the sweep kernel alone are bracketed.
static int enqueue_steps(lbm_handle* h, int64_t t0, int64_t n, hipStream_t s, bool events) {
    const int storage = h->p.storage;
    const int qp = phase_q(&h->p);
    const ReadOut ro = {nullptr, nullptr, nullptr, nullptr};
    const InitIn in = {nullptr, nullptr};
    for (int64_t k = 0; k < n; ++k) {
        const int64_t t = t0 + k;
        const int diag = diag_step(h, t) ? 1 : 0;
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
        if (events) {
            e0 = next_event(h); e1 = next_event(h); e2 = next_event(h);
            if (!e0 || !e1 || !e2) { set_error("event pool"); return LBM_E_DEVICE; }
            HIPRET(hipEventRecord(e0, s));
        }
        const int par = (int)(t & 1);
        HIPRET(launch_phi(storage, qp, par, h->ddesc, h->dtiles, h->ntiles, s));
        if (h->nwalls) HIPRET(launch_wall(storage, MODE_STEP, h->ddesc, h->dwalls, h->nwalls, s));
        if (events) HIPRET(hipEventRecord(e1, s));
        HIPRET(launch_sweep(storage, qp, h->p.subvoxel ? MODE_STEP_SV : MODE_STEP, h->L.tx, par, h->ddesc,
                            h->dtiles, h->ntiles, diag, ro, in, s));
        if (events) HIPRET(hipEventRecord(e2, s));
        if (h->nghosts) HIPRET(launch_ghosts(storage, qp, h->ddesc, h->dghosts, h->nghosts, s));
        HIPRET(launch_advance(h->ddesc, 1, s));
    }
    return LBM_OK;
}

// Capture n steps starting at parity par (diagnostic step or not for a single
// step) into an executable graph.  The kernels read the step, and with it
// the face pressures, from the descriptor, so the graph replays at any step
// of that parity and diagnostic kind.
static int capture_steps(lbm_handle* h, int par, int diag, int64_t n, hipGraphExec_t* out) {
    // a representative step of the wanted kind: the first step >= 2 with the
    // parity par that is (or is not) a diagnostic step
    const int64_t de = h->p.diag_every > 0 ? h->p.diag_every : 0;
    int64_t t0 = -1;
    if (diag) {
        for (int64_t m = 1; m <= 2 && t0 < 0; ++m)
            if (((de * m) & 1) == par) t0 = de * m;
    } else {
        for (int64_t t = 2 + par; t < 2 + 2 * (de + 2) + 2 * n && t0 < 0; t += 2) {
            bool any = false;
            for (int64_t k = 0; k < n; ++k) any |= diag_step(h, t + k);
            if (!any) t0 = t;
        }
    }
    if (t0 < 0) { *out = nullptr; return LBM_OK; }   // no step of this kind exists
    hipGraph_t g = nullptr;
    HIPRET(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_steps(h, t0, n, h->cap_stream, false);
    const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc != LBM_OK) { if (g) hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) { set_error("hipStreamEndCapture: %s", hipGetErrorString(e)); return LBM_E_DEVICE; }
    const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e2 != hipSuccess) { set_error("hipGraphInstantiate: %s", hipGetErrorString(e2)); return LBM_E_DEVICE; }
    return LBM_OK;
}

static int ensure_graphs(lbm_handle* h) {
    if (h->graphs_ready) return LBM_OK;
    if (!h->cap_stream) HIPRET(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    for (int par = 0; par < 2; ++par) {
        for (int diag = 0; diag < 2; ++diag) {
            if (diag && h->p.diag_every <= 0) continue;
            int rc = capture_steps(h, par, diag, 1, &h->one[par][diag]);
            if (rc != LBM_OK) return rc;
        }
        int rc = capture_steps(h, par, 0, GRAPH_CHUNK, &h->chunk[par]);
        if (rc != LBM_OK) return rc;
    }
    h->graphs_ready = true;
    return LBM_OK;
}

extern "C" int lbm_step(lbm_handle* h, int64_t nsteps) {
    if (!h) { set_error("handle is NULL"); return LBM_E_INVAL; }
    if (nsteps < 0) { set_error("nsteps < 0"); return LBM_E_INVAL; }
    int rc = poll_unstable(h, false);
    if (rc != LBM_OK) return rc;
    if (nsteps == 0) return LBM_OK;
    HIPRET(hipSetDevice(h->device));
    const int64_t de = h->p.diag_every > 0 ? h->p.diag_every : 0;
    bool any_diag = false;
    for (int64_t k = 0; k < nsteps && !any_diag; ++k) any_diag = diag_step(h, h->step + k);
    if (h->timing) {
        // timed runs launch each kernel on its own, bracketed by events
        rc = enqueue_steps(h, h->step, nsteps, h->stream, true);
        if (rc != LBM_OK) return rc;
    } else {
        rc = ensure_graphs(h);
        if (rc != LBM_OK) return rc;
        int64_t k = 0;
        while (k < nsteps) {
            const int64_t t = h->step + k;
            const int par = (int)(t & 1);
            bool chunk_ok = h->chunk[par] && nsteps - k >= GRAPH_CHUNK;
            if (chunk_ok && de > 0) {
                const int64_t next_diag = ((t + de - 1) / de) * de;
                chunk_ok = next_diag >= t + GRAPH_CHUNK;
            }
            hipGraphExec_t g = chunk_ok ? h->chunk[par] : h->one[par][diag_step(h, t) ? 1 : 0];
            if (!g) { set_error("no step graph for step %lld", (long long)t); return LBM_E_STATE; }
            HIPRET(hipGraphLaunch(g, h->stream));
            k += chunk_ok ? GRAPH_CHUNK : 1;
        }
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
