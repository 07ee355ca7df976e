// serve.hip -- continuous batching of independent lattices on one GPU.
//
// lbm_submit validates a request, classifies its nodes and lays out its
// device state on the caller's thread and queues it.  A worker thread owns
// the GPU side and runs scheduling intervals of an even number of steps:
// each step is one phi launch over the concatenated tile tables of all
// resident lattices, one wall-pass launch, one sweep launch per (phase
// lattice, tile width, wall kind), one ghost launch and one step-counter
// launch over the resident slots.  While an interval runs on the compute
// stream, the worker reads back the lattices that finished in the previous
// interval and uploads newly admitted ones on a second stream, into arena
// blocks and descriptor slots that no running kernel touches (the tables
// of the running interval list neither).  At the next boundary the new
// lattices join and the finished ones leave the tables.  A request is
// admitted when a descriptor slot is free, its footprint fits a free block
// of the server's HBM arena and the resident node count stays within the
// configured cap (admitting more than fills the GPU only slows every
// resident lattice down).  Every admitted lattice starts at step 0 and joins
// at a boundary, where every resident lattice is at an even step, so all
// share the AA parity of every step; a lattice whose step count is reached
// stops on the device (its tiles return at once).  Tiles never mix lattices
// and every reduction is per lattice, so a lattice's result does not depend
// on what it was batched with.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/lbm.h"
#include "lattice_host.hpp"
#include "pflbm.hpp"

using namespace pflbm;

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of freed blocks.
class ArenaAllocator {
public:
    void reset(size_t size) { free_.clear(); if (size) free_[0] = size; }
    bool alloc(size_t n, size_t* off) {
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = round_up(n);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) { n += next->second; next = free_.erase(next); }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) { prev->second += n; return; }
        }
        free_[off] = n;
    }
    size_t largest() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
private:
    std::map<size_t, size_t> free_;
};

struct Job {
    uint64_t ticket = 0;
    lbm_params p;
    lbm_geometry geo;
    std::vector<uint8_t> solid;
    std::vector<double> sdf;
    std::vector<double> phi0, u0, P0;
    int64_t nsteps = 0;
    double arrival_s = 0.0;
    double t_submit = 0.0, t_admit = 0.0, t_finish = 0.0;
    // placement (the layout is built by lbm_submit)
    LatticeLayout L;
    size_t off = 0, bytes = 0;
    int slot = -1;
    Desc hdesc;
    int64_t step = 0;
    // result
    int status = LBM_OK;
    double *phi = nullptr, *P = nullptr, *u = nullptr;
    lbm_diag diag;
    ~Job() { free(phi); free(P); free(u); }
};

}  // namespace

struct lbm_server {
    lbm_server_cfg cfg;
    int interval = 32;
    hipStream_t stream = nullptr;      // intervals
    hipStream_t up_stream = nullptr;   // uploads and read-backs, beside a running interval
    hipStream_t cap_stream = nullptr;  // graph capture only (nothing executes on it)
    char* arena = nullptr;
    size_t arena_bytes = 0;
    ArenaAllocator alloc;
    Desc* dtable = nullptr;
    Desc* hmirror = nullptr;     // pinned copy of the table after each interval
    std::vector<int> free_slots;
    hipEvent_t ev = nullptr;
    // batched work tables of the resident set (rebuilt at a boundary, when
    // no interval runs; the host vectors stay alive until their copies ran)
    Tile* dtiles = nullptr;
    size_t tiles_cap = 0;
    GhostRef* dghosts = nullptr;
    size_t ghosts_cap = 0;
    WallRef* dwalls = nullptr;         // near-wall fluid nodes of every resident lattice
    size_t walls_cap = 0;
    int* dslots = nullptr;             // descriptor slots of the resident lattices
    size_t slots_cap = 0;
    std::vector<Tile> htiles;
    std::vector<GhostRef> hghosts;
    std::vector<WallRef> hwalls;
    std::vector<int> hslots;
    int nwalls = 0, nslots = 0, nmirror = 0;   // nmirror: highest resident slot + 1
    struct Group { int qp, tx, off, n, sv = 0; };   // sv: lattices with sub-voxel walls
    std::vector<Group> groups;         // sweep launches: one per (phase lattice, tile width)
    std::vector<Group> phi_groups;     // phi launches: one per phase lattice (tx unused)
    std::vector<Group> ghost_groups;   // ghost launches: one per phase lattice (tx unused)
    int ntiles = 0, nghosts = 0;
    int64_t resident_nodes = 0;        // active + pending
    hipGraphExec_t gexec = nullptr;    // the intervals of the current tables (null: not captured)
    // read-back staging (device), grown on demand
    double* dstage = nullptr;
    size_t stage_cap = 0;
    // jobs
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<Job>> queue;
    std::vector<std::unique_ptr<Job>> active;     // in the tables (worker thread only)
    std::vector<std::unique_ptr<Job>> pending;    // uploaded, join at the next boundary
    std::vector<std::unique_ptr<Job>> finishing;  // reached their step count, out of the tables
    std::unordered_map<uint64_t, std::unique_ptr<Job>> done;
    std::unordered_set<uint64_t> in_flight;                     // queued or resident
    uint64_t next_ticket = 1;
    int64_t outstanding = 0;
    bool stop = false;
    int fatal = LBM_OK;
    std::string fatal_msg;
    std::thread worker;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

int device_error(const char* what, hipError_t e) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return LBM_E_DEVICE;
}

#define SRV_CHK(expr)                                          \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return device_error(#expr, e_);  \
    } while (0)

void finish_job(lbm_server* s, std::unique_ptr<Job> job) {
    job->t_finish = s->now();
    std::lock_guard<std::mutex> lk(s->mu);
    s->outstanding -= 1;
    s->in_flight.erase(job->ticket);
    s->done[job->ticket] = std::move(job);
    s->cv_done.notify_all();
}

// Place queue heads that fit, uploading them on the side stream (no running
// kernel touches a free arena block or slot).  Returns LBM_OK or a device
// error.
int admit(lbm_server* s) {
    for (;;) {
        std::unique_ptr<Job> job;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->queue.empty()) return LBM_OK;
            job = std::move(s->queue.front());
            s->queue.pop_front();
        }
        auto requeue = [&]() {
            std::lock_guard<std::mutex> lk(s->mu);
            s->queue.push_front(std::move(job));
        };
        const bool resident = !s->active.empty() || !s->pending.empty();
        const bool over_cap = s->cfg.max_resident_nodes > 0 && resident &&
                              s->resident_nodes + job->L.N > s->cfg.max_resident_nodes;
        if (over_cap || s->free_slots.empty() || !s->alloc.alloc(job->bytes, &job->off)) {
            if (!resident && s->finishing.empty()) {
                // nothing will be freed: the request can never be placed
                set_error("request of %zu bytes does not fit the arena", job->bytes);
                job->status = LBM_E_NOMEM;
                finish_job(s, std::move(job));
                continue;
            }
            requeue();
            return LBM_OK;
        }
        job->slot = s->free_slots.back();
        s->free_slots.pop_back();
        lbm_init init;
        memset(&init, 0, sizeof(init));
        init.kind = LBM_INIT_FIELDS;
        init.phi = job->phi0.data();
        init.u = job->u0.empty() ? nullptr : job->u0.data();
        init.P = job->P0.empty() ? nullptr : job->P0.data();
        int rc = upload_and_init(&job->p, &job->geo, &init, job->L, s->arena + job->off,
                                 &job->hdesc, s->up_stream);
        if (rc == LBM_OK) {
            job->hdesc.stop_step = job->nsteps;
            hipError_t e = hipMemcpyAsync(s->dtable + job->slot, &job->hdesc, sizeof(Desc),
                                          hipMemcpyHostToDevice, s->up_stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s->up_stream);
            if (e != hipSuccess) rc = device_error("descriptor upload", e);
        }
        if (rc != LBM_OK) {
            s->alloc.release(job->off, job->bytes);
            s->free_slots.push_back(job->slot);
            job->status = rc;
            finish_job(s, std::move(job));
            return rc;
        }
        // host copies no longer needed once the lattice is on the device
        std::vector<double>().swap(job->phi0);
        std::vector<double>().swap(job->u0);
        std::vector<double>().swap(job->P0);
        std::vector<uint8_t>().swap(job->solid);
        std::vector<double>().swap(job->sdf);
        std::vector<double>().swap(job->L.wall);
        std::vector<uint8_t>().swap(job->L.flag);
        std::vector<uint32_t>().swap(job->L.link);
        std::vector<int32_t>().swap(job->L.wslot);
        job->geo.solid = nullptr;
        job->geo.sdf = nullptr;
        job->t_admit = s->now();
        job->step = 0;
        s->resident_nodes += job->L.N;
        s->pending.push_back(std::move(job));
    }
}

// Read back every lattice that left the tables, on the side stream, and
// free its arena block and slot.
int read_back(lbm_server* s) {
    for (auto& jp : s->finishing) {
        std::unique_ptr<Job> job = std::move(jp);
        const int64_t N = job->L.N;
        job->phi = (double*)malloc(N * sizeof(double));
        job->P = (double*)malloc(N * sizeof(double));
        job->u = (double*)malloc(3 * N * sizeof(double));
        int rc = LBM_OK;
        if (!job->phi || !job->P || !job->u) {
            set_error("host allocation of a result failed");
            job->status = LBM_E_NOMEM;
        } else {
            const uint32_t mask = LBM_PHI | LBM_P | LBM_U;
            const size_t nd = read_staging_elems(job->hdesc, mask, job->phi, job->P, job->u, nullptr);
            if (nd > s->stage_cap) {
                if (s->dstage) SRV_CHK(hipFree(s->dstage));
                s->dstage = nullptr;
                s->stage_cap = std::max(nd, 2 * s->stage_cap);
                SRV_CHK(hipMalloc(&s->dstage, s->stage_cap * sizeof(double)));
            }
            Desc* dd = s->dtable + job->slot;
            const Tile* dt = (const Tile*)(s->arena + job->off + job->L.off_tiles);
            const WallRef* dw = (const WallRef*)(s->arena + job->off + job->L.off_wrefs);
            rc = read_lattice_staged(s->cfg.storage, job->hdesc, (int)(job->nsteps & 1), dd, dt,
                                     (int)job->L.tiles.size(), dw, (int)job->L.n_wall, mask, job->phi,
                                     job->P, job->u, nullptr, s->dstage, s->up_stream);
            double v[NPART];
            if (rc == LBM_OK) {
                hipError_t e = hipMemcpyAsync(v, dd->diag, sizeof(v), hipMemcpyDeviceToHost, s->up_stream);
                if (e == hipSuccess) e = hipStreamSynchronize(s->up_stream);
                if (e != hipSuccess) rc = device_error("diagnostics copy", e);
            }
            if (rc != LBM_OK) {
                job->status = rc;
            } else {
                lbm_diag& d = job->diag;
                d.step = job->nsteps;
                d.phi_sum = v[P_PHI];
                d.mom[0] = v[P_MX]; d.mom[1] = v[P_MY]; d.mom[2] = v[P_MZ];
                d.u_max = v[P_UMAX];
                d.n_nan = (int64_t)v[P_NAN];
                d.n_liq = (int64_t)v[P_NLIQ];
                d.n_gas = (int64_t)v[P_NGAS];
                d.P_liq_mean = d.n_liq ? v[P_PLIQ] / (double)d.n_liq : 0.0;
                d.P_gas_mean = d.n_gas ? v[P_PGAS] / (double)d.n_gas : 0.0;
                job->status = d.n_nan ? LBM_E_UNSTABLE : LBM_OK;
            }
        }
        s->alloc.release(job->off, job->bytes);
        s->free_slots.push_back(job->slot);
        finish_job(s, std::move(job));
        if (rc != LBM_OK) {
            s->finishing.clear();
            return rc;
        }
    }
    s->finishing.clear();
    return LBM_OK;
}

template <typename V>
int upload_table(V** dptr, size_t* cap, const std::vector<V>& h, hipStream_t st) {
    if (h.size() > *cap) {
        if (*dptr) SRV_CHK(hipFree(*dptr));
        *dptr = nullptr;
        *cap = std::max(h.size(), 2 * *cap);
        SRV_CHK(hipMalloc((void**)dptr, *cap * sizeof(V)));
    }
    if (!h.empty()) SRV_CHK(hipMemcpyAsync(*dptr, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, st));
    return LBM_OK;
}

// Concatenated tile tables of all resident lattices, grouped by phase
// lattice and, within it, by tile width and wall kind (each kernel instance
// handles one of each); ghost tables grouped by phase lattice.  Called at a
// boundary (no interval running); the copies are queued on the compute
// stream ahead of the next interval.
int rebuild_tables(lbm_server* s) {
    std::vector<Tile>& tiles = s->htiles;
    std::vector<GhostRef>& ghosts = s->hghosts;
    std::vector<WallRef>& walls = s->hwalls;
    tiles.clear();
    ghosts.clear();
    walls.clear();
    s->hslots.clear();
    s->groups.clear();
    s->phi_groups.clear();
    s->ghost_groups.clear();
    for (int qp : {7, 19}) {
        const int qoff = (int)tiles.size();
        for (int tx : {64, 32, 16}) {
            // lattices with sub-voxel walls run their own instance of the
            // sweep, the others the plain one: each lattice always runs the
            // same code as when alone (bitwise the same result)
            for (int sv : {0, 1}) {
                const int off = (int)tiles.size();
                for (auto& j : s->active) {
                    if (j->L.tx != tx || phase_q(&j->p) != qp || (j->p.subvoxel ? 1 : 0) != sv) continue;
                    for (Tile t : j->L.tiles) { t.lat = j->slot; tiles.push_back(t); }
                }
                if ((int)tiles.size() > off) s->groups.push_back({qp, tx, off, (int)tiles.size() - off, sv});
            }
        }
        if ((int)tiles.size() > qoff) s->phi_groups.push_back({qp, 0, qoff, (int)tiles.size() - qoff});
        const int goff = (int)ghosts.size();
        for (auto& j : s->active) {
            if (phase_q(&j->p) != qp) continue;
            for (GhostRef g : j->L.ghosts) { g.lat = j->slot; ghosts.push_back(g); }
        }
        if ((int)ghosts.size() > goff)
            s->ghost_groups.push_back({qp, 0, goff, (int)ghosts.size() - goff});
    }
    for (auto& j : s->active) {
        for (WallRef w : j->L.walls) { w.lat = j->slot; walls.push_back(w); }
        // the wall pass takes its lattice constants per block: pad each
        // lattice's list to whole blocks (node -1 is skipped)
        while (walls.size() % NTHREADS) walls.push_back(WallRef{j->slot, -1, 0, 0u});
        s->hslots.push_back(j->slot);
    }
    s->nmirror = 0;
    for (int sl : s->hslots) s->nmirror = std::max(s->nmirror, sl + 1);
    int rc = upload_table(&s->dwalls, &s->walls_cap, walls, s->stream);
    if (rc == LBM_OK) rc = upload_table(&s->dtiles, &s->tiles_cap, tiles, s->stream);
    if (rc == LBM_OK) rc = upload_table(&s->dghosts, &s->ghosts_cap, ghosts, s->stream);
    if (rc == LBM_OK) rc = upload_table(&s->dslots, &s->slots_cap, s->hslots, s->stream);
    if (rc != LBM_OK) return rc;
    s->nwalls = (int)walls.size();
    s->ntiles = (int)tiles.size();
    s->nghosts = (int)ghosts.size();
    s->nslots = (int)s->hslots.size();
    if (s->gexec) { SRV_CHK(hipGraphExecDestroy(s->gexec)); s->gexec = nullptr; }
    return LBM_OK;
}

// The launches of one interval (every step starts at the parity of its index).
hipError_t enqueue_steps(lbm_server* s, hipStream_t st) {
    const int storage = s->cfg.storage;
    const ReadOut ro = {nullptr, nullptr, nullptr, nullptr};
    const InitIn in = {nullptr, nullptr};
    for (int k = 0; k < s->interval; ++k) {
        const int par = k & 1;
        hipError_t e = hipSuccess;
        for (const auto& g : s->phi_groups)
            if (e == hipSuccess)
                e = launch_phi(storage, g.qp, par, s->dtable, s->dtiles + g.off, g.n, st, 0);
        if (e == hipSuccess && s->nwalls)
            e = launch_wall(storage, MODE_STEP, s->dtable, s->dwalls, s->nwalls, st);
        for (const auto& g : s->groups)
            if (e == hipSuccess)
                e = launch_sweep(storage, g.qp, g.sv ? MODE_STEP_SV : MODE_STEP, g.tx, par, s->dtable,
                                 s->dtiles + g.off, g.n, 0, ro, in, st);
        for (const auto& g : s->ghost_groups)
            if (e == hipSuccess)
                e = launch_ghosts(storage, g.qp, s->dtable, s->dghosts + g.off, g.n, st);
        if (e == hipSuccess) e = launch_advance_list(s->dtable, s->dslots, s->nslots, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Queue one interval of the current tables and the copy of the table's step
// counters; the event marks its end.  A freshly rebuilt table set runs as
// plain launches and is captured into a graph afterwards (while the interval
// runs), which the following intervals of the same set replay.
int launch_interval(lbm_server* s) {
    if (s->cfg.use_graph && s->gexec) SRV_CHK(hipGraphLaunch(s->gexec, s->stream));
    else SRV_CHK(enqueue_steps(s, s->stream));
    SRV_CHK(hipMemcpyAsync(s->hmirror, s->dtable, (size_t)s->nmirror * sizeof(Desc),
                           hipMemcpyDeviceToHost, s->stream));
    SRV_CHK(hipEventRecord(s->ev, s->stream));
    return LBM_OK;
}

int capture_interval(lbm_server* s) {
    if (!s->cfg.use_graph || s->gexec) return LBM_OK;
    hipGraph_t g = nullptr;
    SRV_CHK(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipError_t e = enqueue_steps(s, s->cap_stream);
    const hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
    if (e != hipSuccess) { if (g) hipGraphDestroy(g); return device_error("capture", e); }
    if (e2 != hipSuccess) return device_error("hipStreamEndCapture", e2);
    const hipError_t e3 = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e3 != hipSuccess) return device_error("hipGraphInstantiate", e3);
    return LBM_OK;
}

void fail_all(lbm_server* s, int code) {
    const char* msg = lbm_last_error();
    std::string m = msg ? msg : "";
    if (s->stream) hipStreamSynchronize(s->stream);
    if (s->up_stream) hipStreamSynchronize(s->up_stream);
    std::vector<std::unique_ptr<Job>> jobs;
    for (auto* v : {&s->active, &s->pending, &s->finishing}) {
        for (auto& j : *v) jobs.push_back(std::move(j));
        v->clear();
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& j : s->queue) jobs.push_back(std::move(j));
        s->queue.clear();
        s->fatal = code;
        s->fatal_msg = m;
    }
    for (auto& j : jobs) { j->status = code; finish_job(s, std::move(j)); }
}

void worker_main(lbm_server* s) {
    if (hipSetDevice(s->cfg.device) != hipSuccess) { fail_all(s, LBM_E_DEVICE); return; }
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                return s->stop || !s->queue.empty() || !s->active.empty() || !s->pending.empty() ||
                       !s->finishing.empty();
            });
            if (s->stop) break;
        }
        int rc = LBM_OK;
        const bool running = !s->active.empty();
        if (running) rc = launch_interval(s);
        // beside the running interval: read back what left the tables, admit
        // from the queue, capture the running set's graph for its next turn
        if (rc == LBM_OK) rc = read_back(s);
        if (rc == LBM_OK) rc = admit(s);
        if (rc == LBM_OK && running) rc = capture_interval(s);
        if (rc == LBM_OK && running) {
            const hipError_t e = hipEventSynchronize(s->ev);
            if (e != hipSuccess) rc = device_error("interval", e);
        }
        bool changed = !s->pending.empty();
        if (rc == LBM_OK && running) {
            for (size_t k = 0; k < s->active.size();) {
                Job* j = s->active[k].get();
                j->step = std::min(j->step + s->interval, j->nsteps);
                if (s->hmirror[j->slot].step != j->step) {
                    set_error("lattice in slot %d is at step %lld, expected %lld", j->slot,
                              (long long)s->hmirror[j->slot].step, (long long)j->step);
                    rc = LBM_E_STATE;
                    break;
                }
                if (j->step >= j->nsteps) {
                    s->resident_nodes -= j->L.N;
                    s->finishing.push_back(std::move(s->active[k]));
                    s->active.erase(s->active.begin() + k);
                    changed = true;
                } else {
                    ++k;
                }
            }
        }
        if (rc == LBM_OK && changed) {
            for (auto& j : s->pending) s->active.push_back(std::move(j));
            s->pending.clear();
            rc = rebuild_tables(s);
        }
        if (rc != LBM_OK) { fail_all(s, rc); return; }
    }
}

}  // namespace

extern "C" int lbm_server_create(const lbm_server_cfg* cfg, lbm_server** out) {
    if (!out || !cfg) { set_error("NULL argument"); return LBM_E_INVAL; }
    *out = nullptr;
    if (cfg->max_slots < 0 || cfg->max_slots > 256) { set_error("max_slots must be in [0, 256]"); return LBM_E_INVAL; }
    if (cfg->storage < LBM_FP64 || cfg->storage >= LBM_FP16_SHIFT_ALL) {
        set_error(cfg->storage == LBM_FP16_SHIFT_ALL ? "storage LBM_FP16_SHIFT_ALL is not supported"
                                                     : "unknown storage mode %d", cfg->storage);
        return LBM_E_INVAL;
    }
    if (cfg->ticks_per_sync < 0) { set_error("ticks_per_sync < 0"); return LBM_E_INVAL; }
    if (cfg->max_resident_nodes < 0) { set_error("max_resident_nodes < 0"); return LBM_E_INVAL; }
    std::unique_ptr<lbm_server> s(new (std::nothrow) lbm_server());
    if (!s) { set_error("host allocation failed"); return LBM_E_NOMEM; }
    s->cfg = *cfg;
    if (s->cfg.max_slots == 0) s->cfg.max_slots = 256;
    const int k = cfg->ticks_per_sync ? cfg->ticks_per_sync : 32;
    s->interval = (k + 1) / 2 * 2;
    auto cleanup = [&](int rc) {
        if (s->ev) hipEventDestroy(s->ev);
        if (s->hmirror) hipHostFree(s->hmirror);
        if (s->dtable) hipFree(s->dtable);
        if (s->arena) hipFree(s->arena);
        if (s->stream) hipStreamDestroy(s->stream);
        if (s->up_stream) hipStreamDestroy(s->up_stream);
        if (s->cap_stream) hipStreamDestroy(s->cap_stream);
        return rc;
    };
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) return cleanup(device_error("hipSetDevice", e));
    size_t budget = cfg->hbm_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess) return cleanup(device_error("hipMemGetInfo", e));
        budget = fr / 10 * 8;
    }
    budget = budget / kAlign * kAlign;
    if (budget == 0) { set_error("HBM budget is zero"); return LBM_E_INVAL; }
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->up_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&s->arena, budget);
    if (e == hipSuccess) e = hipMalloc(&s->dtable, (size_t)s->cfg.max_slots * sizeof(Desc));
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->hmirror, (size_t)s->cfg.max_slots * sizeof(Desc),
                                           hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        const int rc = e == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_DEVICE;
        set_error("server set-up: %s", hipGetErrorString(e));
        return cleanup(rc);
    }
    // unused slots read as stopped (step 0, stop step 0)
    e = hipMemset(s->dtable, 0, (size_t)s->cfg.max_slots * sizeof(Desc));
    if (e != hipSuccess) return cleanup(device_error("hipMemset", e));
    s->arena_bytes = budget;
    s->alloc.reset(budget);
    for (int i = s->cfg.max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->t0 = std::chrono::steady_clock::now();
    lbm_server* raw = s.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return LBM_OK;
}

extern "C" int lbm_submit(lbm_server* s, const lbm_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) { set_error("NULL argument"); return LBM_E_INVAL; }
    const double t = s->now();
    std::unique_ptr<Job> job(new (std::nothrow) Job());
    if (!job) { set_error("host allocation failed"); return LBM_E_NOMEM; }
    job->p = req->params;
    job->p.storage = s->cfg.storage;
    job->p.diag_every = 0;
    job->geo = req->geometry;
    if (req->init.kind != LBM_INIT_FIELDS || !req->init.phi) {
        set_error("a request starts from fields (LBM_INIT_FIELDS with phi)");
        return LBM_E_INVAL;
    }
    if (req->nsteps < 1) { set_error("nsteps must be >= 1"); return LBM_E_INVAL; }
    int rc = validate_params(&job->p, &job->geo);
    if (rc != LBM_OK) return rc;
    const size_t need = footprint_bytes(&job->p);
    if (need > s->arena_bytes) {
        set_error("footprint %zu bytes exceeds the server budget %zu", need, s->arena_bytes);
        return LBM_E_INVAL;
    }
    const int64_t N = (int64_t)job->p.nx * job->p.ny * job->p.nz;
    try {
        if (req->geometry.solid) job->solid.assign(req->geometry.solid, req->geometry.solid + N);
        if (req->geometry.sdf) job->sdf.assign(req->geometry.sdf, req->geometry.sdf + N);
        job->phi0.assign(req->init.phi, req->init.phi + N);
        if (req->init.u) job->u0.assign(req->init.u, req->init.u + 3 * N);
        if (req->init.P) job->P0.assign(req->init.P, req->init.P + N);
    } catch (...) {
        set_error("host allocation failed");
        return LBM_E_NOMEM;
    }
    job->geo.solid = job->solid.empty() ? nullptr : job->solid.data();
    job->geo.sdf = job->sdf.empty() ? nullptr : job->sdf.data();
    // node classification, tile table and arena layout on the caller's
    // thread: the worker only uploads
    rc = build_layout(&job->p, &job->geo, 0, &job->L);
    if (rc != LBM_OK) return rc;
    job->bytes = job->L.total;
    job->nsteps = req->nsteps;
    job->arrival_s = req->arrival_s;
    job->t_submit = t;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal != LBM_OK) { set_error("server stopped: %s", s->fatal_msg.c_str()); return s->fatal; }
    job->ticket = s->next_ticket++;
    *ticket = job->ticket;
    s->outstanding += 1;
    s->in_flight.insert(job->ticket);
    s->queue.push_back(std::move(job));
    s->cv_work.notify_one();
    return LBM_OK;
}

extern "C" int lbm_poll(lbm_server* s, uint64_t ticket, lbm_result* res) {
    if (!s || !res) { set_error("NULL argument"); return LBM_E_INVAL; }
    std::unique_ptr<Job> job;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->done.find(ticket);
        if (it == s->done.end()) {
            if (s->in_flight.count(ticket)) return LBM_PENDING;
            set_error("ticket %llu is unknown or was already returned", (unsigned long long)ticket);
            return LBM_E_INVAL;
        }
        job = std::move(it->second);
        s->done.erase(it);
    }
    memset(res, 0, sizeof(*res));
    res->status = job->status;
    res->nx = job->p.nx; res->ny = job->p.ny; res->nz = job->p.nz;
    res->phi = job->phi; res->P = job->P; res->u = job->u;
    job->phi = job->P = job->u = nullptr;
    res->diag = job->diag;
    res->t_submit_s = job->t_submit;
    res->t_admit_s = job->t_admit;
    res->t_finish_s = job->t_finish;
    res->steps = job->status == LBM_OK ? job->nsteps : job->step;
    return LBM_OK;
}

extern "C" int lbm_server_drain(lbm_server* s) {
    if (!s) { set_error("NULL argument"); return LBM_E_INVAL; }
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
    if (s->fatal != LBM_OK) { set_error("server stopped: %s", s->fatal_msg.c_str()); return s->fatal; }
    return LBM_OK;
}

extern "C" double lbm_server_clock(const lbm_server* s) { return s ? s->now() : 0.0; }

extern "C" void lbm_result_free(lbm_result* res) {
    if (!res) return;
    free(res->phi); free(res->P); free(res->u);
    res->phi = res->P = res->u = nullptr;
}

extern "C" int lbm_server_destroy(lbm_server* s) {
    if (!s) return LBM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    hipSetDevice(s->cfg.device);
    if (s->stream) hipStreamSynchronize(s->stream);
    if (s->gexec) hipGraphExecDestroy(s->gexec);
    if (s->dtiles) hipFree(s->dtiles);
    if (s->dghosts) hipFree(s->dghosts);
    if (s->dwalls) hipFree(s->dwalls);
    if (s->dslots) hipFree(s->dslots);
    if (s->dstage) hipFree(s->dstage);
    if (s->up_stream) { hipStreamSynchronize(s->up_stream); hipStreamDestroy(s->up_stream); }
    if (s->cap_stream) hipStreamDestroy(s->cap_stream);
    if (s->ev) hipEventDestroy(s->ev);
    if (s->hmirror) hipHostFree(s->hmirror);
    if (s->dtable) hipFree(s->dtable);
    if (s->arena) hipFree(s->arena);
    if (s->stream) hipStreamDestroy(s->stream);
    delete s;
    return LBM_OK;
}
