// server.cpp -- continuous-batching reconstruction server.
//
// Requests (geometry descriptor, parameters, device f/y/r, iterations) are
// queued by pet_os_submit.  Each class of request (2D, 3D) has a lane: its
// own batch, stream and worker thread.  A lane admits the queued requests of
// its class in arrival order as soon as a slot and the device-memory budget
// allow; admitted requests join the lane's running batch between two steps,
// and every step advances all of them by one subiteration (one replay of the
// captured batched launch sequence).  A request that finishes leaves at once
// and frees its memory, so later arrivals are admitted while others still
// run.  The lanes run concurrently on the device, so a slow 3D subiteration
// does not pace the 2D requests.  Geometries (tables, sensitivity,
// autotuned shapes) are cached by descriptor and count against the shared
// budget; unused ones are evicted first.
//
// The device work sits behind a small executor interface.  Besides the HIP
// executor there is a host-only simulation (no device calls) so that the
// scheduling, budget and failure handling can be exercised without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace petos;

extern "C" {
int pet_os_batch_create(int32_t max_slots, pet_os_batch** out);
int pet_os_batch_destroy(pet_os_batch* batch);
int pet_os_batch_add(pet_os_batch* batch, const pet_os_geom* geom, const pet_os_params* params, float* f,
                     const float* y, const float* r, int32_t n_iter, pet_os_stream stream, int32_t* slot);
int pet_os_batch_remove(pet_os_batch* batch, int32_t slot, pet_os_stream stream);
int pet_os_batch_step(pet_os_batch* batch, int32_t n_steps, pet_os_stream stream);
int pet_os_autotune(pet_os_geom* geom, int32_t flags, pet_os_stream stream);
}

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t ticket = 0;
    pet_os_request rq{};
    pet_os_result res{};
    bool done = false;
    bool cancelled = false;
    int slot = -1;
    int64_t remaining = 0;        // subiterations left
    std::string geo_key;
    size_t bytes = 0;             // scratch + schedule charged to the budget
};

std::string desc_key(const pet_os_geom_desc& d) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%d %d %d %d %.17g %.17g %.17g %d %d %.17g %d %d %.17g %.17g %d", d.dim, d.nx, d.ny,
                  d.nz, d.vx, d.vy, d.vz, d.n_angles, d.n_radial, d.ds, d.n_rings, d.max_ring_diff, d.ring_pitch,
                  d.det_radius, d.n_subsets);
    return buf;
}

// bytes of one request's scratch (mirrors work_alloc) and schedule
size_t request_bytes(const pet_os_geom_desc& d, int n_planes, int max_sub, int n_iter, bool nu) {
    const size_t nv = (size_t)d.nx * d.ny * (d.dim == 3 ? d.nz : 1);
    const size_t nb = (size_t)n_planes * d.n_angles * d.n_radial;
    size_t b = (size_t)max_sub * n_planes * d.n_radial * 4 + nv * 4 * (nu ? 4 : 3);
    b += 8 * (2 * nv / 256 + nv / 64 + (size_t)d.n_angles * n_planes * d.n_radial / 16 + 2 * nb / 256 + 64);
    b += (size_t)n_iter * d.n_subsets * 8;
    return b + 4096;
}

size_t geometry_bytes(const pet_os_geom_desc& d, int n_planes) {
    const size_t nv = (size_t)d.nx * d.ny * (d.dim == 3 ? d.nz : 1);
    return nv * 8 + (size_t)d.n_angles * 160 + (size_t)d.n_radial * (48 + 8 * 63) + (size_t)n_planes * 8 + 65536;
}

int n_planes_desc(const pet_os_geom_desc& d) {
    if (d.dim == 2) return 1;
    int n = d.n_rings;
    for (int k = 1; k <= d.max_ring_diff; ++k) n += 2 * (d.n_rings - k);
    return n;
}

// ------------------------------------------------------------------ executors
struct Executor {
    virtual ~Executor() {}
    // geometry for a descriptor (created on first use); *bytes = device bytes held
    virtual int geometry(const pet_os_geom_desc& d, void** g, size_t* bytes) = 0;
    virtual void drop_geometry(void* g) = 0;
    virtual int add(void* g, const pet_os_request& rq, int* slot) = 0;
    virtual int step() = 0;                       // one batched subiteration (asynchronous)
    virtual int sync() = 0;                       // wait for queued steps
    virtual int objective(void* g, const pet_os_request& rq, double* phi) = 0;
    virtual int remove(int slot) = 0;
    virtual int reset() = 0;                      // drop every slot after a device failure
};

struct HipExecutor : Executor {
    pet_os_batch* batch = nullptr;
    hipStream_t stream = nullptr;
    int max_slots;
    explicit HipExecutor(int ms) : max_slots(ms) {}
    ~HipExecutor() override {
        if (batch) pet_os_batch_destroy(batch);
        if (stream) (void)hipStreamDestroy(stream);
    }
    int init() {
        PETOS_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        return pet_os_batch_create(max_slots, &batch);
    }
    int geometry(const pet_os_geom_desc& d, void** g, size_t* bytes) override {
        pet_os_geom* G = nullptr;
        int rc = pet_os_create_geometry(&d, &G);
        if (rc) return rc;
        // the served lanes run the batched kernels, whose 2D shapes the
        // autotuner picks (the 3D batched shape is fixed)
        if (d.dim == 2) rc = pet_os_autotune(G, 0, stream);
        if (rc) { pet_os_destroy_geometry(G); return rc; }
        *g = G;
        *bytes = geometry_bytes(d, G->n_planes);
        return PET_OS_OK;
    }
    void drop_geometry(void* g) override { pet_os_destroy_geometry((pet_os_geom*)g); }
    int add(void* g, const pet_os_request& rq, int* slot) override {
        return pet_os_batch_add(batch, (const pet_os_geom*)g, &rq.params, rq.f, rq.y, rq.r, rq.n_iter, stream, slot);
    }
    int step() override { return pet_os_batch_step(batch, 1, stream); }
    int sync() override {
        PETOS_HIP(hipStreamSynchronize(stream));
        return PET_OS_OK;
    }
    int objective(void* g, const pet_os_request& rq, double* phi) override {
        return pet_os_objective((const pet_os_geom*)g, &rq.params, rq.f, rq.y, rq.r, phi, stream);
    }
    int remove(int slot) override { return pet_os_batch_remove(batch, slot, stream); }
    int reset() override {
        (void)hipDeviceSynchronize();
        if (batch) pet_os_batch_destroy(batch);
        batch = nullptr;
        return pet_os_batch_create(max_slots, &batch);
    }
};

// Host-only stand-in: no device calls; a step takes `step_us` of wall time.
// Fault injection for tests of the failure paths.
struct SimExecutor : Executor {
    int max_slots;
    std::vector<int> used;
    int64_t step_us = 50;
    int fail_add = 0, fail_step = 0, nan_objective = 0, bad_data = 0;
    explicit SimExecutor(int ms) : max_slots(ms), used(ms, 0) {}
    int geometry(const pet_os_geom_desc& d, void** g, size_t* bytes) override {
        *g = new pet_os_geom_desc(d);
        *bytes = geometry_bytes(d, n_planes_desc(d));
        return PET_OS_OK;
    }
    void drop_geometry(void* g) override { delete (pet_os_geom_desc*)g; }
    int add(void*, const pet_os_request&, int* slot) override {
        if (fail_add > 0) { --fail_add; return fail(PET_OS_ERR_OUT_OF_MEMORY, "injected: out of memory on admission"); }
        if (bad_data > 0) { --bad_data; return fail(PET_OS_ERR_INVALID_ARG, "injected: r: 1 entries not > 0 or not finite"); }
        for (int s = 0; s < max_slots; ++s)
            if (!used[s]) { used[s] = 1; *slot = s; return PET_OS_OK; }
        return fail(PET_OS_ERR_BUDGET, "no free slot");
    }
    int step() override {
        if (fail_step > 0) { --fail_step; return fail(PET_OS_ERR_DEVICE, "injected: launch failure"); }
        std::this_thread::sleep_for(std::chrono::microseconds(step_us));
        return PET_OS_OK;
    }
    int sync() override { return PET_OS_OK; }
    int objective(void*, const pet_os_request&, double* phi) override {
        if (nan_objective > 0) { --nan_objective; *phi = std::numeric_limits<double>::quiet_NaN(); return PET_OS_OK; }
        *phi = -1.0;
        return PET_OS_OK;
    }
    int remove(int slot) override {
        if (slot >= 0 && slot < max_slots) used[slot] = 0;
        return PET_OS_OK;
    }
    int reset() override {
        std::fill(used.begin(), used.end(), 0);
        return PET_OS_OK;
    }
};

struct GeoEntry {
    void* g = nullptr;
    size_t bytes = 0;
    int refs = 0;
    uint64_t last_use = 0;
};

}  // namespace

namespace {
constexpr int N_LANES = 2;                    // lane 0: 2D requests, lane 1: 3D
int lane_of(const pet_os_geom_desc& d) { return d.dim == 3 ? 1 : 0; }

struct Lane {
    std::unique_ptr<Executor> ex;
    std::vector<std::shared_ptr<Req>> active;
    std::thread worker;
};
}  // namespace

struct pet_os_server {
    size_t budget = 0;
    int max_slots = 0;
    int device = 0;
    bool simulate = false;
    Lane lanes[N_LANES];
    SimExecutor* sim = nullptr;                           // lane 0's, when simulated
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Req>> queue;               // submitted, not admitted
    std::map<uint64_t, std::shared_ptr<Req>> all;         // every unclaimed request
    std::map<std::string, GeoEntry> geos;
    size_t used_bytes = 0;
    uint64_t next_ticket = 1;
    uint64_t use_clock = 0;
    uint64_t gen = 0;              // bumped on every submit, cancel and departure
    int admitting = 0;             // admissions in progress (slots reserved)
    // Device API calls of the lanes (geometry creation, joining, the step that
    // may capture a graph, objective, leaving) are serialized: a graph capture
    // in one lane must not overlap default-stream work issued by the other
    // (the runtime then invalidates the capture).  Waiting on a lane's own
    // stream is not serialized.  Taken after mu when both are held.
    std::mutex api_mu;
    bool stop = false;
    Clock::time_point t0 = Clock::now();
    // statistics
    int64_t ticks = 0, max_active = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    int64_t n_active() const {
        int64_t n = 0;
        for (const auto& L : lanes) n += (int64_t)L.active.size();
        return n;
    }
    bool queued_for(int lane) const {
        for (const auto& r : queue)
            if (lane_of(r->rq.desc) == lane) return true;
        return false;
    }
    void run(int lane);
    void finish(const std::shared_ptr<Req>& r, int status, const std::string& msg);
    bool try_admit(int lane, std::unique_lock<std::mutex>& lk);
    void evict_unused(size_t need);
};

void pet_os_server::finish(const std::shared_ptr<Req>& r, int status, const std::string& msg) {
    r->res.status = status;
    r->res.t_finish = now();
    if (status != PET_OS_OK) std::snprintf(r->res.message, sizeof(r->res.message), "%s", msg.c_str());
    r->done = true;
}

void pet_os_server::evict_unused(size_t need) {
    while (used_bytes + need > budget) {
        auto victim = geos.end();
        for (auto it = geos.begin(); it != geos.end(); ++it)
            if (it->second.refs == 0 && (victim == geos.end() || it->second.last_use < victim->second.last_use))
                victim = it;
        if (victim == geos.end()) return;
        {
            std::lock_guard<std::mutex> api(api_mu);
            lanes[0].ex->drop_geometry(victim->second.g);     // any lane's executor releases geometries
        }
        used_bytes -= victim->second.bytes;
        geos.erase(victim);
    }
}

// Admit the request at the head of the queue if a slot and the budget allow.
// Called with the lock held; drops it around device work.
bool pet_os_server::try_admit(int lane, std::unique_lock<std::mutex>& lk) {
    if (n_active() + admitting >= max_slots) return false;
    // the oldest queued request of this lane's class
    auto qit = std::find_if(queue.begin(), queue.end(), [&](const std::shared_ptr<Req>& q) {
        return lane_of(q->rq.desc) == lane;
    });
    if (qit == queue.end()) return false;
    std::shared_ptr<Req> r = *qit;
    Executor* ex = lanes[lane].ex.get();
    auto& active = lanes[lane].active;
    if (r->cancelled) {
        queue.erase(qit);
        finish(r, PET_OS_ERR_TIMEOUT, "cancelled before admission");
        cv_done.notify_all();
        return true;
    }
    const pet_os_geom_desc& d = r->rq.desc;
    const int np = n_planes_desc(d);
    const int max_sub = (d.n_angles + d.n_subsets - 1) / d.n_subsets;
    const bool nu = r->rq.params.mode == PET_OS_P1 || r->rq.params.mode == PET_OS_P2;
    r->bytes = request_bytes(d, np, max_sub, r->rq.n_iter, nu);
    auto git = geos.find(r->geo_key);
    const size_t gbytes = git == geos.end() ? geometry_bytes(d, np) : 0;
    if (r->bytes + gbytes > budget) {
        queue.erase(qit);
        finish(r, PET_OS_ERR_BUDGET, "request needs more device memory than the whole budget");
        cv_done.notify_all();
        return true;
    }
    if (used_bytes + r->bytes + gbytes > budget) evict_unused(r->bytes + gbytes);
    if (used_bytes + r->bytes + gbytes > budget) return false;      // wait for running requests to leave
    queue.erase(qit);
    r->res.t_admit = now();
    // reserve the slot, the memory and a cached geometry before the lock is
    // dropped: the other lane admits and evicts meanwhile
    ++admitting;
    used_bytes += r->bytes + gbytes;
    if (git != geos.end()) git->second.refs++;
    const bool new_geo = git == geos.end();
    // device work without the lock
    lk.unlock();
    int rc = PET_OS_OK;
    void* g = nullptr;
    size_t gb = 0;
    if (new_geo) {
        std::lock_guard<std::mutex> api(api_mu);
        rc = ex->geometry(d, &g, &gb);
    }
    int slot = -1;
    lk.lock();
    used_bytes -= gbytes;                  // the estimate; the real geometry bytes follow
    GeoEntry* ge = nullptr;
    if (!rc) {
        if (new_geo) {
            GeoEntry e;
            e.g = g;
            e.bytes = gb;
            e.refs = 1;
            auto ins = geos.emplace(r->geo_key, e);
            if (ins.second) {
                used_bytes += gb;
            } else {                       // made meanwhile by another admission: keep that one
                std::lock_guard<std::mutex> api(api_mu);
                ex->drop_geometry(g);
                ins.first->second.refs++;
            }
            ge = &ins.first->second;
        } else {
            ge = &geos[r->geo_key];
        }
        ge->last_use = ++use_clock;
    } else if (!new_geo) {
        geos[r->geo_key].refs--;
    }
    lk.unlock();
    if (!rc) {
        std::lock_guard<std::mutex> api(api_mu);
        rc = ex->add(ge->g, r->rq, &slot);
    }
    lk.lock();
    --admitting;
    if (rc) {
        if (ge) ge->refs--;
        used_bytes -= r->bytes;
        finish(r, rc, pet_os_last_error());
        cv_done.notify_all();
        return true;
    }
    r->slot = slot;
    r->remaining = (int64_t)r->rq.n_iter * d.n_subsets;
    r->res.t_start = now();
    active.push_back(r);
    max_active = std::max<int64_t>(max_active, n_active());
    return true;
}

void pet_os_server::run(int lane) {
    if (!simulate) (void)hipSetDevice(device);
    Executor* ex = lanes[lane].ex.get();
    auto& active = lanes[lane].active;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        while (try_admit(lane, lk)) {
        }
        if (active.empty()) {
            if (stop && !queued_for(lane)) break;
            // idle until something changes: an arrival, a cancellation, or a
            // departure in the other lane freeing a slot or memory
            const uint64_t seen = gen;
            cv_work.wait(lk, [&] { return stop || gen != seen; });
            continue;
        }
        lk.unlock();
        int rc;
        {
            std::lock_guard<std::mutex> api(api_mu);
            rc = ex->step();
        }
        lk.lock();
        ++ticks;
        if (rc) {
            // device failure: every running request fails, the batch is rebuilt
            std::string msg = pet_os_last_error();
            lk.unlock();
            {
                std::lock_guard<std::mutex> api(api_mu);
                (void)ex->reset();
            }
            lk.lock();
            for (auto& r : active) {
                used_bytes -= r->bytes;
                geos[r->geo_key].refs--;
                finish(r, rc, msg);
            }
            active.clear();
            ++gen;
            cv_done.notify_all();
            cv_work.notify_all();
            continue;
        }
        std::vector<std::shared_ptr<Req>> leaving;
        for (auto& r : active)
            if (--r->remaining <= 0 || r->cancelled) leaving.push_back(r);
        if (leaving.empty()) continue;
        lk.unlock();
        (void)ex->sync();
        std::vector<int> status(leaving.size(), PET_OS_OK);
        std::vector<std::string> msgs(leaving.size());
        for (size_t k = 0; k < leaving.size(); ++k) {
            auto& r = leaving[k];
            r->res.subiterations = (int64_t)r->rq.n_iter * r->rq.desc.n_subsets - std::max<int64_t>(0, r->remaining);
            r->res.objective = std::numeric_limits<double>::quiet_NaN();
            if (r->cancelled && r->remaining > 0) {
                status[k] = PET_OS_ERR_TIMEOUT;
                msgs[k] = "cancelled while running";
            } else if (r->rq.want_objective) {
                void* g = nullptr;
                {
                    std::lock_guard<std::mutex> gl(mu);
                    g = geos[r->geo_key].g;
                }
                double phi = 0;
                int orc;
                {
                    std::lock_guard<std::mutex> api(api_mu);
                    orc = ex->objective(g, r->rq, &phi);
                }
                if (orc) { status[k] = orc; msgs[k] = pet_os_last_error(); }
                else if (!std::isfinite(phi)) { status[k] = PET_OS_ERR_NUMERIC; msgs[k] = "objective is not finite"; }
                r->res.objective = phi;
            }
            {
                std::lock_guard<std::mutex> api(api_mu);
                (void)ex->remove(r->slot);
            }
        }
        lk.lock();
        for (size_t k = 0; k < leaving.size(); ++k) {
            auto& r = leaving[k];
            active.erase(std::find(active.begin(), active.end(), r));
            used_bytes -= r->bytes;
            geos[r->geo_key].refs--;
            finish(r, status[k], msgs[k]);
        }
        ++gen;
        cv_done.notify_all();
        cv_work.notify_all();     // slots and memory are free for the other lane too
    }
}

namespace {

int server_create(size_t budget, int32_t max_slots, bool simulate, int64_t step_us, pet_os_server** out) {
    if (!out) return fail(PET_OS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (budget == 0) return fail(PET_OS_ERR_INVALID_ARG, "hbm_budget_bytes must be > 0");
    if (max_slots < 1 || max_slots > 65536) return fail(PET_OS_ERR_INVALID_ARG, "max_slots must be in [1, 65536]");
    auto* S = new pet_os_server();
    S->budget = budget;
    S->max_slots = max_slots;
    S->simulate = simulate;
    if (!simulate && hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return fail(PET_OS_ERR_DEVICE, "no HIP device");
    }
    for (int l = 0; l < N_LANES; ++l) {
        if (simulate) {
            auto* sim = new SimExecutor(max_slots);
            sim->step_us = std::max<int64_t>(0, step_us);
            if (l == 0) S->sim = sim;
            S->lanes[l].ex.reset(sim);
        } else {
            auto* hx = new HipExecutor(max_slots);
            S->lanes[l].ex.reset(hx);
            int rc = hx->init();
            if (rc) { delete S; return rc; }
        }
    }
    for (int l = 0; l < N_LANES; ++l) S->lanes[l].worker = std::thread([S, l] { S->run(l); });
    *out = S;
    return PET_OS_OK;
}

}  // namespace

extern "C" {

int pet_os_server_create(size_t hbm_budget_bytes, int32_t max_slots, pet_os_server** out) {
    return server_create(hbm_budget_bytes, max_slots, false, 0, out);
}

int pet_os_server_create_simulated(size_t budget_bytes, int32_t max_slots, int64_t step_us, pet_os_server** out) {
    return server_create(budget_bytes, max_slots, true, step_us, out);
}

int pet_os_server_inject(pet_os_server* S, int32_t kind, int32_t count) {
    if (!S || !S->sim) return fail(PET_OS_ERR_INVALID_ARG, "fault injection needs a simulated server");
    std::lock_guard<std::mutex> lk(S->mu);
    switch (kind) {
        case PET_OS_INJECT_ADMIT_OOM: S->sim->fail_add += count; break;
        case PET_OS_INJECT_STEP_FAILURE: S->sim->fail_step += count; break;
        case PET_OS_INJECT_NAN_OBJECTIVE: S->sim->nan_objective += count; break;
        case PET_OS_INJECT_BAD_DATA: S->sim->bad_data += count; break;
        default: return fail(PET_OS_ERR_INVALID_ARG, "unknown fault kind");
    }
    return PET_OS_OK;
}

int pet_os_server_destroy(pet_os_server* S) {
    if (!S) return fail(PET_OS_ERR_INVALID_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& L : S->lanes)
        if (L.worker.joinable()) L.worker.join();
    for (auto& kv : S->geos) S->lanes[0].ex->drop_geometry(kv.second.g);
    S->geos.clear();
    delete S;
    return PET_OS_OK;
}

int pet_os_submit(pet_os_server* S, const pet_os_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    pet_os_geom_desc d = req->desc;
    if (d.dim == 2) { d.nz = 1; d.vz = 1.0; d.n_rings = 1; d.max_ring_diff = 0; d.ring_pitch = 1.0; }
    // synchronous validation: descriptor, parameters, pointers, iterations
    int rc = validate_desc(&d);
    if (rc) return rc;
    rc = validate_params(&req->params, nullptr);
    if (rc) return rc;
    if (req->params.mode == PET_OS_OSEM) return fail(PET_OS_ERR_INVALID_ARG, "OSEM runs on states only, not served");
    if (d.n_subrays > 1 || d.psf_fwhm > 0.0)
        return fail(PET_OS_ERR_INVALID_ARG, "sub-rays and the PSF run on states only, not served");
    if (!S->simulate && (!req->f || !req->y || !req->r)) return fail(PET_OS_ERR_INVALID_ARG, "NULL data pointer");
    if (req->n_iter < 1) return fail(PET_OS_ERR_INVALID_ARG, "n_iter must be >= 1");
    auto r = std::make_shared<Req>();
    r->rq = *req;
    r->rq.desc = d;
    r->geo_key = desc_key(d);
    r->res.status = 1;   // pending
    r->res.objective = std::numeric_limits<double>::quiet_NaN();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return fail(PET_OS_ERR_INVALID_ARG, "server is shutting down");
        r->ticket = S->next_ticket++;
        r->res.t_submit = S->now();
        S->queue.push_back(r);
        S->all[r->ticket] = r;
        *ticket = r->ticket;
        ++S->gen;
    }
    S->cv_work.notify_all();
    return PET_OS_OK;
}

int pet_os_cancel(pet_os_server* S, uint64_t ticket) {
    if (!S) return fail(PET_OS_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(PET_OS_ERR_INVALID_ARG, "unknown ticket");
    it->second->cancelled = true;
    ++S->gen;
    S->cv_work.notify_all();
    return PET_OS_OK;
}

int pet_os_wait(pet_os_server* S, uint64_t ticket, int64_t timeout_us, pet_os_result* out) {
    if (!S || !out) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(PET_OS_ERR_INVALID_ARG, "unknown ticket");
    std::shared_ptr<Req> r = it->second;
    auto pred = [&] { return r->done; };
    if (timeout_us < 0) S->cv_done.wait(lk, pred);
    else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
        return fail(PET_OS_ERR_TIMEOUT, "request not finished yet");
    *out = r->res;
    S->all.erase(ticket);
    return PET_OS_OK;
}

int pet_os_server_stats(pet_os_server* S, pet_os_server_stats_t* out) {
    if (!S || !out) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    out->queued = (int64_t)S->queue.size();
    out->active = S->n_active();
    out->ticks = S->ticks;
    out->max_active = S->max_active;
    out->bytes_in_use = S->used_bytes;
    out->geometries_cached = (int64_t)S->geos.size();
    return PET_OS_OK;
}

}  // extern "C"
