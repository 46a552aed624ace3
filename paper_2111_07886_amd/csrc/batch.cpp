// batch.cpp -- many independent reconstructions of uneven sizes advanced
// together: one batched subiteration (forward + ratio, back-projection +
// stencil, update, advance) for every active request per launch sequence,
// captured once in a hipGraph and replayed.
//
// Each request keeps its iterate, scratch, FP64-derived schedule (lambda_k
// alpha_{k,i} and the nu mode of eq:nuki for every subiteration, evaluated on
// the host at admission) and its subiteration counter on the device.  The
// batched kernels run the same per-block code as the plain path, over a
// device-resident work list of (request, block) items, so a request computes
// exactly what it computes alone.
//
// Also here: the autotuner that picks the forward projector's threads per
// ray and the back-projector's tile for a geometry by timing the candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

using namespace petos;

namespace petos {

struct BatchSlot {
    bool used = false;
    const pet_os_geom* g = nullptr;
    pet_os_params p{};
    float* f = nullptr;
    const float* y = nullptr;
    const float* r = nullptr;
    int64_t J_next = 1, J_end = 0;   // host mirror of the device counter
    Work w;
    float* d_step = nullptr;
    int* d_nu = nullptr;
    int fp_seg = 1, bp_kind = 0;
    size_t bytes = 0;
};

}  // namespace petos

struct pet_os_batch {
    int max_slots = 0;
    std::vector<BatchSlot> slots;
    std::vector<SlotDev> h_slots;
    SlotDev* d_slots = nullptr;
    Item* d_items[WL_COUNT] = {};
    int cap[WL_COUNT] = {};
    int count[WL_COUNT] = {};
    int* d_counts = nullptr;
    int grids[WL_COUNT] = {};
    int live_mask = 0;               // lists launched by the captured graph
    bool lists_dirty = true;
    bool graph_ok = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    size_t bytes = 0;
};

namespace {

constexpr int GRID_CAP = 8192;

void slot_release(BatchSlot& s) {
    work_free(&s.w);
    if (s.d_step) (void)hipFree(s.d_step);
    if (s.d_nu) (void)hipFree(s.d_nu);
    s = BatchSlot{};
}

int upload_slot(pet_os_batch* B, int idx) {
    PETOS_HIP(hipMemcpy(B->d_slots + idx, &B->h_slots[idx], sizeof(SlotDev), hipMemcpyHostToDevice));
    return PET_OS_OK;
}

// one field of a slot's device record (the device advances the slot's
// subiteration counter, so the record is not uploaded whole after admission)
template <typename T>
int upload_slot_field(pet_os_batch* B, int idx, size_t offset, const T& v) {
    PETOS_HIP(hipMemcpy(reinterpret_cast<char*>(B->d_slots + idx) + offset, &v, sizeof(T), hipMemcpyHostToDevice));
    return PET_OS_OK;
}

int rebuild_lists(pet_os_batch* B) {
    // The forward projector's threads per ray: a ray's sum does not depend
    // on it (fp_body), so the batch takes the shape its total number of 2D
    // rays calls for, not each request's single-request shape: about 2^22
    // threads in all.  Fewer threads per ray repeat less set-up, more keep
    // more loads in flight; measured on 96 uneven requests (~3.2e5 rays),
    // 1 / 4 / 16 / 64 threads per ray gave 607 / 765 / 800 / 754 recons/s.
    long long rays2d = 0;
    bool any2d = false;
    for (const BatchSlot& S : B->slots)
        if (S.used && S.g->d.dim == 2) {
            rays2d += (long long)S.g->max_sub_angles * S.g->n_planes * S.g->d.n_radial;
            any2d = true;
        }
    if (any2d) {
        const int seg = rays2d >= (1LL << 22) ? 1 : rays2d >= (1LL << 20) ? 4 : rays2d >= (1LL << 18) ? 16 : 64;
        for (int s = 0; s < B->max_slots; ++s) {
            BatchSlot& S = B->slots[s];
            if (!S.used || S.g->d.dim != 2 || S.fp_seg == seg) continue;
            S.fp_seg = seg;
            SlotDev& D = B->h_slots[s];
            D.fp_seg = seg;
            D.n_fp = fp_grid_seg(S.g, S.g->max_sub_angles, seg);
            int rc = upload_slot_field(B, s, offsetof(SlotDev, fp_seg), D.fp_seg);
            if (!rc) rc = upload_slot_field(B, s, offsetof(SlotDev, n_fp), D.n_fp);
            if (rc) return rc;
        }
    }
    std::vector<Item> L[WL_COUNT];
    for (int s = 0; s < B->max_slots; ++s) {
        const BatchSlot& S = B->slots[s];
        if (!S.used) continue;
        const bool d3 = S.g->d.dim == 3;
        // 2D: forward blocks, then the pixel-pass blocks (snapshot, mu)
        const int nfp = d3 ? fp3_grid(S.g, S.g->max_sub_angles)
                           : fp_grid_seg(S.g, S.g->max_sub_angles, S.fp_seg) + px_items(S.g);
        for (int b = 0; b < nfp; ++b) L[d3 ? WL_FP3 : WL_FP].push_back({s, b});
        const int nbp = d3 ? bp3_grid_batch(S.g) : bp_grid_kind(S.g, S.bp_kind);
        const int zi = d3 ? (bp3_zb(S.g) == 16 ? 0 : (bp3_zb(S.g) == 32 ? 1 : 2)) : 0;
        const int wbp = d3 ? WL_BP3 + 2 * zi + (bp3_nbs_of(S.g) == 40 ? 1 : 0) : WL_BP0 + S.bp_kind;
        for (int b = 0; b < nbp; ++b) L[wbp].push_back({s, b});
        if (d3) {
            const int npen = pen3_grid(S.g);
            for (int b = 0; b < npen; ++b) L[WL_PEN3].push_back({s, b});
            const int nup = upd3_grid(S.g);
            for (int b = 0; b < nup; ++b) L[WL_UPD3].push_back({s, b});
        }
    }
    int mask = 0;
    for (int k = 0; k < WL_COUNT; ++k) {
        const int n = (int)L[k].size();
        if (n > B->cap[k]) {
            if (B->d_items[k]) (void)hipFree(B->d_items[k]);
            B->d_items[k] = nullptr;
            int c = std::max(n, 2 * B->cap[k]);
            if (hipMalloc(&B->d_items[k], (size_t)std::max(c, 1) * sizeof(Item)) != hipSuccess)
                return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc of work list failed");
            B->cap[k] = c;
            B->graph_ok = false;       // captured kernel arguments point at the old list
        }
        if (n) PETOS_HIP(hipMemcpy(B->d_items[k], L[k].data(), (size_t)n * sizeof(Item), hipMemcpyHostToDevice));
        B->count[k] = n;
        if (n) mask |= 1 << k;
    }
    // the graph launches only the non-empty lists: capture again when that set changes
    if (mask != B->live_mask) {
        B->live_mask = mask;
        B->graph_ok = false;
    }
    PETOS_HIP(hipMemcpy(B->d_counts, B->count, sizeof(B->count), hipMemcpyHostToDevice));
    B->lists_dirty = false;
    return PET_OS_OK;
}

int capture(pet_os_batch* B) {
    if (B->exec) { (void)hipGraphExecDestroy(B->exec); B->exec = nullptr; }
    if (B->graph) { (void)hipGraphDestroy(B->graph); B->graph = nullptr; }
    // multiples of 8: the kernels deal contiguous item runs to each XCD
    for (int k = 0; k < WL_COUNT; ++k) B->grids[k] = 8 * ((std::max(1, std::min(B->cap[k], GRID_CAP)) + 7) / 8);
    PETOS_HIP(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = launch_batch_step(B->d_slots, B->max_slots, B->d_items, B->d_counts, B->grids, B->live_mask,
                               B->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(PET_OS_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    B->graph = g;
    PETOS_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->graph_ok = true;
    return PET_OS_OK;
}

}  // namespace

extern "C" {

int pet_os_batch_create(int32_t max_slots, pet_os_batch** out) {
    if (!out) return fail(PET_OS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 65536) return fail(PET_OS_ERR_INVALID_ARG, "max_slots must be in [1, 65536]");
    auto* B = new pet_os_batch();
    B->max_slots = max_slots;
    B->slots.resize(max_slots);
    B->h_slots.assign(max_slots, SlotDev{});
    if (hipMalloc(&B->d_slots, sizeof(SlotDev) * (size_t)max_slots) != hipSuccess ||
        hipMalloc(&B->d_counts, sizeof(int) * WL_COUNT) != hipSuccess) {
        if (B->d_slots) (void)hipFree(B->d_slots);
        delete B;
        return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc of the slot table failed");
    }
    if (hipMemcpy(B->d_slots, B->h_slots.data(), sizeof(SlotDev) * (size_t)max_slots, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(B->d_counts, 0, sizeof(int) * WL_COUNT) != hipSuccess ||
        hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(B->d_slots);
        (void)hipFree(B->d_counts);
        delete B;
        return fail(PET_OS_ERR_DEVICE, "batch initialisation failed");
    }
    *out = B;
    return PET_OS_OK;
}

int pet_os_batch_destroy(pet_os_batch* B) {
    if (!B) return fail(PET_OS_ERR_INVALID_ARG, "batch is NULL");
    (void)hipDeviceSynchronize();
    for (auto& s : B->slots)
        if (s.used) slot_release(s);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (int k = 0; k < WL_COUNT; ++k)
        if (B->d_items[k]) (void)hipFree(B->d_items[k]);
    (void)hipFree(B->d_slots);
    (void)hipFree(B->d_counts);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    delete B;
    return PET_OS_OK;
}

int pet_os_batch_add(pet_os_batch* B, const pet_os_geom* g, const pet_os_params* p, float* f, const float* y,
                     const float* r, int32_t n_iter, pet_os_stream stream, int32_t* slot_out) {
    if (!B || !g || !p || !f || !y || !r) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    if (n_iter < 1) return fail(PET_OS_ERR_INVALID_ARG, "n_iter must be >= 1");
    GeomExtra* ex = extra_of(g);
    if (!ex) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    int rc = validate_params(p, g);
    if (rc) return rc;
    if (p->mode == PET_OS_OSEM) return fail(PET_OS_ERR_INVALID_ARG, "OSEM runs on states only, not in a batch");
    if (g->full_model)
        return fail(PET_OS_ERR_INVALID_ARG, "sub-rays, PSF and attenuation run on states only, not in a batch");
    int idx = -1;
    for (int s = 0; s < B->max_slots; ++s)
        if (!B->slots[s].used) { idx = s; break; }
    if (idx < 0) return fail(PET_OS_ERR_BUDGET, "no free slot");
    hipStream_t st = (hipStream_t)stream;
    PETOS_HIP(hipStreamSynchronize(st));       // the slot table is read by queued steps

    BatchSlot S;
    S.g = g;
    S.p = *p;
    S.f = f;
    S.y = y;
    S.r = r;
    const int M = g->d.n_subsets;
    S.J_next = 1;
    S.J_end = (int64_t)n_iter * M;
    const bool need_nu = p->mode == PET_OS_P1 || p->mode == PET_OS_P2;
    rc = work_alloc(g, need_nu, &S.w);
    if (rc) return rc;
    if ((rc = check_data(g, p, &S.w, f, y, r, st))) {
        work_free(&S.w);
        return rc;
    }
    std::vector<float> step;
    std::vector<int> nu;
    schedule_table(*p, M, S.J_end, step, nu);
    if (hipMalloc(&S.d_step, step.size() * sizeof(float)) != hipSuccess ||
        hipMalloc(&S.d_nu, nu.size() * sizeof(int)) != hipSuccess) {
        slot_release(S);
        return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc of the schedule failed");
    }
    if (hipMemcpy(S.d_step, step.data(), step.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(S.d_nu, nu.data(), nu.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        slot_release(S);
        return fail(PET_OS_ERR_DEVICE, "schedule upload failed");
    }
    S.bytes = S.w.bytes + step.size() * (sizeof(float) + sizeof(int));
    const long long nrays_sub = (long long)g->max_sub_angles * g->n_planes * g->d.n_radial;
    S.fp_seg = fp_seg_for(g, nrays_sub, g->tuned_seg);
    S.bp_kind = bp_kind_of(g);
    // sum of f0 for mean f of the first adaptive subiteration (3D: and the
    // z-fastest copy of f0 read by the forward projector)
    rc = launch_sum_f(g, f, S.w.fz, S.w.red[RED_SUMF], st);
    if (rc) { slot_release(S); return rc; }

    SlotDev D{};
    D.g = g->k;
    D.pnorm = g->pnorm;
    D.f = f;
    D.y = y;
    D.r = r;
    D.w = S.w.w;
    D.G = S.w.G;
    D.mu = S.w.mu;
    D.nu_frozen = S.w.nu_frozen;
    D.fz = S.w.fz;
    D.fsnap = S.w.fsnap;
    D.n_fp = g->d.dim == 3 ? 0 : fp_grid_seg(g, g->max_sub_angles, S.fp_seg);
    D.part_f = S.w.red[RED_SUMF].part;
    D.part_mu = S.w.red[RED_SUMMU].part;
    D.n_part_f = sumf_grid(g);
    D.n_part_mu = g->d.dim == 3 ? pen3_grid(g) : px_grid(g);
    D.subset_lists = ex->subset_lists;
    D.subset_count = ex->d_subset_count;
    D.max_sub = g->max_sub_angles;
    D.sched_step = S.d_step;
    D.sched_nu = S.d_nu;
    D.J = 1;
    D.J_end = (int)S.J_end;
    D.beta_over_M = (float)(p->beta / (double)M);
    D.gamma_R = (float)p->gamma_R;
    D.eps = (float)p->eps;
    D.nu1 = (float)p->nu1;
    D.nu2 = (float)p->nu2;
    D.box = make_box(p->U, p->t_clip);
    D.fp_seg = S.fp_seg;
    D.bp_kind = S.bp_kind;
    if (g->d.dim == 3) {
        rc = bp3_shape(g, D.nb_max, D.zb, D.rows_max, D.chunk);
        if (rc) { slot_release(S); return rc; }
    } else {
        size_t lds;
        bp_stage_shape_kind(g, S.bp_kind, D.nb_max, D.rows_max, D.chunk, lds);
    }
    D.active = 1;
    S.used = true;
    B->slots[idx] = S;
    B->h_slots[idx] = D;
    PETOS_HIP(hipStreamSynchronize(st));
    rc = upload_slot(B, idx);
    if (rc) return rc;
    B->bytes += S.bytes;
    B->lists_dirty = true;
    if (slot_out) *slot_out = idx;
    return PET_OS_OK;
}

int pet_os_batch_remove(pet_os_batch* B, int32_t slot, pet_os_stream stream) {
    if (!B || slot < 0 || slot >= B->max_slots || !B->slots[slot].used)
        return fail(PET_OS_ERR_INVALID_ARG, "no such slot");
    PETOS_HIP(hipStreamSynchronize((hipStream_t)stream));
    B->bytes -= B->slots[slot].bytes;
    slot_release(B->slots[slot]);
    B->h_slots[slot] = SlotDev{};
    int rc = upload_slot(B, slot);
    if (rc) return rc;
    B->lists_dirty = true;
    return PET_OS_OK;
}

int pet_os_batch_step(pet_os_batch* B, int32_t n_steps, pet_os_stream stream) {
    if (!B || n_steps < 0) return fail(PET_OS_ERR_INVALID_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if (B->lists_dirty) {
        PETOS_HIP(hipStreamSynchronize(st));
        if ((rc = rebuild_lists(B))) return rc;
    }
    if (!B->graph_ok && (rc = capture(B))) return rc;
    for (int n = 0; n < n_steps; ++n) PETOS_HIP(hipGraphLaunch(B->exec, st));
    for (auto& s : B->slots)
        if (s.used) s.J_next = std::min<int64_t>(s.J_end + 1, s.J_next + n_steps);
    return PET_OS_OK;
}

int pet_os_batch_run(pet_os_batch* B, pet_os_stream stream) {
    if (!B) return fail(PET_OS_ERR_INVALID_ARG, "batch is NULL");
    int64_t steps = 0;
    for (auto& s : B->slots)
        if (s.used) steps = std::max<int64_t>(steps, s.J_end - s.J_next + 1);
    if (steps > INT32_MAX) return fail(PET_OS_ERR_INVALID_ARG, "too many steps");
    return pet_os_batch_step(B, (int32_t)steps, stream);
}

int pet_os_batch_slot_status(const pet_os_batch* B, int32_t slot, int32_t* active, int64_t* remaining) {
    if (!B || slot < 0 || slot >= B->max_slots) return fail(PET_OS_ERR_INVALID_ARG, "no such slot");
    const BatchSlot& s = B->slots[slot];
    if (active) *active = s.used && s.J_next <= s.J_end ? 1 : 0;
    if (remaining) *remaining = s.used ? std::max<int64_t>(0, s.J_end - s.J_next + 1) : 0;
    return PET_OS_OK;
}

int pet_os_batch_bytes(const pet_os_batch* B, size_t* bytes) {
    if (!B || !bytes) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    *bytes = B->bytes;
    return PET_OS_OK;
}

int pet_os_reconstruct_batch(int32_t n, const pet_os_geom* const* geoms, const pet_os_params* params,
                             float* const* f, const float* const* y, const float* const* r,
                             const int32_t* n_iter, pet_os_stream stream) {
    if (n < 1 || !geoms || !params || !f || !y || !r || !n_iter) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    for (int k = 0; k < n; ++k) {
        if (!geoms[k] || !extra_of(geoms[k]) || !f[k] || !y[k] || !r[k] || n_iter[k] < 1)
            return fail(PET_OS_ERR_INVALID_ARG, "invalid request " + std::to_string(k));
        int rc = validate_params(&params[k], geoms[k]);
        if (rc) return rc;
    }
    pet_os_batch* B = nullptr;
    int rc = pet_os_batch_create(n, &B);
    for (int k = 0; k < n && !rc; ++k) rc = pet_os_batch_add(B, geoms[k], &params[k], f[k], y[k], r[k], n_iter[k], stream, nullptr);
    if (!rc) rc = pet_os_batch_run(B, stream);
    if (!rc && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = fail(PET_OS_ERR_DEVICE, "synchronize failed");
    if (B) pet_os_batch_destroy(B);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner

namespace {

std::mutex g_tune_mu;

std::string tune_key(const pet_os_geom_desc& d) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%d %d %d %d %.17g %.17g %.17g %d %d %.17g %d %d %.17g %.17g %d", d.dim, d.nx, d.ny,
                  d.nz, d.vx, d.vy, d.vz, d.n_angles, d.n_radial, d.ds, d.n_rings, d.max_ring_diff, d.ring_pitch,
                  d.det_radius, d.n_subsets);
    return buf;
}

bool cache_lookup(const std::string& key, int& seg, int& kind) {
    const char* path = std::getenv("PET_OS_TUNE_CACHE");
    if (!path) return false;
    FILE* fh = std::fopen(path, "r");
    if (!fh) return false;
    char line[768];
    bool found = false;
    while (std::fgets(line, sizeof(line), fh)) {
        std::string L(line);
        size_t bar = L.find('|');
        if (bar == std::string::npos) continue;
        if (L.substr(0, bar) == key && std::sscanf(L.c_str() + bar + 1, "%d %d", &seg, &kind) == 2) found = true;
    }
    std::fclose(fh);
    return found;
}

void cache_store(const std::string& key, int seg, int kind) {
    const char* path = std::getenv("PET_OS_TUNE_CACHE");
    if (!path) return;
    FILE* fh = std::fopen(path, "a");
    if (!fh) return;
    std::fprintf(fh, "%s|%d %d\n", key.c_str(), seg, kind);
    std::fclose(fh);
}

// The tuner's choice among shapes timed in turn, the default first: another
// shape replaces the current pick only when at least 3 % faster, so that
// shapes within timing noise of each other do not flip from run to run.
struct TunePick {
    int value = -1;
    float ms = 0.0f;
    void offer(int v, float t) {
        if (value < 0 || t < 0.97f * ms) {
            value = v;
            ms = t;
        }
    }
};

// the shortest device time in ms of `reps` launches of fn on stream s (the
// minimum is the statistic least moved by interference such as a tracer)
template <class Fn>
int time_launch(hipStream_t s, int reps, Fn fn, float* ms_out) {
    hipEvent_t a, b;
    PETOS_HIP(hipEventCreate(&a));
    PETOS_HIP(hipEventCreate(&b));
    std::vector<float> t;
    int rc = fn();                       // warm-up
    for (int k = 0; k < reps && !rc; ++k) {
        (void)hipEventRecord(a, s);
        rc = fn();
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    *ms_out = *std::min_element(t.begin(), t.end());
    return PET_OS_OK;
}

}  // namespace

extern "C" int pet_os_geometry_shapes(const pet_os_geom* g, int32_t* current, int32_t* defaults) {
    if (!g) return fail(PET_OS_ERR_INVALID_ARG, "geom is NULL");
    const bool d3 = g->d.dim == 3;
    const long long nrays = (long long)g->max_sub_angles * g->n_planes * g->d.n_radial;
    int32_t cur[4] = {0, 0, 0, 0}, def[4] = {0, 0, 0, 0};
    if (d3) {
        int nb, rw, dpg, half, lds;
        def[1] = cur[1] = 2;
        def[2] = bp3_zb(g);
        if (bp3_shape_single(g, def[2], 0, nb, rw, dpg, half, lds) == PET_OS_OK) def[3] = dpg;
        cur[2] = g->tuned_zb > 0 ? g->tuned_zb : def[2];
        if (bp3_shape_single(g, cur[2], g->tuned_dpg, nb, rw, dpg, half, lds) == PET_OS_OK) cur[3] = dpg;
    } else {
        def[0] = fp_seg_for(g, nrays, 0);
        cur[0] = fp_seg_for(g, nrays, g->tuned_seg);
        cur[1] = bp_kind_of(g);
        def[1] = bp_kind_default(g);
    }
    for (int k = 0; k < 4; ++k) {
        if (current) current[k] = cur[k];
        if (defaults) defaults[k] = def[k];
    }
    return PET_OS_OK;
}

// 3D: the single-request back-projector's slices per block (16, 32, 64, at
// most the default) and ring differences per staging group (4, 8), timed on
// the first subset; the forward projector has a single shape.  Cached as
// "0 <zb * 16 + dpg>".
static int autotune3(pet_os_geom* g, GeomExtra* ex, int32_t flags, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const std::string key = tune_key(g->d);
    int seg = 0, code = -1;
    if (!(flags & 1) && cache_lookup(key, seg, code) && code > 0) {
        // a cached shape is taken if it is one the tuner could have chosen
        const int zb = code / 16, dpg = code % 16;
        int nb, rw, dq, half, lds;
        if ((zb == 16 || zb == 32 || zb == 64) && zb <= bp3_zb(g) && (dpg == 4 || dpg == 8) &&
            bp3_shape_single(g, zb, dpg, nb, rw, dq, half, lds) == PET_OS_OK) {
            g->tuned_zb = zb;
            g->tuned_dpg = dpg;
            return PET_OS_OK;
        }
    }
    // + 4 floats: the 3D back-projector's 16-byte staging loads may read up to
    // three bins past the last row
    const size_t nw = (size_t)g->max_sub_angles * g->n_planes * g->d.n_radial;
    float *w = nullptr, *img = nullptr;
    if (hipMalloc(&w, (nw + 4) * sizeof(float)) != hipSuccess || hipMalloc(&img, (size_t)g->n_vox * sizeof(float)) != hipSuccess) {
        if (w) (void)hipFree(w);
        return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc failed in autotune");
    }
    int rc = launch_fill(w, (int64_t)nw, 0.5f, s);
    const int saved_zb = g->tuned_zb, saved_dpg = g->tuned_dpg;
    // the default shape first (its staging group as the default rule picks it)
    int nb = 0, rw = 0, dpg0 = 0, half = 0, lds = 0;
    const int zb0 = bp3_zb(g);
    if (!rc) rc = bp3_shape_single(g, zb0, 0, nb, rw, dpg0, half, lds);
    TunePick pick;
    std::vector<int> codes{zb0 * 16 + dpg0};
    const int zbs[] = {16, 32, 64};
    const int dpgs[] = {4, 8};
    for (int zb : zbs)
        for (int dpg : dpgs)
            if (zb <= zb0 && zb * 16 + dpg != codes[0]) codes.push_back(zb * 16 + dpg);
    for (int code : codes) {
        if (rc) break;
        const int zb = code / 16, dpg = code % 16;
        int dq;
        if (bp3_shape_single(g, zb, dpg, nb, rw, dq, half, lds)) continue;   // does not fit
        g->tuned_zb = zb;
        g->tuned_dpg = dpg;
        BPLaunch L{};
        L.w = w; L.w_natural = 0; L.angles = ex->subset_lists; L.n_al = ex->subset_count[0]; L.out = img;
        float ms = 0;
        rc = time_launch(s, 5, [&]() { return launch_bp(g, L, s); }, &ms);
        if (!rc) pick.offer(code, ms);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(w);
    (void)hipFree(img);
    if (rc || pick.value <= 0) {
        g->tuned_zb = saved_zb;
        g->tuned_dpg = saved_dpg;
        return rc ? rc : fail(PET_OS_ERR_INVALID_ARG, "3D geometry: no back-projector shape fits");
    }
    g->tuned_zb = pick.value / 16;
    g->tuned_dpg = pick.value % 16;
    cache_store(key, 0, pick.value);
    return PET_OS_OK;
}

extern "C" int pet_os_autotune(pet_os_geom* g, int32_t flags, pet_os_stream stream) {
    if (!g) return fail(PET_OS_ERR_INVALID_ARG, "geom is NULL");
    GeomExtra* ex = extra_of(g);
    if (!ex) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    if (g->d.dim == 3) return autotune3(g, ex, flags, (hipStream_t)stream);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const std::string key = tune_key(g->d);
    int seg = 0, kind = -1;
    // a cached shape is taken if it is one the tuner could have chosen
    if (!(flags & 1) && cache_lookup(key, seg, kind) && (seg == 1 || seg == 4 || seg == 16 || seg == 64) &&
        (kind == 0 || kind == 1)) {
        g->tuned_seg = seg;
        g->tuned_bp_kind = kind;
        return PET_OS_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t nw = (size_t)g->max_sub_angles * g->n_planes * g->d.n_radial;
    float *f = nullptr, *w = nullptr, *img = nullptr;
    if (hipMalloc(&f, (size_t)g->n_vox * sizeof(float)) != hipSuccess ||
        hipMalloc(&w, (nw + 4) * sizeof(float)) != hipSuccess || hipMalloc(&img, (size_t)g->n_vox * sizeof(float)) != hipSuccess) {
        if (f) (void)hipFree(f);
        if (w) (void)hipFree(w);
        return fail(PET_OS_ERR_OUT_OF_MEMORY, "hipMalloc failed in autotune");
    }
    int rc = launch_fill(f, g->n_vox, 1.0f, s);
    if (!rc) rc = launch_fill(w, (int64_t)nw, 0.5f, s);
    const int* angles = ex->subset_lists;
    const int n_al = ex->subset_count[0];
    // forward projector: threads per ray, the default shape first
    const int seg0 = fp_seg_for(g, (long long)g->max_sub_angles * g->n_planes * g->d.n_radial, 0);
    TunePick seg_pick;
    const int segs2[] = {seg0, 1, 4, 16, 64};
    for (int k = 0; k < 5 && !rc; ++k) {
        const int sg = segs2[k];
        if (k > 0 && sg == seg0) continue;
        FPLaunch F{};
        F.f = f; F.out = w; F.angles = angles; F.n_al = n_al; F.mode = FP_COMPACT; F.seg = sg;
        float ms = 0;
        rc = time_launch(s, 5, [&]() { return launch_fp(g, F, s); }, &ms);
        if (!rc) seg_pick.offer(sg, ms);
    }
    // back-projector tile (2D only), the default tile first
    int best_kind = -1;
    if (!rc && g->d.dim == 2) {
        const int saved = g->tuned_bp_kind;
        const int kind0 = bp_kind_default(g);
        TunePick kind_pick;
        const int kinds[] = {kind0, 1 - kind0};
        for (int kd : kinds) {
            if (rc) break;
            g->tuned_bp_kind = kd;
            BPLaunch L{};
            L.w = w; L.w_natural = 0; L.angles = angles; L.n_al = n_al; L.out = img;
            float ms = 0;
            rc = time_launch(s, 5, [&]() { return launch_bp(g, L, s); }, &ms);
            if (!rc) kind_pick.offer(kd, ms);
        }
        g->tuned_bp_kind = saved;
        best_kind = kind_pick.value;
    }
    const int best_seg = seg_pick.value;
    (void)hipStreamSynchronize(s);
    (void)hipFree(f);
    (void)hipFree(w);
    (void)hipFree(img);
    if (rc) return rc;
    g->tuned_seg = best_seg;
    g->tuned_bp_kind = best_kind;
    cache_store(key, best_seg, best_kind);
    return PET_OS_OK;
}
