// internal.h -- private structures of the pet_os library (not part of the ABI).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pet_os.h"
#include "raygeom.h"

namespace petos {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// Timing events of the next kernel launched on this thread through
// petos_launch: the per-kernel profiler hands them over for a bracket that
// holds a single launch, and the dispatch itself records them (no separate
// event packets around the kernel).  Consumed by that launch.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

template <typename... KArgs, typename... Args>
inline void petos_launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t s,
                         Args... args) {
    const LaunchEvents e = g_launch_events;
    g_launch_events = LaunchEvents{};
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, e.start, e.stop, 0u, args...);
}

#define PETOS_HIP(call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::petos::fail(PET_OS_ERR_DEVICE,                                  \
                                 std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- reductions
// Deterministic FP64 sums without device-wide fences: each block of the
// producing kernel writes one partial; whoever needs the total (the next
// kernel in the stream, or a one-block finalize kernel) adds the partials in
// index order.  One Reduction slot per quantity.
struct Reduction {
    double* part;       // [cap] partials
    double* total;      // [1] filled by launch_finalize
    int cap;
};

constexpr int PSF_KMAX = 16;   // largest PSF radius, in pixels, of the 2D blur

enum RedSlot { RED_SUMF = 0, RED_SUMMU = 1, RED_FID = 2, RED_RDP = 3, RED_SUMY = 4, RED_SUMR = 5,
               RED_SUMS = 6, RED_COUNT = 7 };

// ---------------------------------------------------------------- geometry
}  // namespace petos

struct pet_os_geom {
    pet_os_geom_desc d;
    int n_planes;
    int64_t n_vox, n_bins;
    int max_sub_angles;                 // largest subset
    petos::GeoK k;                      // device tables referenced by pointer
    void* dev_block;                    // single allocation holding all tables
    float* pnorm;                       // p_j of eq:pj (device, n_vox)
    float* sens;                        // A^T 1 (device, n_vox)
    double sens_sum;                    // sum_j (A^T 1)_j
    int device;
    int tuned_seg = 0;                  // forward-projector segments per ray (0: heuristic)
    int tuned_bp_kind = -1;             // back-projector tile kind (-1: heuristic)
    int tuned_zb = 0;                   // 3D back-projector slices per block (0: default)
    int tuned_dpg = 0;                  // 3D ring differences per staging group (0: default)
    bool full_model = false;            // sub-rays, PSF or attenuation (2D; single-request paths only)
    std::vector<int> subset_angles(int subset) const;   // subset in 1..M, 0 = all
};

namespace petos {

// Scratch used by one reconstruction (plain path).
struct Work {
    float* w = nullptr;        // compact subset sinogram [al][plane][b]
    float* G = nullptr;        // subset gradient image
    float* mu = nullptr;       // smoothness measure
    float* nu_frozen = nullptr;
    float* fz = nullptr;       // 3D: copy of the iterate with z fastest [(iy*nx+ix)*nz+iz]
    float* fsnap = nullptr;    // 2D: snapshot of the iterate entering the subiteration
    float* gradR = nullptr;    // 3D: penalty gradient of the entering iterate (same storage as fsnap in 2D)
    float* fb = nullptr;       // 2D PSF: the blurred iterate, then the blurred back-projection
    double* red_block = nullptr;   // reductions' storage
    Reduction red[RED_COUNT];
    int* angle_list = nullptr;     // device copy of all subset angle lists [M][max_sub]
    unsigned* check_part = nullptr;            // data check: per-block counts [CHECK_GRID][4]
    unsigned long long* check_total = nullptr; // data check: the four totals
    size_t bytes = 0;
};

int work_alloc(const pet_os_geom* g, bool need_nu, Work* w);
void work_free(Work* w);
// bytes of one request's scratch, and the same scratch placed in caller
// memory at base (cap bytes, 256-byte aligned): no allocation; the reduction
// totals are cleared by a fill kernel on s
size_t work_bytes(const pet_os_geom* g, bool need_nu);
int work_place(const pet_os_geom* g, bool need_nu, void* base, size_t cap, Work* w, hipStream_t s);

// device angle lists of a geometry
struct GeomExtra {
    int* all_angles;     // [n_angles] 0..Na-1
    int* subset_lists;   // [M][max_sub]
    int* d_subset_count; // [M]
    std::vector<int> subset_count;
};
GeomExtra* extra_of(const pet_os_geom* g);

// FP64 scalar schedule
struct Sched {
    double lam, alpha;
    int nu_mode;
};
Sched sched_next(const pet_os_params& p, int M, int64_t k, int i, double* t_nest, int have_frozen);
// (float)(lambda alpha) and nu mode of subiterations J = 1..n_sub from the start
void schedule_table(const pet_os_params& p, int M, int64_t n_sub, std::vector<float>& step, std::vector<int>& nu);
int validate_params(const pet_os_params* p, const pet_os_geom* g);
// FP32 thresholds and clamp values of the box B for bound U and clamp t
BoxK make_box(double U, double t);
int validate_desc(const pet_os_geom_desc* d);

// ---------------------------------------------------------------- launchers (kernels.hip)
enum FPMode { FP_RATIO = 0, FP_PLAIN = 1, FP_OBJECTIVE = 2, FP_COUNT = 3, FP_COMPACT = 4, FP_EM = 5 };

struct FPLaunch {
    const float* f;
    const float* fz = nullptr;   // 3D: the image with z fastest (the 3D projector reads this, not f)
    const float* y;
    const float* r;
    // 3D: (y, r) pairs bin-major, [(angle * n_radial + bin) * n_planes + plane]
    // (launch_yr3), read instead of y and r by the staged forward projector
    const float2* yr = nullptr;
    float* out;              // FP_RATIO, FP_EM, FP_COUNT, FP_COMPACT: compact [al][plane][b]; FP_PLAIN: natural q
    const int* angles;       // device list of natural angle indices for this pass
    int n_al;                // number of angles
    int mode;
    Reduction red;           // FP_OBJECTIVE
    int seg = 0;             // threads per ray (0: tuned or heuristic)
    int raw = 0;             // 1: no attenuation factors (line integrals of f itself)
    // 2D subiteration: pixel pass in the same launch (snapshot of f and mu)
    const float* px_f = nullptr;   // iterate of the pixel pass when f is its PSF-blurred copy
    float* px_fsnap = nullptr;
    float* px_mu = nullptr;
    int px_want_mu = 0;
    const double* px_part_f = nullptr;
    int px_n_part_f = 0;
    Reduction px_red_mu{};
};
int launch_fp(const pet_os_geom* g, const FPLaunch& L, hipStream_t s);
// 3D: the bin-major copy of y and r that the staged forward projector reads
// (yr: n_bins pairs); whether the geometry's forward projector uses it
int launch_yr3(const pet_os_geom* g, const float* y, const float* r, float2* yr, hipStream_t s);
bool fp3_reads_yr(const pet_os_geom* g);

enum NuMode { NU_ONE = 0, NU_COMPUTE = 1, NU_COMPUTE_FREEZE = 2, NU_FROZEN = 3 };

struct BPLaunch {
    const float* w;          // compact [al][plane][b] or natural; nullptr => unit weights
    int w_natural;           // 1: w in natural layout [plane][angle][bin]
    const int* angles;
    int n_al;
    float* out;              // back-projection (plain) or G (fused)
    // fused stencil (when f != nullptr)
    const float* f;
    float* mu;               // written when want_mu
    int want_mu;
    float beta_over_M, gamma_R, eps;
    const double* part_f;    // partials of sum f of the current iterate (for mean f)
    int n_part_f;
    Reduction red_mu;
    // 2D fused update (fnew non-null; f is the snapshot of the iterate)
    float* fnew = nullptr;
    const float* pnorm = nullptr;
    float* nu_frozen = nullptr;
    int nu_mode = 0;
    float step = 0, nu1 = 0, nu2 = 0;
    BoxK box{};
    const double* part_mu = nullptr;   // partials of sum mu from the pixel pass
    int n_part_mu = 0;
    Reduction red_f{};                 // partials of sum of the new iterate
    const float* osem_sens = nullptr;  // 2D fused OSEM update: subset sensitivity of this subset
    // 3D: the penalty gradient of f computed by extra blocks of the
    // back-projector's launch into gradR (with f, mu, want_mu, the penalty
    // constants, part_f and red_mu); the update then adds it to b
    float* gradR = nullptr;
};
int launch_bp(const pet_os_geom* g, const BPLaunch& L, hipStream_t s);
// 2D full model: out = B in (PSF), and the image-space part of a subiteration
// (or of a gradient) after a blurred back-projection Gb = B A_i^T w
int launch_blur(const pet_os_geom* g, const float* in, float* out, hipStream_t s);
int launch_upd2(const pet_os_geom* g, const BPLaunch& L, const float* Gb, bool blur, hipStream_t s);
// y = exp(-x) elementwise (attenuation factors from line integrals of mu)
int launch_expneg(const float* x, float* y, int64_t n, hipStream_t s);

struct UpdLaunch {
    float* f;
    float* fz = nullptr;     // 3D: z-fastest copy, rewritten with the new iterate
    const float* G;
    const float* mu;
    const float* pnorm;
    float* nu_frozen;
    int nu_mode;
    float step;              // lambda_k * alpha_{k,i}
    float nu1, nu2;
    BoxK box;
    const double* part_mu;   // partials of sum mu (from the back-projection)
    int n_part_mu;
    Reduction red_f;         // sum of the new iterate
    const float* osem_sens = nullptr;   // OSEM: subset sensitivity; G = A_i^T (y/(q+r))
    const float* gradR = nullptr;       // 3D: penalty gradient to add, G = b + beta_over_M gradR
    float beta_over_M = 0.0f;
};
int launch_update(const pet_os_geom* g, const UpdLaunch& L, hipStream_t s);

int launch_sum(const float* x, int64_t n, Reduction red, hipStream_t s);
// data check of Sec. II-A (kernels.hip): counts of y entries that are negative
// or not finite, r entries not > 0 or not finite, f entries outside [0, U]
// (f_lim: the smallest float above U) or not finite, and positive f entries,
// into total[4]; part holds CHECK_GRID * 4 block counts
constexpr int CHECK_GRID = 1024;
int launch_check_data(const float* y, const float* r, int64_t nb, const float* f, int64_t nv, float f_lim,
                      unsigned* part, unsigned long long* total, hipStream_t s);
// the data check of one request on its scratch; synchronises the stream and
// returns INVALID_ARG with the rule that failed (capi.cpp)
int check_data(const pet_os_geom* g, const pet_os_params* p, Work* w, const float* f, const float* y,
               const float* r, hipStream_t s);
int launch_rdp_value(const pet_os_geom* g, const float* f, float gamma_R, float eps, Reduction red,
                     hipStream_t s);
int launch_fill(float* x, int64_t n, float v, hipStream_t s);
// total = sum of the first n partials of red (one block, fixed order)
int launch_finalize(Reduction red, int n, hipStream_t s);

// gradient-consistency measure (diag.hip): sum f, then the eight FP64 sums
// <a,b>, |a|^2, |b|^2, count over the smooth and the variable area, which
// end in the last 8 doubles of scratch (angle_scratch_doubles(n_vox) long)
int angle_grid(int64_t n);
size_t angle_scratch_doubles(int64_t n_vox);
int launch_gradient_angles(const pet_os_geom* G, const float* hp, const float* hc, const float* f,
                           double smooth_frac, double var_frac, double* scratch, hipStream_t s);

// grid sizes (for sizing partial arrays)
int fp_seg_for(const pet_os_geom* g, long long nrays, int requested);
int fp_grid_seg(const pet_os_geom* g, int n_al, int seg);
int fp_grid(const pet_os_geom* g, int n_al);
int bp_kind_of(const pet_os_geom* g);
int bp_kind_default(const pet_os_geom* g);   // the heuristic, before any autotuning
int bp_grid_kind(const pet_os_geom* g, int kind);
int bp_grid(const pet_os_geom* g);
int bp_grid_max(const pet_os_geom* g);
int elem_grid(int64_t n);
int px_grid(const pet_os_geom* g);   // blocks of the 2D pixel pass (partials of sum mu)
int px_items(const pet_os_geom* g);  // batched work items of the 2D pixel pass
// number of partials of sum f left by the update (and by launch_sum / launch_prep3)
int sumf_grid(const pet_os_geom* g);
int launch_sum_f(const pet_os_geom* g, const float* f, float* fz, Reduction red, hipStream_t s);

// 3D projectors and update (kernels3d.hip)
int fp3_grid(const pet_os_geom* g, int n_al);
int fp3_launch_grid(const pet_os_geom* g, int n_al);
int bp3_grid(const pet_os_geom* g);          // single-request launch (autotuned shape)
int bp3_grid_batch(const pet_os_geom* g);    // batched launch (default shape)
int bp3_grid_zb(const pet_os_geom* g, int zb);
int bp3_zb(const pet_os_geom* g);
int bp3_shape_single(const pet_os_geom* G, int zb, int dpg_req, int& nb, int& rw, int& dpg, int& half, int& lds);
int upd3_grid(const pet_os_geom* g);
int bp3_shape(const pet_os_geom* g, int& nb, int& zb, int& rw, int& dpg);
int launch_fp3(const pet_os_geom* g, const FPLaunch& L, hipStream_t s);
int launch_bp3(const pet_os_geom* g, const BPLaunch& L, hipStream_t s);
int launch_update3(const pet_os_geom* g, const UpdLaunch& L, hipStream_t s);
// 3D: G = out + (beta/M) grad R(f) in place over the back-projection in
// L.out, mu and the partials of sum mu (L.f, mu, want_mu, beta_over_M,
// gamma_R, eps, part_f, n_part_f, red_mu); one partial per block of pen3_grid
int launch_pen3(const pet_os_geom* g, const BPLaunch& L, hipStream_t s);
int pen3_grid(const pet_os_geom* g);
// z-fastest copy of f and the partials of sum f (same tiles and order as the 3D update)
int launch_prep3(const pet_os_geom* g, const float* f, float* fz, Reduction red, hipStream_t s);
void bp_stage_shape_kind(const pet_os_geom* G, int kind, int& nb_max, int& rows_max, int& chunk, size_t& lds);
size_t bp_lds_budget(int kind);

// ---------------------------------------------------------------- batched execution
// One reconstruction request inside a batch, as the batched kernels see it.
struct SlotDev {
    GeoK g;
    const float* pnorm;
    float* f;
    const float* y;
    const float* r;
    float* w;
    float* G;
    float* mu;
    float* nu_frozen;
    float* fz;                 // 3D: z-fastest copy of f
    float* fsnap;              // 2D: snapshot of f
    int n_fp;                  // 2D: forward-projection blocks before the pixel blocks
    double* part_f;
    double* part_mu;
    int n_part_f, n_part_mu;
    const int* subset_lists;
    const int* subset_count;
    int max_sub;
    const float* sched_step;   // [J_end] lambda_k alpha_{k,i} of subiteration J (index J-1)
    const int* sched_nu;       // [J_end] nu mode of subiteration J
    int J, J_end;              // next subiteration (device-advanced), last one
    float beta_over_M, gamma_R, eps, nu1, nu2;
    BoxK box;
    int fp_seg, bp_kind;
    int nb_max, rows_max, chunk;   // back-projector staging (3D: bins, rows, ring differences per group)
    int zb;                        // 3D: slices per back-projection block
    int active;
};

struct Item {
    int slot;
    int block;
};

// work lists: 2D forward + pixel pass, 2D back-projection + update per tile
// kind, and the 3D forward, back-projection per z-block size (16/32/64),
// penalty gradient and mu, and update
// (lists WL_BP3 + 2 * zi + wi: z-block 16/32/64 for zi = 0/1/2, LDS row
// stride 20/40 bins for wi = 0/1)
enum { WL_FP = 0, WL_BP0 = 1, WL_BP1 = 2, WL_FP3 = 3, WL_BP3 = 4, WL_UPD3 = 10, WL_PEN3 = 11, WL_COUNT = 12 };

// Queue one batched subiteration (every active slot advances by one):
// forward, back-projection (one launch per tile kind), update, advance.
// Lists whose bit is clear in `live_mask` are not launched.
int launch_batch_step(SlotDev* d_slots, int n_slots, Item* const lists[WL_COUNT], const int* d_counts,
                      const int grids[WL_COUNT], int live_mask, hipStream_t s);
void launch_batch3_fp(const SlotDev* d_slots, const Item* list, const int* cnt, int grid, hipStream_t s);
void launch_batch3_bp(const SlotDev* d_slots, const Item* list, const int* cnt, int grid, int zb, int nbs,
                      hipStream_t s);
int bp3_nbs_of(const pet_os_geom* g);   // LDS row stride of the 3D back-projector (20 or 40)
void launch_batch3_upd(const SlotDev* d_slots, const Item* list, const int* cnt, int grid, hipStream_t s);
void launch_batch3_pen(const SlotDev* d_slots, const Item* list, const int* cnt, int grid, hipStream_t s);

}  // namespace petos

namespace petos {
// n_iter iterations of Table I on a state (no objective evaluations), queued on s
int run_plain(pet_os_state* st, float* f, const float* y, const float* r, int n_iter, hipStream_t s);
}  // namespace petos

// per-request state of the plain path
struct pet_os_state {
    const pet_os_geom* g;
    pet_os_params p;
    int64_t k;
    int32_t i;
    double t_nest;
    int have_frozen;
    petos::Work w;
    float* osem_sens = nullptr;         // OSEM: the M subset sensitivities [M][n_voxels]
    double* obj_dev = nullptr;          // (fid, R) pairs of queued objective evaluations
    int obj_cap = 0;
    int prof_kernel = -1;               // kernel bracketed by events, -1 = none
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
    size_t prof_used = 0;
    // the (f, y, r) buffers whose data last passed the check of Sec. II-A
    const float* checked_f = nullptr;
    const float* checked_y = nullptr;
    const float* checked_r = nullptr;
    // 3D: bin-major copy of the (y, r) buffers yr_y, yr_r (made with the data
    // check, when the state may allocate)
    float2* yr = nullptr;
    const float* yr_y = nullptr;
    const float* yr_r = nullptr;
    bool may_allocate = true;
};

