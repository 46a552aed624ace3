// internal.h -- private structures of the pet_os library (not part of the ABI).
#pragma once
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
    std::vector<int> subset_angles(int subset) const;   // subset in 1..M, 0 = all
};

namespace petos {

// Scratch used by one reconstruction (plain path).
struct Work {
    float* w = nullptr;        // compact subset sinogram [al][plane][b]
    float* G = nullptr;        // subset gradient image
    float* mu = nullptr;       // smoothness measure
    float* nu_frozen = nullptr;
    float* q_all = nullptr;    // (unused placeholder for objective if needed)
    double* red_block = nullptr;   // reductions' storage
    Reduction red[RED_COUNT];
    int* angle_list = nullptr;     // device copy of all subset angle lists [M][max_sub]
    size_t bytes = 0;
};

int work_alloc(const pet_os_geom* g, bool need_nu, Work* w);
void work_free(Work* w);

// ---------------------------------------------------------------- launchers (kernels.hip)
enum FPMode { FP_RATIO = 0, FP_PLAIN = 1, FP_OBJECTIVE = 2, FP_COUNT = 3 };

struct FPLaunch {
    const float* f;
    const float* y;
    const float* r;
    float* out;              // FP_RATIO, FP_COUNT: compact [al][plane][b]; FP_PLAIN: natural q
    const int* angles;       // device list of natural angle indices for this pass
    int n_al;                // number of angles
    int mode;
    Reduction red;           // FP_OBJECTIVE
};
int launch_fp(const pet_os_geom* g, const FPLaunch& L, hipStream_t s);

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
};
int launch_bp(const pet_os_geom* g, const BPLaunch& L, hipStream_t s);

struct UpdLaunch {
    float* f;
    const float* G;
    const float* mu;
    const float* pnorm;
    float* nu_frozen;
    int nu_mode;
    float step;              // lambda_k * alpha_{k,i}
    float nu1, nu2, U, t_clip;
    const double* part_mu;   // partials of sum mu (from the back-projection)
    int n_part_mu;
    Reduction red_f;         // sum of the new iterate
};
int launch_update(const pet_os_geom* g, const UpdLaunch& L, hipStream_t s);

int launch_sum(const float* x, int64_t n, Reduction red, hipStream_t s);
int launch_rdp_value(const pet_os_geom* g, const float* f, float gamma_R, float eps, Reduction red,
                     hipStream_t s);
int launch_fill(float* x, int64_t n, float v, hipStream_t s);
// total = sum of the first n partials of red (one block, fixed order)
int launch_finalize(Reduction red, int n, hipStream_t s);

// grid sizes (for sizing partial arrays)
int fp_grid(const pet_os_geom* g, int n_al);
int bp_grid(const pet_os_geom* g);
int elem_grid(int64_t n);

}  // namespace petos
