// noalloc.cpp -- pet_os_reconstruct_noalloc: the plain reconstruction with the
// request's scratch in a static device array instead of allocated memory, for
// callers that cannot allocate device memory.
//
// The array below is this library's own global in device memory: every GPU
// the library runs on holds one copy of PET_OS_NOALLOC_SCRATCH_BYTES until the
// process ends.  Host code never uses its name as an address: at a device's
// first call the device address of that device's copy is looked up once
// (hipGetSymbolAddress) and kept, and only that address reaches kernels and
// fills.  Every call on a GPU shares the GPU's copy, so calls that overlap on
// one GPU (other streams, other threads) race; calls queued on one stream run
// one after the other.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)PET_OS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};   // device address of scratch, per device

// the current device's copy of scratch (looked up at its first use)
int scratch_of_current_device(int* device, void** out) {
    int dev = -1;
    PETOS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return petos::fail(PET_OS_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return petos::fail(PET_OS_ERR_DEVICE,
                               std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *device = dev;
    *out = g_scratch_ptr[dev];
    return PET_OS_OK;
}

}  // namespace

using namespace petos;

extern "C" int pet_os_reconstruct_noalloc(const pet_os_geom* g, const pet_os_params* p, float* f, const float* y,
                                          const float* r, int32_t n_iter, pet_os_stream stream) {
    if (!g || !p || !f || !y || !r) return fail(PET_OS_ERR_INVALID_ARG, "NULL argument");
    if (!extra_of(g)) return fail(PET_OS_ERR_INVALID_ARG, "invalid geometry");
    if (n_iter < 0) return fail(PET_OS_ERR_INVALID_ARG, "n_iter must be >= 0");
    int rc = validate_params(p, g);
    if (rc) return rc;
    if (p->mode == PET_OS_OSEM)
        return fail(PET_OS_ERR_INVALID_ARG, "OSEM needs the subset sensitivities of a state: use pet_os_reconstruct");
    int dev = -1;
    void* base = nullptr;
    if ((rc = scratch_of_current_device(&dev, &base))) return rc;
    if (dev != g->device) return fail(PET_OS_ERR_INVALID_ARG, "the geometry belongs to another device");
    hipStream_t s = (hipStream_t)stream;
    // a state on the stack: its scratch is placed in the static area, it owns
    // no memory and takes no profiling events
    pet_os_state st;
    st.g = g;
    st.p = *p;
    st.k = 0;
    st.i = 1;
    st.t_nest = 1.0;
    st.have_frozen = 0;
    st.may_allocate = false;    // y and r read in their natural layout
    const bool need_nu = p->mode == PET_OS_P1 || p->mode == PET_OS_P2;
    if ((rc = work_place(g, need_nu, base, SCRATCH_BYTES, &st.w, s))) return rc;
    // the data check of Sec. II-A before anything of the iterations is queued
    if ((rc = check_data(g, p, &st.w, f, y, r, s))) return rc;
    return run_plain(&st, f, y, r, n_iter, s);
}
