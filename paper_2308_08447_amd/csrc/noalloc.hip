// noalloc.hip -- RK4 steps that allocate no device memory (llg_step_noalloc).
//
// llg_step keeps its four RK4 stage buffers (H, A, B and the slope
// accumulator, 12 N floats) in the plan and allocates them on first use, and
// its multi-step path instantiates a HIP graph.  Callers that may not allocate
// (code under stream capture, tight serving loops, harnesses that forbid
// hipMalloc) take llg_step_noalloc instead: its stage buffers are the fixed
// array below, one copy per GPU that the library runs on, held until the
// process ends, and its steps are launched eagerly.
//
// In host code the array's name stands for a host-side shadow, not for device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels.  Every call on a GPU shares that GPU's copy; calls that
// overlap on one GPU (different streams or threads) race on it.  The stage
// kernels write each buffer before they read it (the accumulator is set, not
// added to, by the first stage), so the array needs no clearing.
#include <map>
#include <mutex>
#include <string>

#include "plan.h"

namespace dm {

// 64 MiB: RK4 buffers for up to 1,398,101 cells (48 bytes per cell)
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;

static __device__ __align__(256) float scratch[NOALLOC_SCRATCH_BYTES / sizeof(float)];

static std::mutex g_scratch_mu;
static std::map<int, float*> g_scratch_ptr;  // device -> device address of `scratch`

// Device address of this device's copy of `scratch` (looked up on first use).
static int scratch_address(int dev, float** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return DEMAG_OK;
    }
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        return fail(DEMAG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
    *out = static_cast<float*>(ptr);
    return DEMAG_OK;
}

}  // namespace dm

using namespace dm;

extern "C" {

size_t llg_noalloc_max_cells(void) { return NOALLOC_SCRATCH_BYTES / (12 * sizeof(float)); }

int llg_step_noalloc(demag_plan* plan, float* m, const llg_params* prm, double dt, int32_t nsteps,
                     void* stream) {
    if (!plan || !m) return fail(DEMAG_EINVAL, "plan and m must be non-NULL");
    int rc = check_llg_params(prm, dt, nsteps);
    if (rc) return rc;
    if (plan->flags & DEMAG_EXTRAPOLATE_HD)
        return fail(DEMAG_EUNSUPPORTED,
                    "llg_step_noalloc: plans with DEMAG_EXTRAPOLATE_HD keep an H_d history; use llg_step");
    const size_t need = 12 * plan->g.cells() * sizeof(float);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(DEMAG_EINVAL, "llg_step_noalloc: the mesh needs " + std::to_string(need) +
                                      " bytes of RK4 buffers, more than the fixed " +
                                      std::to_string(NOALLOC_SCRATCH_BYTES) + " (at most " +
                                      std::to_string(llg_noalloc_max_cells()) + " cells)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DEMAG_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev != plan->device)
        return fail(DEMAG_EINVAL, "llg_step_noalloc: the current device is not the plan's device");
    float* rk = nullptr;
    if ((rc = scratch_address(dev, &rk))) return rc;
    LLGStep st{plan, m, *prm, dt};
    st.rk = rk;
    hipStream_t s = (hipStream_t)stream;
    for (int step = 0; step < nsteps; ++step)
        if ((rc = rk4_step_batch(&st, 1, s))) return rc;
    return DEMAG_OK;
}

}  // extern "C"
