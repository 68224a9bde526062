// fmbym_search_noalloc: the forward search with its workspace in a static
// device array of the library, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid it).
//
// `scratch` is a file-scope device array; every GPU the library runs on holds
// its own copy from module load until the process ends.  Host code never uses
// the array's name as an address: the device address of each GPU's copy comes
// from hipGetSymbolAddress, taken once per device (with that device current)
// on the first call there, and only that address is handed to the kernels.
// The forward writes every workspace word it reads, so nothing in the array
// has to start at zero; calls that overlap on one GPU share the array and race.
#include <mutex>

#include "internal.hpp"
#include "profile.hpp"

using namespace fmbym;

static __device__ __align__(256) char scratch[FMBYM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];     // device address of each device's copy, or null

// Address of the current device's copy of `scratch` (looked up once per device).
int scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return FMBYM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!ptr) return FMBYM_EHIP;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return FMBYM_OK;
}

}  // namespace

extern "C" {

int fmbym_search_noalloc(fmbym_plan plan, int32_t batch, const float* f, const float* g, const float* m_f,
                         const float* m_g, float* pose, float* c_theta, float* c_xy, float* saved,
                         void* stream) {
    const TraceRange trace_range("fmbym_search_noalloc");
    int rc = check_call(plan, batch);
    if (rc) return rc;
    if (!f || !g || !pose) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (m_g == nullptr)) return FMBYM_EINVAL;
    const Plan* pl = plan_cast(plan);
    if (run_fwd_workspace(*pl, batch) > (size_t)FMBYM_NOALLOC_SCRATCH_BYTES) return FMBYM_EWORKSPACE;
    int device = -1;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e);
    if (device != pl->device) return FMBYM_EINVAL;   // the plan's tables live on its own device
    void* ws = nullptr;
    rc = scratch_address(device, &ws);
    if (rc) return rc;
    rc = run_forward(*pl, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, (char*)ws, (hipStream_t)stream,
                     nullptr);
    if (rc) return rc;
    e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

}  // extern "C"
