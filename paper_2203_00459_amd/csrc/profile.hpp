// Optional per-kernel timing: when enabled, every launch of the library is
// bracketed by two HIP events on its stream.  Events come from a pool created
// by fmbym_profile_enable, so the search calls still allocate nothing.
#pragma once
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

namespace fmbym {

enum KernelId {
    kKRows1 = 0, kKCols1, kKPolar, kKAngleFin, kKRows2, kKCols2, kKRows3, kKXyFin,
    kKBRowsFwd2, kKBColsXy, kKBRowsXy, kKBDtheta, kKBPolar, kKBDmag, kKBColsMag, kKBRowsFinal,
    kMInput, kMConvFwd, kMBnStats, kMBnRelu, kMPool, kMUpCat, kMHeadFwd, kMHeadBwd, kMBnBwd, kMWgrad,
    kMConvDgrad, kMPoolBwd, kMUpBwd, kMPack, kMAdam, kMLoss, kKRotate, kKBRotateAdj,
    kKJointSetup, kKJointPeak, kKJointPick, kKTurnSetup, kKTurnPick, kKFinite, kMInputGrad,
    kORows1, kOCols1, kOPolar, kOAngleFin, kORotate, kORows2, kOCols2, kORows3,
    kKernelCount
};

extern const char* const kKernelNames[kKernelCount];

void prof_before(hipStream_t s, int id);
void prof_after(hipStream_t s, int id);

// A named range on the host timeline (roctx) for the lifetime of the object:
// every entry point opens one, so a marker trace (rocprofv3 --marker-trace)
// shows which call enqueued which kernels.  Costs nothing measurable when no
// tool is attached.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// While alive, launches on this thread are not timed (used around graph capture).
struct ProfilePause {
    ProfilePause();
    ~ProfilePause();
};

}  // namespace fmbym

#define FMBYM_LAUNCH(id, kernel, grid, block, stream, ...)                     \
    FMBYM_LAUNCH_LDS(id, kernel, grid, block, 0, stream, __VA_ARGS__)

#define FMBYM_LAUNCH_LDS(id, kernel, grid, block, lds, stream, ...)            \
    do {                                                                      \
        ::fmbym::prof_before((stream), (id));                                 \
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);    \
        ::fmbym::prof_after((stream), (id));                                  \
    } while (0)
