// Per-kernel event timing behind fmbym_profile_enable / fmbym_profile_read.
#include <atomic>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "profile.hpp"

namespace fmbym {

static_assert(kKernelCount <= 64, "profile_read hands out at most 64 entries");

const char* const kKernelNames[kKernelCount] = {
    "k_rows1", "k_cols1", "k_polar", "k_angle_fin", "k_rows2", "k_cols2", "k_rows3", "k_xy_fin",
    "kb_rows_fwd2", "kb_cols_xy", "kb_rows_xy", "kb_dtheta", "kb_polar", "kb_dmag", "kb_cols_mag",
    "kb_rows_final",
    "m_input8", "m_conv_fwd", "m_bn_stats", "m_bn_relu", "m_maxpool", "m_up_concat", "m_head_fwd",
    "m_head_bwd", "m_bn_bwd", "m_wgrad", "m_conv_dgrad", "m_pool_bwd", "m_up_bwd", "m_pack", "m_adam",
    "m_pose_loss", "k_rotate", "kb_rotate_adj", "k_joint_setup", "k_joint_peak", "k_joint_pick",
    "k_turn_setup", "k_turn_pick", "k_finite", "m_input_grad",
    "ko_rows1", "ko_cols1", "ko_polar", "ko_angle_fin", "ko_rotate", "ko_rows2", "ko_cols2", "ko_rows3",
};

namespace {

struct Rec {
    hipEvent_t a, b;
    int id;
};

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Rec> g_pool;   // pre-created events
size_t g_used = 0;
int g_open_id = -1;
bool g_overflow = false;
thread_local int g_paused = 0;

}  // namespace

ProfilePause::ProfilePause() { ++g_paused; }
ProfilePause::~ProfilePause() { --g_paused; }

void prof_before(hipStream_t s, int id) {
    if (g_paused || !g_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_used >= g_pool.size()) {
        g_overflow = true;
        g_open_id = -1;
        return;
    }
    g_pool[g_used].id = id;
    g_open_id = id;
    (void)hipEventRecord(g_pool[g_used].a, s);
}

void prof_after(hipStream_t s, int id) {
    if (g_paused || !g_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_open_id != id) return;
    (void)hipEventRecord(g_pool[g_used].b, s);
    ++g_used;
    g_open_id = -1;
}

}  // namespace fmbym

using namespace fmbym;

extern "C" {

FMBYM_API int fmbym_profile_enable(int32_t capacity) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on.store(0);
    for (auto& r : g_pool) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_pool.clear();
    g_used = 0;
    g_overflow = false;
    g_open_id = -1;
    if (capacity <= 0) return FMBYM_OK;
    g_pool.resize((size_t)capacity);
    for (auto& r : g_pool) {
        hipError_t e = hipEventCreate(&r.a);
        if (e == hipSuccess) e = hipEventCreate(&r.b);
        if (e != hipSuccess) {
            g_pool.clear();
            return FMBYM_EHIP;
        }
    }
    g_on.store(1);
    return FMBYM_OK;
}

FMBYM_API int fmbym_profile_read(int32_t max_kernels, const char** names, double* total_ms,
                                 int32_t* launches) {
    if (max_kernels < 64 || !names || !total_ms || !launches) return FMBYM_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    for (int k = 0; k < kKernelCount; ++k) {
        names[k] = kKernelNames[k];
        total_ms[k] = 0.0;
        launches[k] = 0;
    }
    for (size_t i = 0; i < g_used; ++i) {
        hipError_t e = hipEventSynchronize(g_pool[i].b);
        if (e != hipSuccess) return FMBYM_EHIP;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, g_pool[i].a, g_pool[i].b);
        if (e != hipSuccess) return FMBYM_EHIP;
        total_ms[g_pool[i].id] += ms;
        launches[g_pool[i].id] += 1;
    }
    return g_overflow ? FMBYM_EWORKSPACE : (int)kKernelCount;
}

}  // extern "C"
