// Ragged work lists: pairs of mixed scan sizes searched as one replayable
// launch.  Pairs are grouped by (n, mask kind) in size order, the kinds being
// unmasked, caller masks and network masks; each group is the batched forward
// search of its plan reading its scans through a per-pair pointer table
// (network-masked groups first run the mask network in inference mode on
// their 2 count scans, read through a second table), followed by a small kernel
// that moves the group's poses to the caller's order and stamps the device
// wall clock.  The groups are
// independent branches of one HIP graph captured at creation, so the small
// sizes do not wait behind the large ones and a replay costs one launch call.
#include <algorithm>
#include <new>
#include <vector>

#include "internal.hpp"
#include "mask_net.hpp"
#include "profile.hpp"

namespace fmbym {

namespace {

enum MaskKind { kUnmasked = 0, kGiven = 1, kNet = 2 };

struct Group {
    const Plan* plan;
    int kind;
    int first;          // first slot (row of the pointer table)
    int count;
    size_t ws_off;      // forward workspace of the group
    size_t pose_off;    // [count][3] float poses of the group
    size_t act_off, act_bytes, mask_off;   // network groups: activations, masks [2 count][n][n]
    int xtab_first;     // network groups: first row of the scan table (2 count rows)
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Validate the work list and lay out its groups; slots[] lists the pairs in
// group order.  Returns FMBYM_OK or an error code; sets *bytes to the workspace.
int plan_groups(const fmbym_plan* plans, int n_plans, const fmbym_pair* pairs, int n_pairs,
                const fmbym_mask_desc* net, std::vector<Group>& groups, std::vector<int>& slots,
                size_t* bytes) {
    if (!plans || n_plans < 1 || n_plans > 64 || !pairs || n_pairs < 1 || n_pairs > (1 << 20))
        return FMBYM_EINVAL;
    for (int k = 0; k < n_plans; ++k) {
        if (!plans[k]) return FMBYM_EINVAL;
        if (odd_side(plan_cast(plans[k])->p.n)) return FMBYM_EUNSUPPORTED;   // odd sides: packed batches only
        for (int j = 0; j < k; ++j)
            if (plan_cast(plans[j])->p.n == plan_cast(plans[k])->p.n) return FMBYM_EINVAL;
    }
    std::vector<int> plan_of(n_pairs), kind(n_pairs);
    for (int i = 0; i < n_pairs; ++i) {
        const fmbym_pair& q = pairs[i];
        if ((q.flags & ~FMBYM_PAIR_NET_MASK) || !q.f || !q.g || (q.m_f == nullptr) != (q.m_g == nullptr))
            return FMBYM_EINVAL;
        if (q.flags & FMBYM_PAIR_NET_MASK) {
            if (!net || q.m_f) return FMBYM_EINVAL;
            kind[i] = kNet;
        } else {
            kind[i] = q.m_f ? kGiven : kUnmasked;
        }
        plan_of[i] = -1;
        for (int k = 0; k < n_plans; ++k)
            if (plan_cast(plans[k])->p.n == q.n) plan_of[i] = k;
        if (plan_of[i] < 0) return FMBYM_EINVAL;
    }
    // groups in increasing n, then by mask kind; pairs keep their order
    std::vector<int> key(n_pairs);
    for (int i = 0; i < n_pairs; ++i) key[i] = pairs[i].n * 4 + kind[i];
    slots.resize(n_pairs);
    for (int i = 0; i < n_pairs; ++i) slots[i] = i;
    std::stable_sort(slots.begin(), slots.end(), [&](int a, int b) { return key[a] < key[b]; });
    groups.clear();
    size_t off = 0;
    int xrows = 0;
    for (int s = 0; s < n_pairs;) {
        int e = s;
        while (e < n_pairs && key[slots[e]] == key[slots[s]]) ++e;
        Group gr{};
        gr.plan = plan_cast(plans[plan_of[slots[s]]]);
        gr.kind = kind[slots[s]];
        gr.first = s;
        gr.count = e - s;
        gr.ws_off = off;
        off = align256(off + fwd_layout(gr.plan->p, gr.count).total);
        gr.pose_off = off;
        off = align256(off + (size_t)gr.count * 3 * sizeof(float));
        if (gr.kind == kNet) {
            const int n = gr.plan->p.n;
            gr.act_bytes = fmbym_mask_activation_bytes(net, 2 * gr.count, n);
            if (gr.act_bytes == 0) return FMBYM_EUNSUPPORTED;
            gr.act_off = off;
            off = align256(off + gr.act_bytes);
            gr.mask_off = off;
            off = align256(off + (size_t)2 * gr.count * n * n * sizeof(float));
            gr.xtab_first = xrows;
            xrows += 2 * gr.count;
        }
        groups.push_back(gr);
        s = e;
    }
    *bytes = off;
    return FMBYM_OK;
}

// Host copy of the device pointer table: rows (f, g, m_f, m_g) of every pair in
// slot order, then the scan rows of the network groups; network masks of a
// group live at its mask_off in `workspace`.
std::vector<const float*> pointer_table(const std::vector<Group>& groups, const std::vector<int>& slots,
                                        const fmbym_pair* pairs, int n_pairs, const void* workspace) {
    size_t xrows = 0;
    for (const Group& gr : groups)
        if (gr.kind == kNet) xrows += 2 * (size_t)gr.count;
    std::vector<const float*> tab(4 * (size_t)n_pairs + xrows);
    for (const Group& gr : groups) {
        const int n = gr.plan->p.n;
        for (int b = 0; b < gr.count; ++b) {
            const int s = gr.first + b;
            const fmbym_pair& q = pairs[slots[s]];
            tab[4 * s] = q.f;
            tab[4 * s + 1] = q.g;
            tab[4 * s + 2] = q.m_f;
            tab[4 * s + 3] = q.m_g;
            if (gr.kind == kNet) {
                const float* masks = (const float*)((const char*)workspace + gr.mask_off);
                tab[4 * s + 2] = masks + (size_t)b * n * n;                 // network mask of f
                tab[4 * s + 3] = masks + (size_t)(gr.count + b) * n * n;    // and of g
                tab[4 * (size_t)n_pairs + gr.xtab_first + b] = q.f;
                tab[4 * (size_t)n_pairs + gr.xtab_first + gr.count + b] = q.g;
            }
        }
    }
    return tab;
}

__global__ void k_ragged_start(unsigned long long* __restrict__ stamps, int n_pairs) {
    if (threadIdx.x == 0) stamps[n_pairs] = (unsigned long long)wall_clock64();
}

// Poses of one group to the caller's order, then the time they were written.
__global__ void k_ragged_poses(const float* __restrict__ pose_g, const int* __restrict__ slot_pair,
                               int count, float* __restrict__ pose,
                               unsigned long long* __restrict__ stamps) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const int i = slot_pair[b];
    pose[3 * i] = pose_g[3 * b];
    pose[3 * i + 1] = pose_g[3 * b + 1];
    pose[3 * i + 2] = pose_g[3 * b + 2];
    if (stamps) stamps[i] = (unsigned long long)wall_clock64();
}

}  // namespace

struct Ragged {
    int device = 0;
    int n_pairs = 0;
    fmbym_mask_desc net{};          // copy of the network descriptor (network groups)
    const float** tab = nullptr;    // device [n_pairs][4] (f, g, m_f, m_g) in slot order,
                                    // then the network groups' scan rows
    int* slot_pair = nullptr;       // device [n_pairs] pair index of each slot
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static hipError_t ragged_free(Ragged* r) {
    hipError_t first = hipSuccess;
    auto keep = [&](hipError_t e) {
        if (first == hipSuccess) first = e;
    };
    if (r->exec) keep(hipGraphExecDestroy(r->exec));
    if (r->graph) keep(hipGraphDestroy(r->graph));
    for (hipEvent_t e : r->events) keep(hipEventDestroy(e));
    for (hipStream_t s : r->streams) keep(hipStreamDestroy(s));
    if (r->tab) keep(hipFree(r->tab));
    if (r->slot_pair) keep(hipFree(r->slot_pair));
    delete r;
    return first;
}

// Enqueue the work list on s0, forking one branch per group (used under capture).
static int record_launch(Ragged& r, const std::vector<Group>& groups, float* pose,
                         unsigned long long* stamps, char* ws) {
    hipStream_t s0 = r.streams[0];
    if (stamps) hipLaunchKernelGGL(k_ragged_start, dim3(1), dim3(64), 0, s0, stamps, r.n_pairs);
    hipError_t e = hipEventRecord(r.events[0], s0);
    for (size_t k = 0; k < groups.size() && e == hipSuccess; ++k) {
        const Group& gr = groups[k];
        hipStream_t sg = r.streams[1 + k];
        e = hipStreamWaitEvent(sg, r.events[0], 0);
        if (e != hipSuccess) break;
        float* pose_g = (float*)(ws + gr.pose_off);
        if (gr.kind == kNet) {
            const int rc = mask_forward(&r.net, 2 * gr.count, gr.plan->p.n, nullptr,
                                        r.tab + 4 * (size_t)r.n_pairs + gr.xtab_first,
                                        (float*)(ws + gr.mask_off), ws + gr.act_off, gr.act_bytes, 0, sg);
            if (rc) return rc;
        }
        const int rc = launch_forward(*gr.plan, gr.count, nullptr, nullptr, nullptr, nullptr, pose_g,
                                      nullptr, nullptr, nullptr, ws + gr.ws_off, sg,
                                      r.tab + 4 * (size_t)gr.first);
        if (rc) return rc;
        hipLaunchKernelGGL(k_ragged_poses, dim3((gr.count + 63) / 64), dim3(64), 0, sg, pose_g,
                           r.slot_pair + gr.first, gr.count, pose, stamps);
        e = hipEventRecord(r.events[1 + k], sg);
        if (e == hipSuccess) e = hipStreamWaitEvent(s0, r.events[1 + k], 0);
    }
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

}  // namespace fmbym

namespace fmbym {
namespace {

// The one-call form's workspace: the groups' regions, then the pointer table
// and the slot list that fmbym_ragged_create would allocate.
struct OneCall {
    size_t tab_off, slot_off, total;
};

OneCall one_call_layout(size_t groups_bytes, size_t tab_rows, int n_pairs) {
    OneCall o{};
    o.tab_off = align256(groups_bytes);
    o.slot_off = align256(o.tab_off + tab_rows * sizeof(const float*));
    o.total = align256(o.slot_off + (size_t)n_pairs * sizeof(int));
    return o;
}

size_t net_rows(const std::vector<Group>& groups) {
    size_t x = 0;
    for (const Group& gr : groups)
        if (gr.kind == kNet) x += 2 * (size_t)gr.count;
    return x;
}

}  // namespace
}  // namespace fmbym

using namespace fmbym;

extern "C" {

size_t fmbym_ragged_workspace_size(const fmbym_plan* plans, int32_t n_plans, const fmbym_pair* pairs,
                                   int32_t n_pairs, const fmbym_mask_desc* net) {
    std::vector<Group> groups;
    std::vector<int> slots;
    size_t bytes = 0;
    if (plan_groups(plans, n_plans, pairs, n_pairs, net, groups, slots, &bytes)) return 0;
    return bytes;
}

int fmbym_ragged_create(const fmbym_plan* plans, int32_t n_plans, const fmbym_pair* pairs,
                        int32_t n_pairs, const fmbym_mask_desc* net, float* pose, uint64_t* stamps,
                        void* workspace, size_t workspace_bytes, fmbym_ragged* out) {
    if (!out) return FMBYM_EINVAL;
    *out = nullptr;
    std::vector<Group> groups;
    std::vector<int> slots;
    size_t bytes = 0;
    int rc = plan_groups(plans, n_plans, pairs, n_pairs, net, groups, slots, &bytes);
    if (rc) return rc;
    if (!pose) return FMBYM_EINVAL;
    if (!workspace || workspace_bytes < bytes) return FMBYM_EWORKSPACE;

    Ragged* r = new (std::nothrow) Ragged();
    if (!r) return FMBYM_EINVAL;
    r->n_pairs = n_pairs;
    if (net) r->net = *net;
    const std::vector<const float*> tab = pointer_table(groups, slots, pairs, n_pairs, workspace);
    hipError_t e = hipGetDevice(&r->device);
    if (e == hipSuccess) e = hipMalloc((void**)&r->tab, sizeof(const float*) * tab.size());
    if (e == hipSuccess) e = hipMalloc((void**)&r->slot_pair, sizeof(int) * n_pairs);
    if (e == hipSuccess)
        e = hipMemcpy(r->tab, tab.data(), sizeof(const float*) * tab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(r->slot_pair, slots.data(), sizeof(int) * n_pairs, hipMemcpyHostToDevice);
    for (size_t k = 0; k <= groups.size() && e == hipSuccess; ++k) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) r->streams.push_back(st);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) r->events.push_back(ev);
    }
    if (e != hipSuccess) {
        ragged_free(r);
        return hip_fail(e);
    }
    // capture: the profiling hooks stay out of the graph
    ProfilePause pause;
    e = hipStreamBeginCapture(r->streams[0], hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        ragged_free(r);
        return hip_fail(e);
    }
    rc = record_launch(*r, groups, pose, (unsigned long long*)stamps, (char*)workspace);
    hipGraph_t graph = nullptr;
    hipError_t e_end = hipStreamEndCapture(r->streams[0], &graph);
    r->graph = graph;
    if (rc == FMBYM_OK && e_end != hipSuccess) rc = hip_fail(e_end);
    if (rc == FMBYM_OK) {
        e = hipGraphInstantiate(&r->exec, r->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    if (rc) {
        ragged_free(r);
        return rc;
    }
    *out = (fmbym_ragged)r;
    return FMBYM_OK;
}

size_t fmbym_search_ragged_workspace_size(const fmbym_plan* plans, int32_t n_plans, const fmbym_pair* pairs,
                                          int32_t n_pairs, const fmbym_mask_desc* net) {
    std::vector<Group> groups;
    std::vector<int> slots;
    size_t bytes = 0;
    if (plan_groups(plans, n_plans, pairs, n_pairs, net, groups, slots, &bytes)) return 0;
    return one_call_layout(bytes, 4 * (size_t)n_pairs + net_rows(groups), n_pairs).total;
}

int fmbym_search_ragged(const fmbym_plan* plans, int32_t n_plans, const fmbym_pair* pairs, int32_t n_pairs,
                        const fmbym_mask_desc* net, float* pose, uint64_t* stamps, void* workspace,
                        size_t workspace_bytes, void* stream) {
    const TraceRange trace_range("fmbym_search_ragged");
    std::vector<Group> groups;
    std::vector<int> slots;
    size_t bytes = 0;
    int rc = plan_groups(plans, n_plans, pairs, n_pairs, net, groups, slots, &bytes);
    if (rc) return rc;
    if (!pose) return FMBYM_EINVAL;
    const std::vector<const float*> tab_h = pointer_table(groups, slots, pairs, n_pairs, workspace);
    const OneCall L = one_call_layout(bytes, tab_h.size(), n_pairs);
    if (!workspace || workspace_bytes < L.total) return FMBYM_EWORKSPACE;
    char* ws = (char*)workspace;
    const float** tab = (const float**)(ws + L.tab_off);
    int* slot_pair = (int*)(ws + L.slot_off);
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* st = (unsigned long long*)stamps;
    // the tables go into the workspace in stream order (the host vectors may be
    // released once the copies return: pageable sources are staged by then)
    hipError_t e = hipMemcpyAsync(tab, tab_h.data(), sizeof(const float*) * tab_h.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(slot_pair, slots.data(), sizeof(int) * (size_t)n_pairs, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
    if (st) hipLaunchKernelGGL(k_ragged_start, dim3(1), dim3(64), 0, s, st, n_pairs);
    fmbym_mask_desc net_copy{};
    if (net) net_copy = *net;
    for (const Group& gr : groups) {
        float* pose_g = (float*)(ws + gr.pose_off);
        if (gr.kind == kNet) {
            rc = mask_forward(&net_copy, 2 * gr.count, gr.plan->p.n, nullptr,
                              tab + 4 * (size_t)n_pairs + gr.xtab_first, (float*)(ws + gr.mask_off),
                              ws + gr.act_off, gr.act_bytes, 0, s);
            if (rc) return rc;
        }
        rc = launch_forward(*gr.plan, gr.count, nullptr, nullptr, nullptr, nullptr, pose_g, nullptr, nullptr,
                            nullptr, ws + gr.ws_off, s, tab + 4 * (size_t)gr.first);
        if (rc) return rc;
        hipLaunchKernelGGL(k_ragged_poses, dim3((gr.count + 63) / 64), dim3(64), 0, s, pose_g,
                           slot_pair + gr.first, gr.count, pose, st);
    }
    e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

int fmbym_ragged_launch(fmbym_ragged rg, void* stream) {
    const TraceRange trace_range("fmbym_ragged_launch");
    if (!rg) return FMBYM_EINVAL;
    Ragged* r = reinterpret_cast<Ragged*>(rg);
    hipError_t e = hipGraphLaunch(r->exec, (hipStream_t)stream);
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

int fmbym_wall_clock_khz(int32_t* khz) {
    if (!khz) return FMBYM_EINVAL;
    int dev = 0, v = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return hip_fail(e);
    *khz = v;
    return FMBYM_OK;
}

int fmbym_ragged_destroy(fmbym_ragged rg) {
    if (!rg) return FMBYM_EINVAL;
    hipError_t e = ragged_free(reinterpret_cast<Ragged*>(rg));
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

}  // extern "C"
