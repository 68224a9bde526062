// Autotuner of the column-tile widths (the plan's fmbym_tuning): times whole
// search steps on synthetic scans and keeps, pass by pass, the fastest width.
// The widths only group columns into blocks; each column's transform is the
// same arithmetic for every width, so tuning never changes a result.
#include "internal.hpp"
#include "profile.hpp"

namespace fmbym {

fmbym_tuning default_tuning(int n) {
    fmbym_tuning t;
    t.cols1 = n >= 512 ? 8 : 16;
    t.cols2 = n >= 512 ? 4 : (n >= 256 ? 8 : 16);
    t.cols_xy = n >= 512 ? 4 : (n >= 256 ? 8 : 16);
    t.cols_mag = n >= 512 ? 4 : 16;
    t.split = n >= 512 ? 2 : 1;
    t.rows1 = t.rows2 = 2;
    t.radix1 = t.radix_mag = 8;
    return t;
}

bool valid_tile(int c) { return c == 4 || c == 8 || c == 16; }

bool tuning_ok(const fmbym_tuning& t, int n) {
    if (!valid_tile(t.cols1) || !valid_tile(t.cols2) || !valid_tile(t.cols_xy) || !valid_tile(t.cols_mag))
        return false;
    if (t.split != 1 && t.split != 2) return false;
    if ((t.rows1 != 1 && t.rows1 != 2) || (t.rows2 != 1 && t.rows2 != 2)) return false;
    if ((t.radix1 != 8 && t.radix1 != 4) || (t.radix_mag != 8 && t.radix_mag != 4)) return false;
    return t.cols1 * n / t.radix1 <= 1024 && t.cols_mag * n / t.radix_mag <= 1024;
}

namespace {

// Each candidate: warm-up steps, then the fastest of kTuneReps timings of
// kTuneSteps steps (the minimum rejects interference from other work).
constexpr int kTuneWarmup = 2, kTuneSteps = 8, kTuneReps = 3;

// Uniform values in [0, 1) from a counter hash (splitmix-style mixing of the index).
__global__ void k_tune_fill(float* __restrict__ x, size_t count, unsigned seed, int ones) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    if (ones) {
        x[i] = 1.f;
        return;
    }
    unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ull + seed;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (float)(z >> 40) * (1.f / 16777216.f);
}

struct TuneLayout {
    size_t f, g, pose, cth, cxy, saved, dpose, df, dg, state, ws, total;
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

TuneLayout tune_layout(const Plan& pl, int B, int with_bwd) {
    const size_t n2 = (size_t)pl.p.n * pl.p.n;
    TuneLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = al(off + bytes);
        return at;
    };
    L.f = take(B * n2 * 4);
    L.g = take(B * n2 * 4);
    L.pose = take(B * 3 * 4);
    L.cth = take((size_t)B * pl.p.n_theta * 4);
    L.cxy = take(B * n2 * 4);
    L.saved = take((size_t)B * FMBYM_SAVED * 4);
    L.dpose = take(B * 3 * 4);
    L.df = with_bwd ? take(B * n2 * 4) : 0;
    L.dg = with_bwd ? take(B * n2 * 4) : 0;
    L.state = with_bwd ? take(keep_bytes(pl.p, B)) : 0;
    const size_t fw = run_fwd_workspace(pl, B), bw = with_bwd ? run_bwd_workspace(pl, B) : 0;
    L.ws = take(fw > bw ? fw : bw);
    L.total = off;
    return L;
}

}  // namespace
}  // namespace fmbym

using namespace fmbym;

extern "C" {

size_t fmbym_autotune_workspace_size(fmbym_plan plan, int32_t batch, int with_backward) {
    // odd sides have no tunable column tiles; the readings have no adjoint
    if (with_backward ? check_adjoint(plan, batch) : check_full_path(plan, batch)) return 0;
    return tune_layout(*plan_cast(plan), batch, with_backward ? 1 : 0).total;
}

int fmbym_autotune(fmbym_plan plan, int32_t batch, int with_backward, void* workspace, size_t workspace_bytes,
                   void* stream, fmbym_tuning* best, float* ms_per_step) {
    int rc = with_backward ? check_adjoint(plan, batch) : check_full_path(plan, batch);
    if (rc) return rc;
    if (!best) return FMBYM_EINVAL;
    Plan& pl = *plan_cast(plan);
    const int bwd = with_backward ? 1 : 0;
    const TuneLayout L = tune_layout(pl, batch, bwd);
    if (!workspace || workspace_bytes < L.total) return FMBYM_EWORKSPACE;
    char* w = (char*)workspace;
    hipStream_t s = (hipStream_t)stream;
    ProfilePause pause;   // tuning launches are not part of a profile
    const size_t n2 = (size_t)pl.p.n * pl.p.n, cnt = batch * n2;
    hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, (float*)(w + L.f), cnt,
                       1u, 0);
    hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, (float*)(w + L.g), cnt,
                       2u, 0);
    hipLaunchKernelGGL(k_tune_fill, dim3(1), dim3(256), 0, s, (float*)(w + L.dpose), (size_t)batch * 3, 0u, 1);
    const Keep keep = bwd ? keep_pointers(pl.p, batch, w + L.state) : Keep{};
    auto step = [&]() -> int {
        int r = run_forward(pl, batch, (float*)(w + L.f), (float*)(w + L.g), nullptr, nullptr,
                            (float*)(w + L.pose), (float*)(w + L.cth), (float*)(w + L.cxy),
                            (float*)(w + L.saved), w + L.ws, s, bwd ? &keep : nullptr);
        if (r || !bwd) return r;
        return run_backward(pl, batch, (float*)(w + L.f), (float*)(w + L.g), nullptr, nullptr,
                            (float*)(w + L.pose), (float*)(w + L.cth), (float*)(w + L.cxy),
                            (float*)(w + L.saved), (float*)(w + L.dpose), (float*)(w + L.df),
                            (float*)(w + L.dg), nullptr, nullptr, w + L.ws, s, &keep);
    };
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e);
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(e);
    }
    auto timed = [&](float* ms) -> int {
        for (int i = 0; i < kTuneWarmup; ++i)
            if (int r = step()) return r;
        for (int rep = 0; rep < kTuneReps; ++rep) {
            hipEventRecord(e0, s);
            for (int i = 0; i < kTuneSteps; ++i)
                if (int r = step()) return r;
            hipEventRecord(e1, s);
            float t = 0.f;
            hipError_t he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
            if (he != hipSuccess) return hip_fail(he);
            t /= kTuneSteps;
            if (rep == 0 || t < *ms) *ms = t;
        }
        return FMBYM_OK;
    };
    const fmbym_tuning start = pl.tune;
    // knobs in order; the adjoint's (cols_xy, cols_mag, radix_mag) only when it is timed
    struct Knob {
        int32_t* v;
        const int* cand;
        int ncand;
        bool bwd_only;
    };
    const int widths[3] = {4, 8, 16}, pair12[2] = {1, 2}, radices[2] = {8, 4};
    const Knob knobs[] = {
        {&pl.tune.split, pair12, batch >= 2 ? 2 : 1, false}, {&pl.tune.cols1, widths, 3, false},
        {&pl.tune.cols2, widths, 3, false},                  {&pl.tune.cols_xy, widths, 3, true},
        {&pl.tune.cols_mag, widths, 3, true},                {&pl.tune.rows1, pair12, 2, false},
        {&pl.tune.rows2, pair12, 2, false},                  {&pl.tune.radix1, radices, 2, false},
        {&pl.tune.radix_mag, radices, 2, true},
    };
    float best_ms = 0.f;
    rc = timed(&best_ms);
    for (const Knob& k : knobs) {
        if (rc != FMBYM_OK) break;
        if (k.bwd_only && !bwd) continue;
        int keep_w = *k.v;
        for (int ci = 0; ci < k.ncand; ++ci) {
            const int c = k.cand[ci];
            if (c == keep_w) continue;
            *k.v = c;
            if (!tuning_ok(pl.tune, pl.p.n)) continue;   // a block beyond 1024 threads
            float ms = 0.f;
            rc = timed(&ms);
            if (rc) break;
            if (ms < best_ms) {
                best_ms = ms;
                keep_w = c;
            }
        }
        *k.v = keep_w;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) {
        pl.tune = start;
        return rc;
    }
    *best = pl.tune;
    if (ms_per_step) *ms_per_step = best_ms;
    return FMBYM_OK;
}

}  // extern "C"
