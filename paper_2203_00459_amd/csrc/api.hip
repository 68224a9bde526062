// C ABI of the search: plan construction, host-side validation, workspace
// sizing and dispatch to the kernel launchers.  No call here throws; every
// argument is checked before anything is enqueued.
#include <math.h>
#include <new>

#include "internal.hpp"
#include "profile.hpp"

using namespace fmbym;

namespace fmbym {

namespace {
thread_local int g_last_hip = 0;
}

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return FMBYM_EHIP;
}

int check_call(fmbym_plan plan, int32_t batch) {
    if (!plan) return FMBYM_EINVAL;
    if (batch < 1 || batch > plan_cast(plan)->max_batch) return FMBYM_EINVAL;
    return FMBYM_OK;
}

int check_full_path(fmbym_plan plan, int32_t batch) {
    const int rc = check_call(plan, batch);
    if (rc) return rc;
    return odd_side(plan_cast(plan)->p.n) ? FMBYM_EUNSUPPORTED : FMBYM_OK;
}

int check_adjoint(fmbym_plan plan, int32_t batch) {
    const int rc = check_full_path(plan, batch);
    if (rc) return rc;
    return (plan_cast(plan)->p.flags & kReadingFlags) ? FMBYM_EUNSUPPORTED : FMBYM_OK;
}

}  // namespace fmbym

namespace {

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int check_params(const fmbym_params* p) {
    if (!p) return FMBYM_EINVAL;
    if (!(p->delta_xy > 0.f) || !isfinite(p->delta_xy)) return FMBYM_EINVAL;
    if (!(p->temp_theta > 0.f) || !isfinite(p->temp_theta)) return FMBYM_EINVAL;
    if (!(p->temp_xy > 0.f) || !isfinite(p->temp_xy)) return FMBYM_EINVAL;
    if (!isfinite(p->band_lo) || !isfinite(p->band_hi)) return FMBYM_EINVAL;
    if (p->band_hi > 0.f && (p->band_lo < 0.f || p->band_lo > p->band_hi)) return FMBYM_EINVAL;
    if (p->n <= 0 || p->n_theta <= 0 || p->n_r <= 0) return FMBYM_EINVAL;
    if (p->flags & ~(uint32_t)(FMBYM_HANN | FMBYM_XY_UNWINDOWED | FMBYM_CHECK_FINITE | kReadingFlags))
        return FMBYM_EUNSUPPORTED;
    if (p->n_r > 4096) return FMBYM_EUNSUPPORTED;
    if (odd_side(p->n)) {   // forward only; any number of heading bins
        if (p->n_theta < 16 || p->n_theta > 1024) return FMBYM_EUNSUPPORTED;
        if (p->flags & (FMBYM_CHECK_FINITE | kReadingFlags)) return FMBYM_EUNSUPPORTED;
        return FMBYM_OK;
    }
    if (p->n != 128 && p->n != 256 && p->n != 512) return FMBYM_EUNSUPPORTED;
    if (!pow2(p->n_theta) || p->n_theta < 16 || p->n_theta > 1024) return FMBYM_EUNSUPPORTED;
    return FMBYM_OK;
}

// Tables of the odd-side path: the Bluestein chirp c_j = exp(i pi (j^2 mod 2n) / n),
// the spectrum of its wrapped filter divided by the line length (a direct DFT in
// FP64 with the phase reduced modulo the length), and the polar angles.
hipError_t odd_tables(Plan& pl) {
    const int n = pl.p.n, M = odd_m1(n), nt = pl.p.n_theta;
    float2* chirp = new (std::nothrow) float2[n];
    float2* bspec = new (std::nothrow) float2[M];
    float2* cs = new (std::nothrow) float2[nt];
    double* wre = new (std::nothrow) double[2 * M];
    double* b = new (std::nothrow) double[2 * M];
    hipError_t e = hipSuccess;
    if (!chirp || !bspec || !cs || !wre || !b) {
        e = hipErrorOutOfMemory;
    } else {
        for (int j = 0; j < n; ++j) {
            const long long q = ((long long)j * j) % (2LL * n);
            const double a = M_PI * (double)q / n;
            chirp[j] = make_float2((float)cos(a), (float)sin(a));
        }
        for (int m = 0; m < 2 * M; ++m) b[m] = 0.0;
        for (int m = 0; m < n; ++m) {
            const long long q = ((long long)m * m) % (2LL * n);
            const double a = M_PI * (double)q / n;
            b[2 * m] = cos(a);
            b[2 * m + 1] = sin(a);
            if (m > 0) {
                b[2 * (M - m)] = cos(a);
                b[2 * (M - m) + 1] = sin(a);
            }
        }
        for (int m = 0; m < M; ++m) {   // W_M^m
            const double a = -2.0 * M_PI * (double)m / M;
            wre[2 * m] = cos(a);
            wre[2 * m + 1] = sin(a);
        }
        for (int k = 0; k < M; ++k) {
            double sr = 0.0, si = 0.0;
            for (int m = 0; m < M; ++m) {
                const long long q = ((long long)k * m) % M;
                const double cr = wre[2 * q], ci = wre[2 * q + 1];
                sr += b[2 * m] * cr - b[2 * m + 1] * ci;
                si += b[2 * m] * ci + b[2 * m + 1] * cr;
            }
            bspec[k] = make_float2((float)(sr / M), (float)(si / M));
        }
        for (int a = 0; a < nt; ++a) {
            const double phi = M_PI * (double)a / nt;
            cs[a] = make_float2((float)cos(phi), (float)sin(phi));
        }
        e = hipMalloc((void**)&pl.chirp, sizeof(float2) * n);
        if (e == hipSuccess) e = hipMalloc((void**)&pl.bspec, sizeof(float2) * M);
        if (e == hipSuccess) e = hipMalloc((void**)&pl.polar_cs, sizeof(float2) * nt);
        if (e == hipSuccess) e = hipMemcpy(pl.chirp, chirp, sizeof(float2) * n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl.bspec, bspec, sizeof(float2) * M, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(pl.polar_cs, cs, sizeof(float2) * nt, hipMemcpyHostToDevice);
    }
    delete[] chirp;
    delete[] bspec;
    delete[] cs;
    delete[] wre;
    delete[] b;
    return e;
}

hipError_t free_plan_tables(Plan* pl) {
    hipError_t first = hipSuccess;
    if (pl->join) first = hipEventDestroy(pl->join);
    if (pl->fork) {
        hipError_t e = hipEventDestroy(pl->fork);
        if (first == hipSuccess) first = e;
    }
    if (pl->aux) {
        hipError_t e = hipStreamDestroy(pl->aux);
        if (first == hipSuccess) first = e;
    }
    void* ptrs[] = {pl->twiddle, pl->twiddle3, pl->hann,     pl->csr_ptr, pl->csr_col, pl->csr_val,
                    pl->csr_dst, pl->dmag_part, pl->chirp, pl->bspec, pl->polar_cs};
    for (void* q : ptrs) {
        if (!q) continue;
        hipError_t e = hipFree(q);
        if (first == hipSuccess) first = e;
    }
    return first;
}

}  // namespace

extern "C" {

int fmbym_plan_create(const fmbym_params* p, int32_t max_batch, fmbym_plan* out) {
    if (!out) return FMBYM_EINVAL;
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    if (max_batch < 1 || max_batch > (1 << 20)) return FMBYM_EINVAL;
    Plan* pl = new (std::nothrow) Plan();
    if (!pl) return FMBYM_EINVAL;
    pl->p = *p;
    pl->max_batch = max_batch;
    pl->tune = default_tuning(p->n);
    hipError_t e = hipGetDevice(&pl->device);
    if (e != hipSuccess) {
        delete pl;
        return hip_fail(e);
    }
    float2 tw[kTwiddleLen], tw3[kTwiddleLen3];
    for (int m = 0; m < kTwiddleLen; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)kTwiddleLen;
        tw[m] = make_float2((float)cos(a), (float)sin(a));
    }
    for (int m = 0; m < kTwiddleLen3; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)kTwiddleLen3;
        tw3[m] = make_float2((float)cos(a), (float)sin(a));
    }
    float* hann = new (std::nothrow) float[p->n];
    if (!hann) {
        delete pl;
        return FMBYM_EINVAL;
    }
    // the periodic Hann; at odd sides the same window written about the origin
    // pixel (n - 1)/2, which keeps it symmetric about the sensor
    for (int k = 0; k < p->n; ++k)
        hann[k] = (p->n & 1) ? (float)(0.5 * (1.0 + cos(2.0 * M_PI * (k - p->n / 2) / p->n)))
                             : (float)(0.5 * (1.0 - cos(2.0 * M_PI * k / p->n)));
    pl->band_on = p->band_hi > 0.f ? 1 : 0;
    if (pl->band_on) {
        const double lo = (double)p->band_lo * p->n, hi = (double)p->band_hi * p->n;
        pl->band_lo2 = (int)ceil(lo * lo);
        pl->band_hi2 = (int)floor(hi * hi);
    }
    e = hipMalloc((void**)&pl->twiddle, sizeof(tw));
    if (e == hipSuccess) e = hipMalloc((void**)&pl->twiddle3, sizeof(tw3));
    if (e == hipSuccess) e = hipMemcpy(pl->twiddle3, tw3, sizeof(tw3), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->hann, sizeof(float) * p->n);
    if (e == hipSuccess) e = hipMemcpy(pl->twiddle, tw, sizeof(tw), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pl->hann, hann, sizeof(float) * p->n, hipMemcpyHostToDevice);
    delete[] hann;
    if (e == hipSuccess) e = odd_side(p->n) ? (hipError_t)odd_tables(*pl) : (hipError_t)build_polar_csr(*pl);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_plan_tables(pl);
        delete pl;
        return hip_fail(e);
    }
    *out = (fmbym_plan)pl;
    return FMBYM_OK;
}

int fmbym_plan_destroy(fmbym_plan plan) {
    if (!plan) return FMBYM_EINVAL;
    Plan* pl = plan_cast(plan);
    hipError_t e = free_plan_tables(pl);
    delete pl;
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

size_t fmbym_search_workspace_size(fmbym_plan plan, int32_t batch, int with_backward) {
    if (check_call(plan, batch)) return 0;
    if (with_backward && check_adjoint(plan, batch)) return 0;   // odd sides and the readings: forward only
    const Plan* pl = plan_cast(plan);
    const size_t fwd = run_fwd_workspace(*pl, batch);
    if (!with_backward) return fwd;
    const size_t bwd = run_bwd_workspace(*pl, batch);
    return bwd > fwd ? bwd : fwd;
}

int fmbym_search(fmbym_plan plan, int32_t batch, const float* f, const float* g, const float* m_f,
                 const float* m_g, float* pose, float* c_theta, float* c_xy, float* saved,
                 void* workspace, size_t workspace_bytes, void* stream) {
    const TraceRange trace_range("fmbym_search");
    int rc = check_call(plan, batch);
    if (rc) return rc;
    if (!f || !g || !pose) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (m_g == nullptr)) return FMBYM_EINVAL;
    const Plan* pl = plan_cast(plan);
    if (!workspace || workspace_bytes < run_fwd_workspace(*pl, batch)) return FMBYM_EWORKSPACE;
    rc = run_forward(*pl, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, (char*)workspace,
                     (hipStream_t)stream, nullptr);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

int fmbym_search_backward(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                          const float* m_f, const float* m_g, const float* pose,
                          const float* c_theta, const float* c_xy, const float* saved,
                          const float* d_pose, float* d_f, float* d_g, float* d_m_f, float* d_m_g,
                          void* workspace, size_t workspace_bytes, void* stream) {
    const TraceRange trace_range("fmbym_search_backward");
    int rc = check_adjoint(plan, batch);
    if (rc) return rc;
    if (!f || !g || !pose || !c_theta || !c_xy || !saved || !d_pose || !d_f || !d_g)
        return FMBYM_EINVAL;
    if ((m_f == nullptr) != (m_g == nullptr)) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (d_m_f == nullptr) || (m_g == nullptr) != (d_m_g == nullptr))
        return FMBYM_EINVAL;
    const Plan* pl = plan_cast(plan);
    if (!workspace || workspace_bytes < run_bwd_workspace(*pl, batch)) return FMBYM_EWORKSPACE;
    rc = run_backward(*pl, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, d_pose, d_f, d_g, d_m_f,
                      d_m_g, (char*)workspace, (hipStream_t)stream, nullptr);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

int fmbym_plan_get_tuning(fmbym_plan plan, fmbym_tuning* out) {
    if (!plan || !out) return FMBYM_EINVAL;
    *out = plan_cast(plan)->tune;
    return FMBYM_OK;
}

int fmbym_plan_set_tuning(fmbym_plan plan, const fmbym_tuning* t) {
    if (!plan || !t) return FMBYM_EINVAL;
    if (!tuning_ok(*t, plan_cast(plan)->p.n)) return FMBYM_EINVAL;
    plan_cast(plan)->tune = *t;
    return FMBYM_OK;
}

size_t fmbym_joint_workspace_size(fmbym_plan plan, int32_t batch, int32_t n_angles) {
    if (check_full_path(plan, batch) || n_angles < 1 || n_angles > 4096) return 0;
    return joint_workspace(plan_cast(plan)->p, batch, n_angles);
}

int fmbym_search_joint(fmbym_plan plan, int32_t batch, int32_t n_angles, const float* f, const float* g,
                       const float* m_f, const float* m_g, float* pose, float* peak, void* workspace,
                       size_t workspace_bytes, void* stream) {
    const TraceRange trace_range("fmbym_search_joint");
    int rc = check_full_path(plan, batch);
    if (rc) return rc;
    if (n_angles < 1 || n_angles > 4096 || !f || !g || !pose) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (m_g == nullptr)) return FMBYM_EINVAL;
    const Plan* pl = plan_cast(plan);
    if (!workspace || workspace_bytes < joint_workspace(pl->p, batch, n_angles)) return FMBYM_EWORKSPACE;
    rc = launch_joint(*pl, batch, n_angles, f, g, m_f, m_g, pose, peak, (char*)workspace,
                      (hipStream_t)stream);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

size_t fmbym_full_circle_workspace_size(fmbym_plan plan, int32_t batch) {
    if (check_full_path(plan, batch)) return 0;
    return run_full_circle_workspace(*plan_cast(plan), batch);
}

int fmbym_search_full_circle(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                             const float* m_f, const float* m_g, float* pose, float* peaks, void* workspace,
                             size_t workspace_bytes, void* stream) {
    const TraceRange trace_range("fmbym_search_full_circle");
    int rc = check_full_path(plan, batch);
    if (rc) return rc;
    if (plan_cast(plan)->p.flags & (FMBYM_LOGIT_ZSCORE | FMBYM_HARD_ARGMAX)) return FMBYM_EUNSUPPORTED;
    if (!f || !g || !pose) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (m_g == nullptr)) return FMBYM_EINVAL;
    const Plan* pl = plan_cast(plan);
    if (!workspace || workspace_bytes < run_full_circle_workspace(*pl, batch)) return FMBYM_EWORKSPACE;
    rc = run_full_circle(*pl, batch, f, g, m_f, m_g, pose, peaks, (char*)workspace, (hipStream_t)stream);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

size_t fmbym_search_state_size(fmbym_plan plan, int32_t batch) {
    if (check_adjoint(plan, batch)) return 0;
    return keep_bytes(plan_cast(plan)->p, batch);
}

int fmbym_search_train(fmbym_plan plan, int32_t batch, const float* f, const float* g, const float* m_f,
                       const float* m_g, float* pose, float* c_theta, float* c_xy, float* saved,
                       void* state, size_t state_bytes, void* workspace, size_t workspace_bytes,
                       void* stream) {
    const TraceRange trace_range("fmbym_search_train");
    int rc = check_adjoint(plan, batch);
    if (rc) return rc;
    if (!f || !g || !pose || !c_theta || !c_xy || !saved) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (m_g == nullptr)) return FMBYM_EINVAL;
    const Plan* pl = plan_cast(plan);
    if (!state || state_bytes < keep_bytes(pl->p, batch)) return FMBYM_EWORKSPACE;
    if (!workspace || workspace_bytes < run_fwd_workspace(*pl, batch)) return FMBYM_EWORKSPACE;
    const Keep keep = keep_pointers(pl->p, batch, state);
    rc = run_forward(*pl, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, (char*)workspace,
                     (hipStream_t)stream, &keep);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

int fmbym_search_backward_state(fmbym_plan plan, int32_t batch, const float* f, const float* g,
                                const float* m_f, const float* m_g, const float* pose,
                                const float* c_theta, const float* c_xy, const float* saved,
                                const void* state, size_t state_bytes, const float* d_pose, float* d_f,
                                float* d_g, float* d_m_f, float* d_m_g, void* workspace,
                                size_t workspace_bytes, void* stream) {
    const TraceRange trace_range("fmbym_search_backward_state");
    int rc = check_adjoint(plan, batch);
    if (rc) return rc;
    if (!f || !g || !pose || !c_theta || !c_xy || !saved || !d_pose || !d_f || !d_g)
        return FMBYM_EINVAL;
    if ((m_f == nullptr) != (m_g == nullptr)) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (d_m_f == nullptr) || (m_g == nullptr) != (d_m_g == nullptr))
        return FMBYM_EINVAL;
    const Plan* pl = plan_cast(plan);
    if (!state || state_bytes < keep_bytes(pl->p, batch)) return FMBYM_EWORKSPACE;
    if (!workspace || workspace_bytes < run_bwd_workspace(*pl, batch)) return FMBYM_EWORKSPACE;
    const Keep keep = keep_pointers(pl->p, batch, (void*)state);
    rc = run_backward(*pl, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, d_pose, d_f, d_g, d_m_f,
                      d_m_g, (char*)workspace, (hipStream_t)stream, &keep);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

int fmbym_search_vjp(fmbym_plan plan, int32_t batch, const float* f, const float* g, const float* m_f,
                     const float* m_g, float* pose, float* c_theta, float* c_xy, float* saved, void* state,
                     size_t state_bytes, const float* d_pose, float* d_f, float* d_g, float* d_m_f,
                     float* d_m_g, void* workspace, size_t workspace_bytes, void* stream) {
    const TraceRange trace_range("fmbym_search_vjp");
    int rc = check_adjoint(plan, batch);
    if (rc) return rc;
    if (!f || !g || !pose || !c_theta || !c_xy || !saved || !d_pose || !d_f || !d_g) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (m_g == nullptr)) return FMBYM_EINVAL;
    if ((m_f == nullptr) != (d_m_f == nullptr) || (m_g == nullptr) != (d_m_g == nullptr))
        return FMBYM_EINVAL;
    const Plan* pl = plan_cast(plan);
    if (!state || state_bytes < keep_bytes(pl->p, batch)) return FMBYM_EWORKSPACE;
    if (!workspace || workspace_bytes < run_bwd_workspace(*pl, batch)) return FMBYM_EWORKSPACE;
    const Keep keep = keep_pointers(pl->p, batch, state);
    rc = run_vjp(*pl, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, d_pose, d_f, d_g, d_m_f, d_m_g,
                 (char*)workspace, (hipStream_t)stream, keep);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

const char* fmbym_strerror(int code) {
    switch (code) {
        case FMBYM_OK: return "success";
        case FMBYM_EINVAL: return "invalid argument";
        case FMBYM_EUNSUPPORTED: return "unsupported size or flag";
        case FMBYM_EWORKSPACE: return "workspace missing or too small";
        case FMBYM_EHIP: return "HIP runtime error";
        default: return "unknown error code";
    }
}

int fmbym_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
