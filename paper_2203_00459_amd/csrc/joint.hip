// Brute-force joint comparator of the decoupled search (Eq. 2-3 searched
// exhaustively over headings): for K candidate headings theta_k = -pi/2 +
// k pi / K, the stage-2 correlation of f_w with g_w rotated by theta_k on the
// translation stage's lag grid, J_k(s') = sum_x f_w(x) Rotate(g_w, theta_k)(x + s'),
// then the hard argmax over (k, s') with t = R(theta_k) s' delta.  The decoupled
// search replaces this K-fold work by one polar angular correlation (Eq. 8).
//
// Every (pair, heading) is a virtual pair of the stage-2 kernels: a pointer
// table presents f_b and g_b for each of them (no copies) and its saved slots
// carry cos/sin(theta_k).  Headings run in chunks so that the workspace stays
// bounded; each chunk's c_xy surfaces are reduced to their peak (value, first
// index) per virtual pair, and a last kernel takes the first best heading.
#include <math.h>

#include "internal.hpp"
#include "profile.hpp"

namespace fmbym {

namespace {

constexpr int kJointVirtual = 256;   // virtual pairs per chunk (bounds the workspace)

__global__ void k_joint_setup(const float* __restrict__ f, const float* __restrict__ g,
                              const float* __restrict__ mf, const float* __restrict__ mg, int n, int kc,
                              int k0, int n_angles, int nv, const float** __restrict__ tab,
                              float* __restrict__ saved) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int b = v / kc, k = k0 + v % kc;
    const size_t off = (size_t)b * n * n;
    tab[4 * v + 0] = f + off;
    tab[4 * v + 1] = g + off;
    tab[4 * v + 2] = mf ? mf + off : nullptr;
    tab[4 * v + 3] = mg ? mg + off : nullptr;
    const double th = -M_PI / 2 + (double)k * (M_PI / n_angles);
    float* sv = saved + (size_t)v * FMBYM_SAVED;
    sv[kSavedTheta] = (float)th;
    sv[kSavedCos] = (float)cos(th);
    sv[kSavedSin] = (float)sin(th);
}

// Peak of one virtual pair's c_xy: largest value, first flat index among equals.
__global__ __launch_bounds__(256) void k_joint_peak(const float* __restrict__ c_xy, int n2, int kc, int k0,
                                                    int n_angles, float* __restrict__ peak,
                                                    int* __restrict__ where) {
    __shared__ float sv[256];
    __shared__ int si[256];
    const int v = blockIdx.x;
    const float* c = c_xy + (size_t)v * n2;
    float best = -INFINITY;
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < n2; i += 256) {
        const float x = c[i];
        if (x > best) {   // increasing i within a thread: the first maximum is kept
            best = x;
            bi = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const float o = sv[threadIdx.x + w];
            const int oi = si[threadIdx.x + w];
            if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = o;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int b = v / kc, k = k0 + v % kc;
        peak[b * n_angles + k] = sv[0];
        where[b * n_angles + k] = si[0];
    }
}

// Per pair: the first heading with the largest peak -> pose.
__global__ void k_joint_pick(const float* __restrict__ peak, const int* __restrict__ where, int n_angles,
                             int n, float delta, float* __restrict__ pose, float* __restrict__ peak_out) {
    const int b = blockIdx.x;
    if (threadIdx.x != 0) return;
    const float* pk = peak + (size_t)b * n_angles;
    int kb = 0;
    for (int k = 1; k < n_angles; ++k)
        if (pk[k] > pk[kb]) kb = k;
    if (peak_out)
        for (int k = 0; k < n_angles; ++k) peak_out[(size_t)b * n_angles + k] = pk[k];
    const int idx = where[(size_t)b * n_angles + kb];
    const double th = -M_PI / 2 + (double)kb * (M_PI / n_angles);
    const float ct = (float)cos(th), st = (float)sin(th);
    const float tpx = (float)(idx % n - n / 2) * delta, tpy = (float)(idx / n - n / 2) * delta;
    pose[b * 3 + 0] = (float)th;
    pose[b * 3 + 1] = ct * tpx - st * tpy;
    pose[b * 3 + 2] = st * tpx + ct * tpy;
}

struct JointLayout {
    size_t stage2, tab, saved, cxy, peak, where, total;
    int kc, nv;
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

JointLayout joint_layout(const fmbym_params& p, int batch, int n_angles) {
    JointLayout L{};
    L.kc = kJointVirtual / batch;
    if (L.kc < 1) L.kc = 1;
    if (L.kc > n_angles) L.kc = n_angles;
    L.nv = batch * L.kc;
    const size_t n = p.n;
    size_t off = 0;
    L.stage2 = off;
    off = al256(off + fwd_layout(p, L.nv).total);
    L.tab = off;
    off = al256(off + (size_t)L.nv * 4 * sizeof(void*));
    L.saved = off;
    off = al256(off + (size_t)L.nv * FMBYM_SAVED * sizeof(float));
    L.cxy = off;
    off = al256(off + (size_t)L.nv * n * n * sizeof(float));
    L.peak = off;
    off = al256(off + (size_t)batch * n_angles * sizeof(float));
    L.where = off;
    off = al256(off + (size_t)batch * n_angles * sizeof(int));
    L.total = off;
    return L;
}

}  // namespace

size_t joint_workspace(const fmbym_params& p, int batch, int n_angles) {
    return joint_layout(p, batch, n_angles).total;
}

int launch_joint(const Plan& pl, int batch, int n_angles, const float* f, const float* g, const float* mf,
                 const float* mg, float* pose, float* peak_out, char* ws, hipStream_t s) {
    const JointLayout L = joint_layout(pl.p, batch, n_angles);
    const float** tab = (const float**)(ws + L.tab);
    float* saved = (float*)(ws + L.saved);
    float* cxy = (float*)(ws + L.cxy);
    float* peak = (float*)(ws + L.peak);
    int* where = (int*)(ws + L.where);
    const int n = pl.p.n;
    for (int k0 = 0; k0 < n_angles; k0 += L.kc) {
        const int kc = k0 + L.kc <= n_angles ? L.kc : n_angles - k0;
        const int nv = batch * kc;
        FMBYM_LAUNCH(kKJointSetup, k_joint_setup, dim3((nv + 63) / 64), dim3(64), s, f, g, mf, mg, n, kc, k0,
                     n_angles, nv, tab, saved);
        launch_stage2(pl, nv, nullptr, nullptr, nullptr, nullptr, saved, cxy, ws + L.stage2, s,
                      (const float* const*)tab);
        FMBYM_LAUNCH(kKJointPeak, k_joint_peak, dim3(nv), dim3(256), s, cxy, n * n, kc, k0, n_angles, peak,
                     where);
    }
    FMBYM_LAUNCH(kKJointPick, k_joint_pick, dim3(batch), dim3(64), s, peak, where, n_angles, n,
                 pl.p.delta_xy, pose, peak_out);
    return FMBYM_OK;
}

}  // namespace fmbym
