// Full-circle heading, for the metric localisation with arbitrary rotational
// offset that the paper's Conclusion proposes.  Stage 1 correlates magnitude
// spectra, which are point symmetric for real scans (|F(-k)| = |F(k)|, the
// property behind Eq. 5-6), so it fixes the heading modulo pi.  theta and
// theta + pi rotate g differently, so stage 2 (Eq. 9) tells them apart: the
// forward search runs as usual, stage 2 runs again at theta + pi (wrapped to
// [-pi, pi)), and each pair keeps the heading whose correlation surface has
// the larger peak, max over lags of c_xy (the stage-1 heading on ties).
//
// R(theta + pi) = -R(theta), so the second run's cos/sin are the negated
// values the first run used (no new rounding), and its translation is the
// soft-argmax of its own surface with t = R(theta + pi) t'.
#include <math.h>

#include "internal.hpp"
#include "profile.hpp"

namespace fmbym {

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of one call: the forward's layout (reused by the second stage-2
// run once the forward is done), then per pair the two saved records and the
// turned pose.
struct TurnLayout {
    size_t saved1, saved2, pose2, total;
};

TurnLayout turn_layout(const fmbym_params& p, int batch) {
    TurnLayout L{};
    size_t off = al256(fwd_layout(p, batch).total);
    L.saved1 = off;
    off = al256(off + (size_t)batch * FMBYM_SAVED * sizeof(float));
    L.saved2 = off;
    off = al256(off + (size_t)batch * FMBYM_SAVED * sizeof(float));
    L.pose2 = off;
    off = al256(off + (size_t)batch * 3 * sizeof(float));
    L.total = off;
    return L;
}

// saved2[b] = saved1[b] turned by pi: heading wrapped to [-pi, pi), cos and
// sin negated; pose2[b][0] = that heading.
__global__ void k_turn_setup(const float* __restrict__ saved1, float* __restrict__ saved2,
                             float* __restrict__ pose2, int batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const float* a = saved1 + (size_t)b * FMBYM_SAVED;
    float* c = saved2 + (size_t)b * FMBYM_SAVED;
#pragma unroll
    for (int i = 0; i < FMBYM_SAVED; ++i) c[i] = a[i];
    const double th = a[kSavedTheta];
    const float alt = (float)(th < 0.0 ? th + M_PI : th - M_PI);
    c[kSavedTheta] = alt;
    c[kSavedCos] = -a[kSavedCos];
    c[kSavedSin] = -a[kSavedSin];
    pose2[b * 3 + 0] = alt;
}

// Per pair: the turned pose where its peak is strictly larger; both peaks out.
__global__ void k_turn_pick(const float* __restrict__ saved1, const float* __restrict__ saved2,
                            const float* __restrict__ pose2, float* __restrict__ pose,
                            float* __restrict__ peaks, int batch) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const float p1 = saved1[(size_t)b * FMBYM_SAVED + kSavedXyMax];
    const float p2 = saved2[(size_t)b * FMBYM_SAVED + kSavedXyMax];
    if (peaks) {
        peaks[2 * b + 0] = p1;
        peaks[2 * b + 1] = p2;
    }
    if (p2 > p1) {
#pragma unroll
        for (int i = 0; i < 3; ++i) pose[3 * b + i] = pose2[3 * b + i];
    }
}

}  // namespace

size_t full_circle_workspace(const fmbym_params& p, int batch) { return turn_layout(p, batch).total; }

int launch_full_circle(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                       const float* mg, float* pose, float* peaks, char* ws, hipStream_t s) {
    const TurnLayout L = turn_layout(pl.p, batch);
    float* saved1 = (float*)(ws + L.saved1);
    float* saved2 = (float*)(ws + L.saved2);
    float* pose2 = (float*)(ws + L.pose2);
    int rc = launch_forward(pl, batch, f, g, mf, mg, pose, nullptr, nullptr, saved1, ws, s);
    if (rc) return rc;
    const int blocks = (batch + 63) / 64;
    FMBYM_LAUNCH(kKTurnSetup, k_turn_setup, dim3(blocks), dim3(64), s, saved1, saved2, pose2, batch);
    launch_stage2(pl, batch, f, g, mf, mg, saved2, nullptr, ws, s, nullptr);
    launch_xy_fin(pl, batch, ws, pose2, saved2, s);
    FMBYM_LAUNCH(kKTurnPick, k_turn_pick, dim3(blocks), dim3(64), s, saved1, saved2, pose2, pose, peaks,
                 batch);
    return FMBYM_OK;
}

}  // namespace fmbym
