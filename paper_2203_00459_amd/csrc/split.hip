// The batch split of a plan's search calls: two halves of the batch run
// concurrently, the first on the caller's stream, the second on the plan's
// auxiliary stream, forked from and joined back into the caller's stream by
// events (so a graph capture of the caller's stream captures both).  Each
// half is an ordinary search of its pairs with its own workspace region; the
// tails of one half's kernels overlap the other half's work.
#include "internal.hpp"

namespace fmbym {

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Halves {
    int n;          // 1 or 2
    int b0[2], nb[2];
};

Halves halves(const Plan& pl, int batch) {
    Halves h{};
    if (pl.tune.split == 2 && batch >= 2) {
        h.n = 2;
        h.nb[0] = (batch + 1) / 2;
        h.nb[1] = batch - h.nb[0];
        h.b0[0] = 0;
        h.b0[1] = h.nb[0];
    } else {
        h.n = 1;
        h.nb[0] = batch;
    }
    return h;
}

size_t fwd_ws(const fmbym_params& p, int b) { return fwd_layout(p, b).total; }
size_t bwd_ws(const fmbym_params& p, int b) {
    const size_t f = fwd_ws(p, b), w = bwd_workspace(p, b);
    return f > w ? f : w;
}

// Workspace that both the whole batch and its two halves fit in.
template <class Size>
size_t both(const Plan& pl, int batch, Size size) {
    const size_t whole = size(pl.p, batch);
    if (batch < 2) return whole;
    const int a = (batch + 1) / 2, b = batch - a;
    const size_t split = al256(size(pl.p, a)) + size(pl.p, b);
    return whole > split ? whole : split;
}

template <class Launch>
int run_halves(const Plan& pl, int batch, hipStream_t s, size_t (*size)(const fmbym_params&, int), Launch launch) {
    const Halves h = halves(pl, batch);
    if (h.n == 1) return launch(0, batch, s, (size_t)0);
    hipError_t e = hipEventRecord(pl.fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(pl.aux, pl.fork, 0);
    if (e != hipSuccess) return hip_fail(e);
    int rc = launch(h.b0[0], h.nb[0], s, (size_t)0);
    if (rc == FMBYM_OK) rc = launch(h.b0[1], h.nb[1], pl.aux, al256(size(pl.p, h.nb[0])));
    // join even after an error, so the caller's stream never runs ahead of work on aux
    e = hipEventRecord(pl.join, pl.aux);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, pl.join, 0);
    if (rc) return rc;
    return e == hipSuccess ? FMBYM_OK : hip_fail(e);
}

template <class T>
T* at_pair(T* x, int b0, size_t per_pair) { return x ? x + (size_t)b0 * per_pair : nullptr; }

}  // namespace

size_t run_fwd_workspace(const Plan& pl, int batch) { return both(pl, batch, fwd_ws); }
size_t run_full_circle_workspace(const Plan& pl, int batch) {
    return both(pl, batch, full_circle_workspace);
}
size_t run_bwd_workspace(const Plan& pl, int batch) { return both(pl, batch, bwd_ws); }

int run_forward(const Plan& pl, int batch, const float* f, const float* g, const float* mf, const float* mg,
                float* pose, float* c_theta, float* c_xy, float* saved, char* ws, hipStream_t s,
                const Keep* keep_full) {
    const size_t n2 = (size_t)pl.p.n * pl.p.n;
    return run_halves(pl, batch, s, fwd_ws, [&](int b0, int nb, hipStream_t st, size_t off) {
        Keep k{};
        if (keep_full) k = keep_slice(*keep_full, pl.p, b0);
        return launch_forward(pl, nb, at_pair(f, b0, n2), at_pair(g, b0, n2), at_pair(mf, b0, n2),
                              at_pair(mg, b0, n2), at_pair(pose, b0, 3), at_pair(c_theta, b0, pl.p.n_theta),
                              at_pair(c_xy, b0, n2), at_pair(saved, b0, FMBYM_SAVED), ws + off, st, nullptr,
                              keep_full ? &k : nullptr);
    });
}

int run_full_circle(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                    const float* mg, float* pose, float* peaks, char* ws, hipStream_t s) {
    const size_t n2 = (size_t)pl.p.n * pl.p.n;
    return run_halves(pl, batch, s, full_circle_workspace, [&](int b0, int nb, hipStream_t st, size_t off) {
        return launch_full_circle(pl, nb, at_pair(f, b0, n2), at_pair(g, b0, n2), at_pair(mf, b0, n2),
                                  at_pair(mg, b0, n2), at_pair(pose, b0, 3), at_pair(peaks, b0, 2), ws + off,
                                  st);
    });
}

int run_backward(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                 const float* mg, const float* pose, const float* c_theta, const float* c_xy,
                 const float* saved, const float* d_pose, float* d_f, float* d_g, float* d_mf, float* d_mg,
                 char* ws, hipStream_t s, const Keep* keep_full) {
    const size_t n2 = (size_t)pl.p.n * pl.p.n;
    return run_halves(pl, batch, s, bwd_ws, [&](int b0, int nb, hipStream_t st, size_t off) {
        Keep k{};
        if (keep_full) k = keep_slice(*keep_full, pl.p, b0);
        return launch_backward(pl, nb, at_pair(f, b0, n2), at_pair(g, b0, n2), at_pair(mf, b0, n2),
                               at_pair(mg, b0, n2), at_pair(pose, b0, 3), at_pair(c_theta, b0, pl.p.n_theta),
                               at_pair(c_xy, b0, n2), at_pair(saved, b0, FMBYM_SAVED), at_pair(d_pose, b0, 3),
                               at_pair(d_f, b0, n2), at_pair(d_g, b0, n2), at_pair(d_mf, b0, n2),
                               at_pair(d_mg, b0, n2), ws + off, st, keep_full ? &k : nullptr);
    });
}

int run_vjp(const Plan& pl, int batch, const float* f, const float* g, const float* mf, const float* mg,
            float* pose, float* c_theta, float* c_xy, float* saved, const float* d_pose, float* d_f,
            float* d_g, float* d_mf, float* d_mg, char* ws, hipStream_t s, const Keep& keep_full) {
    const size_t n2 = (size_t)pl.p.n * pl.p.n;
    // a half's adjoint follows its own forward on its stream: the region sized
    // for the adjoint holds the forward's workspace too
    return run_halves(pl, batch, s, bwd_ws, [&](int b0, int nb, hipStream_t st, size_t off) {
        const Keep k = keep_slice(keep_full, pl.p, b0);
        int rc = launch_forward(pl, nb, at_pair(f, b0, n2), at_pair(g, b0, n2), at_pair(mf, b0, n2),
                                at_pair(mg, b0, n2), at_pair(pose, b0, 3), at_pair(c_theta, b0, pl.p.n_theta),
                                at_pair(c_xy, b0, n2), at_pair(saved, b0, FMBYM_SAVED), ws + off, st, nullptr,
                                &k);
        if (rc) return rc;
        return launch_backward(pl, nb, at_pair(f, b0, n2), at_pair(g, b0, n2), at_pair(mf, b0, n2),
                               at_pair(mg, b0, n2), at_pair(pose, b0, 3), at_pair(c_theta, b0, pl.p.n_theta),
                               at_pair(c_xy, b0, n2), at_pair(saved, b0, FMBYM_SAVED), at_pair(d_pose, b0, 3),
                               at_pair(d_f, b0, n2), at_pair(d_g, b0, n2), at_pair(d_mf, b0, n2),
                               at_pair(d_mg, b0, n2), ws + off, st, &k);
    });
}

}  // namespace fmbym
