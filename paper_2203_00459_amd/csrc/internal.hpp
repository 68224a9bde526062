// Internal declarations shared by the search's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fmbym.h"
#include "fft_core.hpp"

namespace fmbym {

// Per-pair statistics kept in `saved` (FMBYM_SAVED floats).
enum SavedSlot {
    kSavedTheta = FMBYM_SAVED_THETA,         // heading soft-argmax (rad)
    kSavedCos = FMBYM_SAVED_COS,             // cos/sin(theta): rounded once, reused by later kernels
    kSavedSin = FMBYM_SAVED_SIN,
    kSavedThetaMax = FMBYM_SAVED_THETA_MAX,  // max of the centred c_theta
    kSavedThetaSum = FMBYM_SAVED_THETA_SUM,  // sum exp((c_theta - max) / T_theta)
    kSavedXyMax = FMBYM_SAVED_XY_MAX,        // max of c_xy
    kSavedXySum = FMBYM_SAVED_XY_SUM,        // sum exp((c_xy - max) / T_xy)
    kSavedTpx = FMBYM_SAVED_TPX,             // t' (metres) before the frame change
    kSavedTpy = FMBYM_SAVED_TPY,
    kSavedThetaMean = FMBYM_SAVED_THETA_MEAN,  // mean heading score over the lags
    kSavedThetaArg = FMBYM_SAVED_THETA_ARG,    // lag of the largest heading score
    kSavedThetaNu = FMBYM_SAVED_THETA_NU,      // sum_l p_l (l - argmax lag)
    kSavedStatus = FMBYM_SAVED_STATUS,         // non-finite input count (FMBYM_CHECK_FINITE)
};

struct Plan {
    fmbym_params p;
    int32_t max_batch;
    int device;
    float2* twiddle;   // [kTwiddleLen] W_2048^m
    float2* twiddle3;  // [kTwiddleLen3] W_3072^m (stage-2 lines of 3n/2 points)
    float* hann;       // [n] periodic Hann, FP64-evaluated, rounded once
    int band_on;
    int band_lo2;      // keep ceil((lo n)^2) <= ky^2 + kx^2 <= floor((hi n)^2)
    int band_hi2;
    // Transpose of the polar gather as a CSR matrix whose rows are the
    // half-plane bins in tile order (16 x 16 tiles of kx < n/2, then the
    // column kx = n/2): row p is bin csr_dst[p] (offset ky pitch_mag + kx in
    // a magnitude plane) and reads the polar samples csr_col (b n_theta + a)
    // with the bilinear weights csr_val.
    int* csr_ptr;
    int* csr_col;
    float* csr_val;
    int* csr_dst;
    int* dmag_part;    // [dmag_nparts + 1] first CSR row of each adjoint block
    int dmag_nparts;
    // Odd sides (forward only): the Bluestein chirp c_j = exp(i pi j^2 / n)
    // [n], its filter spectrum DFT_M(c wrapped) / M [odd_m1(n)], and the polar
    // angles (cos, sin)(pi a / n_theta) [n_theta].
    float2* chirp;
    float2* bspec;
    float2* polar_cs;
    fmbym_tuning tune; // column-tile widths of the column passes, batch split
    hipStream_t aux;   // second stream of a split batch (default priority)
    hipEvent_t fork, join;
};

// Widths measured best at 512 x 512 before tuning (8 float4 columns read whole
// 128-byte lines in stage 1; the 3n/2-point columns run 4 wide at 512).
fmbym_tuning default_tuning(int n);
bool valid_tile(int c);
// Every field in its range and every block within 1024 threads at side n.
bool tuning_ok(const fmbym_tuning& t, int n);

constexpr int kDmagTile = 16;     // bins per side of one tile of the CSR row order
constexpr int kDmagRows = 256;    // at most this many CSR rows per adjoint block
constexpr int kDmagChunk = 512;   // and about this many entries (more only for a single row)

// Build the plan's CSR transpose of the polar gather; returns a hipError_t.
int build_polar_csr(Plan& pl);

inline Plan* plan_cast(fmbym_plan p) { return reinterpret_cast<Plan*>(p); }

// FMBYM_EINVAL unless plan is set and 1 <= batch <= its max_batch.
int check_call(fmbym_plan plan, int32_t batch);
// check_call, and FMBYM_EUNSUPPORTED for plans whose path is forward only (odd sides).
int check_full_path(fmbym_plan plan, int32_t batch);
// The alternative readings of the scores (forward only).
constexpr uint32_t kReadingFlags = FMBYM_ANGLE_MARGINAL | FMBYM_LOGIT_ZSCORE | FMBYM_HARD_ARGMAX;
// check_full_path, and FMBYM_EUNSUPPORTED for plans with a reading flag (no adjoint).
int check_adjoint(fmbym_plan plan, int32_t batch);

// Record e as this thread's last HIP error (fmbym_last_hip_error); returns FMBYM_EHIP.
int hip_fail(hipError_t e);

// Geometry of the polar-gather blocks: radii per block of 256 threads, one
// line per n_theta / 8 threads; at least 4 so that blocks of long lines still
// sum several radii, and for n_theta >= 512 a single pass (the grid then fills
// the GPU in whole rounds of blocks rather than leaving a nearly empty one).
__host__ __device__ constexpr int radii_per_block(int n_theta) { return 2048 / n_theta > 4 ? 2048 / n_theta : 4; }
inline int radius_blocks(int n_r, int n_theta) {
    return (n_r + radii_per_block(n_theta) - 1) / radii_per_block(n_theta);
}

// Stage 2 correlates zero-padded scans of length pad2(n) = 3n/2 per axis: the
// smallest length at which the circular correlation equals the linear one for
// every lag of the window [-n/2, n/2) (a wrapped index lands in the zero
// padding).  Its lines use kE2 = 12 elements per thread: radix 4, 4, ..., 3.
__host__ __device__ constexpr int pad2(int n) { return 3 * n / 2; }
constexpr int kE2 = 12;

// Row pitches, in elements.  Every row array keeps its unique columns
// (n/2 + 1 in stage 1, 3n/4 + 1 in stage 2) plus room for the last, partial
// column tile of the column kernels (at most kPitchPad columns wide).
constexpr int kPitchPad = 16;
__host__ __device__ constexpr int pitch_rows1(int n) { return n / 2 + kPitchPad; }      // float4 (F_f, F_g)
__host__ __device__ constexpr int pitch_mag(int n) { return n / 2 + kPitchPad; }        // float2 (A_f, A_g)
__host__ __device__ constexpr int pitch_rows2(int n) { return 3 * n / 4 + kPitchPad; }  // float4 (F, G')
__host__ __device__ constexpr int pitch_lag(int n) { return 3 * n / 4 + kPitchPad; }    // float2

// Lines per 256-thread block of a stage-2 row kernel, and the softmax
// partials per pair of the inverse-row kernel (one per block of lag-row pairs).
__host__ __device__ constexpr int rows2_lines(int n) { return 256 / (pad2(n) / kE2); }
inline int xy_partials_per_pair(int n) { return (n / 2) / rows2_lines(n); }

// ------------------------------------------------------------ odd sides
//
// Scan sides 2^a - 1 (the paper's 127, 255 and 511 px) run a forward path of
// their own (search_odd.hip): stage-1 DFTs of n points by Bluestein's chirp
// transform over a power-of-two line of odd_m1(n) >= 2n - 1 points, stage 2
// zero-padded to odd_m2(n) = 3 2^b >= n + (n - 1)/2 points, and the heading
// correlation over any n_theta as a linear correlation over odd_lt(n_theta)
// points folded back onto the circle.
inline bool odd_side(int n) { return n == 127 || n == 255 || n == 511; }
inline int odd_m1(int n) { return n == 127 ? 256 : n == 255 ? 512 : 1024; }
inline int odd_m2(int n) { return n == 127 ? 192 : n == 255 ? 384 : 768; }
inline int odd_lt(int n_theta) {
    const int need = 2 * n_theta - 1;
    return need <= 512 ? 512 : need <= 768 ? 768 : need <= 1024 ? 1024 : need <= 1536 ? 1536 : 2048;
}
size_t odd_fwd_workspace(const fmbym_params& p, int batch);
int launch_forward_odd(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                       const float* mg, float* pose, float* c_theta, float* c_xy, float* saved, char* ws,
                       hipStream_t s);
// The translation soft-argmax's final merge over `ppp` online-softmax partials per pair.
void launch_xy_fin_parts(const float4* part, int ppp, float temp_xy, float delta_xy, int batch, float* pose,
                         float* saved, hipStream_t s);

// Workspace carve-up shared by forward and backward launchers.
struct FwdLayout {
    size_t r1r2;      // stage-1 row spectra [B][n][pitch_rows1] float4, then stage-2 [B][n][pitch_rows2] float4
    size_t mag_r3;    // magnitudes [B][n][pitch_mag] float2, then stage-2 columns [B][n][pitch_lag] float2
    size_t ptheta;    // [B][radius_blocks][n_theta/2 + 1] float2
    size_t pxy;       // [B][xy_partials] float4
    size_t saved;     // [B][FMBYM_SAVED] float (used when the caller passes none)
    size_t grot;      // [B][n][n] float: g' = Rotate(g_w), the rotated stage-2 scan
    size_t fin;       // [B][kFiniteSlices] int: non-finite input counts per slice
    size_t total;
};
FwdLayout fwd_layout(const fmbym_params& p, int batch);
constexpr int kFiniteSlices = 64;   // blocks per pair of the non-finite count

// Intermediates a training forward keeps in the caller's state buffer, so that
// its adjoint reads them instead of recomputing them.
struct Keep {
    float4* r1;    // stage-1 row spectra [B][n][pitch_rows1] float4
    float2* pspec; // angular DFT of each radius of (P_f + i P_g) [B][n_r][n_theta] float2
    float* gr;     // g' = Rotate(g_w) [B][n][n]
    float* jac;    // d g' / d theta [B][n][n]
    float4* r2;    // stage-2 row spectra [B][n][pitch_rows2] float4
};
size_t keep_bytes(const fmbym_params& p, int batch);
Keep keep_pointers(const fmbym_params& p, int batch, void* state);

// tab: null for packed batches (scan b at x + b n^2), else a device table of
// 4 pointers per pair, (f, g, m_f, m_g), for a ragged work list.  keep: null,
// or where the forward leaves its intermediates for the adjoint.
int launch_forward(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                   const float* mg, float* pose, float* c_theta, float* c_xy, float* saved,
                   char* ws, hipStream_t s, const float* const* tab = nullptr, const Keep* keep = nullptr);

// Stage 2 alone (k_rotate, k_rows2, k_cols2, k_rows3) for `batch` pairs whose
// heading is in saved[b] (cos, sin); writes c_xy [batch][n][n] and the
// softmax partials into the forward layout of ws.  tab as for launch_forward.
void launch_stage2(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                   const float* mg, const float* saved, float* c_xy, char* ws, hipStream_t s,
                   const float* const* tab);

// Stage-2 rows of f_w + i g' (k_rows2, g' read from gr) for a packed batch -> out.
void launch_rows2(const Plan& pl, int batch, const float* f, const float* g, const float* mf, const float* mg,
                  const float* gr, float4* out, int win2, hipStream_t s);

// The translation soft-argmax of stage 2 (k_xy_fin) over the partials that
// launch_stage2 left in the forward layout of ws: t' and t = R t' with the
// cos/sin in saved[b]; writes pose[b][1..2] and the softmax statistics.
void launch_xy_fin(const Plan& pl, int batch, char* ws, float* pose, float* saved, hipStream_t s);

// Full-circle heading: the forward, stage 2 again at theta + pi, the larger
// correlation peak kept.  One call for `batch` pairs in ws (full_circle_workspace).
size_t full_circle_workspace(const fmbym_params& p, int batch);
int launch_full_circle(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                       const float* mg, float* pose, float* peaks, char* ws, hipStream_t s);

// Joint comparator: K headings -pi/2 + k pi / K, stage 2 at each, hard argmax.
size_t joint_workspace(const fmbym_params& p, int batch, int n_angles);
int launch_joint(const Plan& pl, int batch, int n_angles, const float* f, const float* g, const float* mf,
                 const float* mg, float* pose, float* peak, char* ws, hipStream_t s);

// Stage-1 row DFTs and |F| (k_rows1, k_cols1), shared by forward and adjoint.
void launch_stage1_spectra(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                           const float* mg, float4* r1, float2* mag, hipStream_t s);

size_t bwd_workspace(const fmbym_params& p, int batch);
// The pairs [b0, b0 + ...) of a full-batch state (every kept array is batch-major).
Keep keep_slice(const Keep& k, const fmbym_params& p, int b0);

// Search calls with the plan's batch split: the halves run on the caller's
// stream and the plan's aux stream (fork/join by events), each in its own
// region of the workspace; keep_full is the state of the whole batch or null.
size_t run_fwd_workspace(const Plan& pl, int batch);
size_t run_bwd_workspace(const Plan& pl, int batch);
int run_forward(const Plan& pl, int batch, const float* f, const float* g, const float* mf, const float* mg,
                float* pose, float* c_theta, float* c_xy, float* saved, char* ws, hipStream_t s,
                const Keep* keep_full);
int run_backward(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                 const float* mg, const float* pose, const float* c_theta, const float* c_xy,
                 const float* saved, const float* d_pose, float* d_f, float* d_g, float* d_mf, float* d_mg,
                 char* ws, hipStream_t s, const Keep* keep_full);
// Training forward then adjoint per half of the batch, one fork and join.
int run_vjp(const Plan& pl, int batch, const float* f, const float* g, const float* mf, const float* mg,
            float* pose, float* c_theta, float* c_xy, float* saved, const float* d_pose, float* d_f,
            float* d_g, float* d_mf, float* d_mg, char* ws, hipStream_t s, const Keep& keep_full);
size_t run_full_circle_workspace(const Plan& pl, int batch);
int run_full_circle(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                    const float* mg, float* pose, float* peaks, char* ws, hipStream_t s);

// keep: null (recompute the spectra and g'), or the state of a training forward.
int launch_backward(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                    const float* mg, const float* pose, const float* c_theta, const float* c_xy,
                    const float* saved, const float* d_pose, float* d_f, float* d_g, float* d_mf,
                    float* d_mg, char* ws, hipStream_t s, const Keep* keep = nullptr);

// ------------------------------------------------------------------ sampling

// The scans of pair b: packed batches, or row b of a ragged pointer table.
struct PairScans {
    const float* f;
    const float* g;
    const float* mf;
    const float* mg;
};
__device__ __forceinline__ PairScans pair_scans(const float* const* __restrict__ tab, int b, int n,
                                                const float* f, const float* g, const float* mf,
                                                const float* mg) {
    if (tab) return PairScans{tab[4 * b], tab[4 * b + 1], tab[4 * b + 2], tab[4 * b + 3]};
    const size_t o = (size_t)b * n * n;
    return PairScans{f + o, g + o, mf ? mf + o : nullptr, mg ? mg + o : nullptr};
}

// Windowed (and masked) scan value at an integer pixel.  Branch-free: the
// mask is read through x when there is none and the window values always
// (hann has n entries), and both are applied by selects, so that the loads of
// a whole row are issued before the first use instead of each behind a branch.
__device__ __forceinline__ float scan_w(const float* __restrict__ x, const float* __restrict__ m,
                                        const float* __restrict__ hann, int n, int r, int c,
                                        bool win) {
    const float* mp = m ? m : x;
    const float xv = x[r * n + c], mv = mp[r * n + c], wv = hann[r] * hann[c];
    return xv * (m ? mv : 1.f) * (win ? wv : 1.f);
}

// Source position of output pixel (i, j) under Rotate: R(theta) y about the centre.
__device__ __forceinline__ void rot_src(int n, int i, int j, float ct, float st, float& py, float& px) {
    const float yx = (float)(j - n / 2);
    const float yy = (float)(i - n / 2);
    px = ct * yx - st * yy + (float)(n / 2);
    py = st * yx + ct * yy + (float)(n / 2);
}

// g'(i, j) = bilinear(g_w)(R(theta) y), lattice points outside the scan read as zero.
__device__ __forceinline__ float rotate_sample(const float* __restrict__ g, const float* __restrict__ m,
                                               const float* __restrict__ hann, int n, int i, int j,
                                               float ct, float st, bool win) {
    float py, px;
    rot_src(n, i, j, ct, st, py, px);
    const float fy = floorf(py), fx = floorf(px);
    const float wy = py - fy, wx = px - fx;
    const int y0 = (int)fy, x0 = (int)fx;
    float acc = 0.f;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int r = y0 + dy, c = x0 + dx;
            if (r >= 0 && r < n && c >= 0 && c < n) {
                const float w = (dy ? wy : 1.f - wy) * (dx ? wx : 1.f - wx);
                acc += w * scan_w(g, m, hann, n, r, c, win);
            }
        }
    }
    return acc;
}

// d g'(i, j) / d theta: the bilinear gradient of g_w at the sample position
// times the derivative of the position, R'(theta) y.
__device__ __forceinline__ float rotate_dtheta(const float* __restrict__ g, const float* __restrict__ m,
                                               const float* __restrict__ hann, int n, int i, int j,
                                               float ct, float st, bool win) {
    float py, px;
    rot_src(n, i, j, ct, st, py, px);
    const float fy = floorf(py), fx = floorf(px);
    const float wy = py - fy, wx = px - fx;
    const int y0 = (int)fy, x0 = (int)fx;
    float G[2][2];
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int r = y0 + dy, c = x0 + dx;
            G[dy][dx] = (r >= 0 && r < n && c >= 0 && c < n) ? scan_w(g, m, hann, n, r, c, win) : 0.f;
        }
    const float gx = (1.f - wy) * (G[0][1] - G[0][0]) + wy * (G[1][1] - G[1][0]);
    const float gy = (1.f - wx) * (G[1][0] - G[0][0]) + wx * (G[1][1] - G[0][1]);
    const float yx = (float)(j - n / 2), yy = (float)(i - n / 2);
    return gx * (-st * yx - ct * yy) + gy * (ct * yx - st * yy);
}

// Output tiles of the rotation kernels and the side of the LDS box that holds
// the source pixels of one tile at any angle.
constexpr int kRotTY = 16, kRotTX = 64;
constexpr int kRotBox = 72;   // > sqrt(kRotTX^2 + kRotTY^2) + 6

// Stage rows by0 .. by0+bh-1, columns bx0 .. bx0+bw-1 of x (times m if MASKED,
// times the separable window if WIN) into box at a pitch of kRotBox words,
// lattice points outside the n x n scan as zero.  For blocks of 256 threads.
// The loads are unconditional at clamped addresses (hann has n entries), so
// four of them per thread are in flight before the LDS stores.
template <bool MASKED, bool WIN>
__device__ __forceinline__ void stage_box(float* __restrict__ box, const float* __restrict__ x,
                                          const float* __restrict__ m, const float* __restrict__ hann,
                                          int n, int by0, int bx0, int bh, int bw) {
    const int lim = bh * kRotBox;
    for (int k0 = threadIdx.x; k0 < lim; k0 += 4 * 256) {
        float val[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 256 * u, cc = k % kRotBox;
            const int r = by0 + k / kRotBox, c = bx0 + cc;
            const int rc = min(max(r, 0), n - 1), ccl = min(max(c, 0), n - 1);
            float v = x[(size_t)rc * n + ccl];
            if (MASKED) v *= m[(size_t)rc * n + ccl];
            if (WIN) v *= hann[rc] * hann[ccl];
            // a factor rather than a branch: the load stays unconditional (scans are finite)
            val[u] = v * (float)((r == rc) & (c == ccl));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 256 * u;
            if (k < lim && k % kRotBox < bw) box[k] = val[u];
        }
    }
}

// Rotate g_w by the pair's heading into gr (and its theta derivative into jac
// when not null), one pixel per thread: the gathers run in a kernel of their
// own so that their latency is hidden by many light waves.
void launch_rotate(const Plan& pl, int batch, const float* g, const float* mg, const float* saved,
                   float* gr, float* jac, int win, hipStream_t s, const float* const* tab);

// Polar sample (radius b, angle a): frequency u = rho (cos phi, sin phi) in bins.
__device__ __forceinline__ void polar_uv(const float2* __restrict__ tw, int n, int n_r, int n_theta,
                                         int b, int a, float& uy, float& ux) {
    const float rho = (float)((n / 2) * b) / (float)n_r;
    const float2 w = tw[a * (kTwiddleLen / (2 * n_theta))];   // exp(-i pi a / n_theta)
    ux = rho * w.x;
    uy = rho * (-w.y);
}

// Bilinear read of both half-plane magnitude spectra (interleaved) at
// (uy, ux), using |F(-k)| = |F(k)| for corners with negative column and
// indices modulo n.
__device__ __forceinline__ float2 mag_sample(const float2* __restrict__ A, int n, float uy, float ux) {
    const int P = pitch_mag(n);
    const float fy = floorf(uy), fx = floorf(ux);
    const float wy = uy - fy, wx = ux - fx;
    const int y0 = (int)fy, x0 = (int)fx;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            int ky = y0 + dy, kx = x0 + dx;
            if (kx < 0) {
                ky = -ky;
                kx = -kx;
            }
            ky &= (n - 1);
            const float w = (dy ? wy : 1.f - wy) * (dx ? wx : 1.f - wx);
            const float2 a = A[ky * P + kx];
            acc.x += w * a.x;
            acc.y += w * a.y;
        }
    }
    return acc;
}

// ------------------------------------------------------------ block reductions

// Deterministic reductions over the first `cnt` threads (a power of two) of
// the block; every thread of the block must call them (they hold barriers).
__device__ __forceinline__ float block_max(float v, float* red, int cnt) {
    if ((int)threadIdx.x < cnt) red[threadIdx.x] = v;
    __syncthreads();
    for (int s = cnt / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}
__device__ __forceinline__ float block_sum(float v, float* red, int cnt) {
    if ((int)threadIdx.x < cnt) red[threadIdx.x] = v;
    __syncthreads();
    for (int s = cnt / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

// Largest value and its lowest index, over the block (deterministic tree).
__device__ __forceinline__ void block_argmax(float v, int idx, float* rv, int* ri, int cnt,
                                             float& out_v, int& out_i) {
    if ((int)threadIdx.x < cnt) {
        rv[threadIdx.x] = v;
        ri[threadIdx.x] = idx;
    }
    __syncthreads();
    for (int s = cnt / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const float a = rv[threadIdx.x], b = rv[threadIdx.x + s];
            const int ia = ri[threadIdx.x], ib = ri[threadIdx.x + s];
            if (b > a || (b == a && ib < ia)) {
                rv[threadIdx.x] = b;
                ri[threadIdx.x] = ib;
            }
        }
        __syncthreads();
    }
    out_v = rv[0];
    out_i = ri[0];
    __syncthreads();
}

// Online-softmax merge of two partials (max, sum of exp, and two weighted sums).
__device__ __forceinline__ float4 softmax_merge(float4 a, float4 c, float inv_t) {
    if (c.x == -INFINITY) return a;   // empty partials (threads past the end)
    if (a.x == -INFINITY) return c;
    const float M = fmaxf(a.x, c.x);
    const float ea = expf((a.x - M) * inv_t), ec = expf((c.x - M) * inv_t);
    return make_float4(M, a.y * ea + c.y * ec, a.z * ea + c.z * ec, a.w * ea + c.w * ec);
}

}  // namespace fmbym
