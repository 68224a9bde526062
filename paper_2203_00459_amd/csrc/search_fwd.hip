// Forward decoupled search (Algorithm 1) on gfx950.
//
// Stage 1 (heading, Eq. 5-8)
//   k_rows1      Hann (+mask) and row DFTs of f + i g (one complex FFT serves
//                both real scans), split into the two spectra, n/2 + 1 columns.
//   k_cols1      column DFTs of both spectra, band-pass and magnitude.
//   k_polar      bilinear polar gather of both magnitude spectra, angular DFT
//                per radius, conj(A_f) A_g summed over a block of radii.
//   k_angle_fin  sum over radius blocks, inverse angular DFT -> c_theta,
//                temperature softmax and soft-argmax -> theta (stays on device).
// Stage 2 (translation, Eq. 9)
//   k_rotate     g' = Rotate(g_w, theta) through an LDS-staged source box.
//   k_rows2      f_w and g' zero-padded to 3n/2 (the shortest length whose
//                circular correlation equals the linear one on the searched
//                lag window), row DFTs; 3n/4 + 1 unique columns kept.
//   k_cols2      column DFTs of both, conj(F) G', inverse column DFT, keeping
//                the n central lag rows.
//   k_rows3      inverse row DFTs of two lag rows at a time -> c_xy, and
//                online-softmax partials.
//   k_xy_fin     fixed-order merge of the partials -> t' -> t = R(theta) t'.
//
// Data between passes: row kernels write the two spectra they produce
// interleaved (float4 per column), so a column tile of 8 reads 128-byte
// segments; every row keeps all its unique columns (0 .. n/2 or 0 .. 3n/4), so
// column kernels treat every column alike.  All reductions are in a fixed
// order; results are bitwise reproducible.
#include "internal.hpp"
#include "profile.hpp"

namespace fmbym {

constexpr int kE = 8;   // elements per thread in every FFT line

// ------------------------------------------------------------------ stage 1

template <int N, int SEQ>
__global__ __launch_bounds__(256) void k_rows1(const float* __restrict__ f, const float* __restrict__ g,
                                               const float* __restrict__ mf, const float* __restrict__ mg,
                                               const float* __restrict__ hann,
                                               const float2* __restrict__ tw, float4* __restrict__ out,
                                               int win, const float* const* __restrict__ tab) {
    constexpr int L = N, T = L / kE, LPB = 256 / T, H = N / 2, P = pitch_rows1(N);
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    // windowed, masked row of f + i g; branch-free (masks through a fallback
    // pointer, window always read, selects), so a row's loads issue together
    auto load = [&](int grow, float2 (&v)[kE]) {
        const int i = grow % N;
        const PairScans sc = pair_scans(tab, grow / N, N, f, g, mf, mg);
        const size_t off = (size_t)i * N;
        const float* fr = sc.f + off;
        const float* gr = sc.g + off;
        const float* mfr = (sc.mf ? sc.mf : sc.f) + off;
        const float* mgr = (sc.mg ? sc.mg : sc.g) + off;
        const bool mfo = sc.mf != nullptr, mgo = sc.mg != nullptr;
        const float hi = hann[i];
#pragma unroll
        for (int m = 0; m < kE; ++m) {
            const int x = t + m * T;
            const float hx = hann[x], a = fr[x], c = gr[x], ma = mfr[x], mc = mgr[x];
            const float w = win ? hi * hx : 1.f;
            v[m] = make_float2((mfo ? a * ma : a) * w, (mgo ? c * mc : c) * w);
        }
    };
    // SEQ rows per line in sequence: the next row's loads overlap the current transform
    const int grow0 = (blockIdx.x * SEQ) * LPB + line;
    float2 v[kE];
    load(grow0, v);
#pragma unroll
    for (int it = 0; it < SEQ; ++it) {
        const int grow = grow0 + it * LPB;
        float2 nx[kE];
        if (it + 1 < SEQ) load(grow + LPB, nx);
        fft_line<L, kE>(v, lre[line], lim[line], fresh_index(t), tw);
        float2 mir[kE];
        mirror_line<L, kE>(v, mir, lre[line], lim[line], fresh_index(t));
        float4* o = out + (size_t)grow * P;
#pragma unroll
        for (int m = 0; m <= kE / 2; ++m) {
            const int k = t + m * T;
            if (k <= H) {
                const float2 X = split_x(v[m], mir[m]), Y = split_y(v[m], mir[m]);
                o[k] = make_float4(X.x, X.y, Y.x, Y.y);
            }
        }
        if (it + 1 < SEQ) {
#pragma unroll
            for (int m = 0; m < kE; ++m) v[m] = nx[m];
        }
    }
}

__device__ __forceinline__ float band_gain(int ky_signed, int kx, int on, int lo2, int hi2) {
    if (!on) return 1.f;
    const int r2 = ky_signed * ky_signed + kx * kx;
    return (r2 >= lo2 && r2 <= hi2) ? 1.f : 0.f;
}

// Column DFTs of both stage-1 spectra and their band-passed magnitudes,
// written interleaved.  Tiles of C columns cover 0 .. n/2; the last tile has
// one live column.  E elements per thread set the radix plan (radix-8 stages
// for E = 8, radix-4 for E = 4; a tuning choice).
template <int N, int C, int E>
__global__ __launch_bounds__(C * N / E) void k_cols1(const float4* __restrict__ in,
                                                      float2* __restrict__ A,
                                                      const float2* __restrict__ tw, int band_on,
                                                      int lo2, int hi2, int batch) {
    constexpr int L = N, T = L / E, H = N / 2, P1 = pitch_rows1(N), PA = pitch_mag(N);
    constexpr int TILES = H / C + 1;
    __shared__ float lre[C][LdsCols<C>::words(L)];
    __shared__ float lim[C][LdsCols<C>::words(L)];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int per_xcd = gridDim.x / 8;   // grid is a multiple of 8
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;   // adjacent tiles on one XCD
    if (work >= batch * TILES) return;
    const int tile = work % TILES, b = work / TILES;
    const int col = tile * C + c;
    const float4* src = in + (size_t)b * N * P1;
    float2 vf[E], vg[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const float4 q = src[(size_t)(t + m * T) * P1 + col];
        vf[m] = make_float2(q.x, q.y);
        vg[m] = make_float2(q.z, q.w);
    }
    fft_line<L, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
    fft_line<L, E, LdsCols<C>>(vg, lre[c], lim[c], fresh_index(t), tw);
    if (col > H) return;   // padding lane of the last tile (no barriers follow)
    float2* dst = A + (size_t)b * N * PA;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int ky = t + m * T;
        const float gain = band_gain(ky < H ? ky : ky - N, col, band_on, lo2, hi2);
        dst[ky * PA + col] = make_float2(sqrtf(vf[m].x * vf[m].x + vf[m].y * vf[m].y) * gain,
                                         sqrtf(vg[m].x * vg[m].x + vg[m].y * vg[m].y) * gain);
    }
}

// One block per (pair, block of radii_per_block(NT) radii); grid is remapped so
// that all blocks of one pair run on the same XCD (its L2 keeps the pair's
// magnitude spectra).
// MARG (the marginal reading of Alg. 1's "Mean over r"): the block writes the
// sums over its radii of the angular spectra of both profiles (P_f, then P_g,
// HK bins each) instead of the sum of their products.
template <int NT, int N, bool MARG>
__global__ __launch_bounds__(256) void k_polar(const float2* __restrict__ A,
                                               const float2* __restrict__ tw,
                                               float2* __restrict__ part, int n_r, int batch,
                                               float2* __restrict__ spec_out) {
    constexpr int L = NT, T = L / kE, LPB = 256 / T, RPB = radii_per_block(NT), PASSES = (RPB + LPB - 1) / LPB;
    constexpr int HK = NT / 2 + 1;
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    const int nrb = (n_r + radii_per_block(NT) - 1) / radii_per_block(NT);
    const int total = batch * nrb;
    // XCD-aware remap: hardware deals consecutive block ids round-robin over 8 XCDs
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= total) return;   // block-uniform
    const int b = work / nrb, rb = work % nrb;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const float2* Ab = A + (size_t)b * N * pitch_mag(N);
    float2 acc[kE / 2 + 1], accg[kE / 2 + 1];
#pragma unroll
    for (int m = 0; m <= kE / 2; ++m) acc[m] = accg[m] = make_float2(0.f, 0.f);
    for (int pass = 0; pass < PASSES; ++pass) {
        const int slot = pass * LPB + line;
        const int rad = rb * RPB + slot;
        const bool live = slot < RPB && rad < n_r;
        float2 v[kE];
#pragma unroll
        for (int m = 0; m < kE; ++m) {
            if (live) {
                float uy, ux;
                polar_uv(tw, N, n_r, NT, rad, t + m * T, uy, ux);
                v[m] = mag_sample(Ab, N, uy, ux);
            } else {
                v[m] = make_float2(0.f, 0.f);
            }
        }
        fft_line<L, kE>(v, lre[line], lim[line], fresh_index(t), tw);
        if (spec_out && live) {   // kept for the adjoint (training forward)
            float2* o = spec_out + ((size_t)b * n_r + rad) * NT;
#pragma unroll
            for (int m = 0; m < kE; ++m) o[t + m * T] = v[m];
        }
        float2 mir[kE];
        mirror_line<L, kE>(v, mir, lre[line], lim[line], fresh_index(t));
#pragma unroll
        for (int m = 0; m <= kE / 2; ++m) {
            const float2 Xf = split_x(v[m], mir[m]);
            const float2 Xg = split_y(v[m], mir[m]);
            if constexpr (MARG) {
                acc[m] = cadd(acc[m], Xf);
                accg[m] = cadd(accg[m], Xg);
            } else {
                acc[m] = cadd(acc[m], cmulcj(Xf, Xg));
            }
        }
    }
    // fixed-order sum over the lines of the block, through LDS (2 HK <= the words of a line)
    constexpr int NS = MARG ? 2 : 1, W = NS * HK;
    __syncthreads();
    float* sre = &lre[0][0];
    float* sim = &lim[0][0];
    for (int m = 0; m <= kE / 2; ++m) {
        const int k = t + m * T;
        if (k < HK) {
            sre[line * W + k] = acc[m].x;
            sim[line * W + k] = acc[m].y;
            if constexpr (MARG) {
                sre[line * W + HK + k] = accg[m].x;
                sim[line * W + HK + k] = accg[m].y;
            }
        }
    }
    __syncthreads();
    float2* dst = part + ((size_t)b * nrb + rb) * W;
    for (int k = threadIdx.x; k < W; k += blockDim.x) {
        float2 s = make_float2(0.f, 0.f);
        for (int l = 0; l < LPB; ++l) s = cadd(s, make_float2(sre[l * W + k], sim[l * W + k]));
        dst[k] = s;
    }
}

// Sum over radius blocks, inverse angular DFT without its k = 0 term (the
// mean over lags, kept apart so that the lag-dependent part is exact to its
// own rounding), softmax and soft-argmax.  theta is formed as (l* + nu) dtheta
// with nu = sum p_l (l - l*), which stays accurate when the softmax is sharp.
constexpr int kAngleGroups = 4;   // thread groups that share the radius-block sum

// MARG: the partials hold the radius sums of both angular spectra; groups 0, 1
// add those of P_f over alternate radius blocks, groups 2, 3 those of P_g, and
// the score spectrum is conj(S_f) S_g.  mode bit kScoreZ standardises the
// scores (softmax of (c - max c) / (T sigma), sigma their standard deviation
// over the lags), bit kScoreHard takes theta = l* dtheta (the first maximum).
constexpr int kScoreZ = 1, kScoreHard = 2;

template <int NT, bool MARG>
__global__ __launch_bounds__(kAngleGroups * NT / kE) void k_angle_fin(
    const float2* __restrict__ part, int n_r, const float2* __restrict__ tw, float temp,
    float* __restrict__ c_theta, float* __restrict__ pose, float* __restrict__ saved, int mode) {
    constexpr int L = NT, T = L / kE, HK = NT / 2 + 1;
    __shared__ float lre[kAngleGroups][LdsRows<L>::words(L)];   // one line per group: the groups
    __shared__ float lim[kAngleGroups][LdsRows<L>::words(L)];   // repeat the transform, race-free
    __shared__ float2 psum[kAngleGroups][HK];
    __shared__ float red[T];
    __shared__ int redi[T];
    const int b = blockIdx.x;
    const int nrb = (n_r + radii_per_block(NT) - 1) / radii_per_block(NT);
    constexpr int W = MARG ? 2 * HK : HK;   // floats2 per radius block of the partials
    const float2* src = part + (size_t)b * nrb * W;
    {   // group q sums radius blocks q, q + G, ... ; the groups are then added in order
        // (MARG: groups 0, 1 over alternate blocks of S_f, groups 2, 3 of S_g)
        const int q = threadIdx.x / T, tt = threadIdx.x % T;
        const int r0 = MARG ? (q & 1) : q, rs = MARG ? 2 : kAngleGroups, off = MARG ? (q >> 1) * HK : 0;
        for (int k = tt; k < HK; k += T) {
            float2 s = make_float2(0.f, 0.f);
#pragma unroll 8
            for (int r = r0; r < nrb; r += rs) s = cadd(s, src[(size_t)r * W + off + k]);   // loads overlap
            psum[q][k] = s;
        }
    }
    __syncthreads();
    // the transform and softmax run on the first group; the others idle through
    // the barriers (their values are never stored)
    const int t = threadIdx.x % T;
    const bool lead = (int)threadIdx.x < T;
    float2 v[kE];
    float dc = 0.f;
#pragma unroll
    for (int m = 0; m < kE; ++m) {
        const int k = t + m * T;
        const int kk = k < HK ? k : NT - k;
        float2 s;
        if constexpr (MARG) {
            s = cmulcj(cadd(psum[0][kk], psum[1][kk]), cadd(psum[2][kk], psum[3][kk]));
        } else {
            s = psum[0][kk];
#pragma unroll
            for (int q = 1; q < kAngleGroups; ++q) s = cadd(s, psum[q][kk]);
        }
        if (k == 0) {
            dc = s.x;
            s = make_float2(0.f, 0.f);
        }
        v[m] = k < HK ? s : cconj(s);
    }
    ifft_line<L, kE>(v, lre[threadIdx.x / T], lim[threadIdx.x / T], t, tw);
    const float scale = 1.f / ((float)NT * (float)n_r);
    float c[kE];
    float lmax = -INFINITY;
    int larg = 0;
#pragma unroll
    for (int m = 0; m < kE; ++m) {
        const int n = t + m * T;
        const int k = n < NT / 2 ? n + NT / 2 : n - NT / 2;   // storage index of lag n
        c[m] = v[m].x * scale;
        if (c[m] > lmax || (c[m] == lmax && k < larg)) {
            lmax = c[m];
            larg = k;
        }
    }
    float cmax;
    int kmax;
    block_argmax(lmax, larg, red, redi, T, cmax, kmax);
    const int lag_star = kmax - NT / 2;
    float sigma = 1.f;
    if (mode & kScoreZ) {   // standard deviation of the scores over the lags (two fixed-order passes)
        float s1 = 0.f;
#pragma unroll
        for (int m = 0; m < kE; ++m) s1 += c[m];
        const float mean = block_sum(s1, red, T) / (float)NT;
        float s2 = 0.f;
#pragma unroll
        for (int m = 0; m < kE; ++m) s2 += (c[m] - mean) * (c[m] - mean);
        sigma = sqrtf(block_sum(s2, red, T) / (float)NT);
    }
    const float inv_t = 1.f / (temp * sigma);
    float se = 0.f, sn = 0.f;
#pragma unroll
    for (int m = 0; m < kE; ++m) {
        const int n = t + m * T;
        const int lag = n < NT / 2 ? n : n - NT;
        const float e = expf((c[m] - cmax) * inv_t);
        se += e;
        sn += e * (float)(lag - lag_star);
        if (c_theta && lead) c_theta[(size_t)b * NT + lag + NT / 2] = c[m];
    }
    const float Z = block_sum(se, red, T);
    const float SN = block_sum(sn, red, T);
    if (threadIdx.x == 0) {
        const float nu = (mode & kScoreHard) ? 0.f : SN / Z;
        const float theta = ((float)lag_star + nu) * (3.14159265358979323846f / (float)NT);
        pose[b * 3 + 0] = theta;
        float* sv = saved + (size_t)b * FMBYM_SAVED;
        sv[kSavedTheta] = theta;
        float snt, cst;
        sincosf(theta, &snt, &cst);
        sv[kSavedCos] = cst;
        sv[kSavedSin] = snt;
        sv[kSavedThetaMax] = cmax;
        sv[kSavedThetaSum] = Z;
        sv[kSavedThetaMean] = dc * scale;
        sv[kSavedThetaArg] = (float)lag_star;
        sv[kSavedThetaNu] = nu;
        // the status slot (set afterwards when the inputs are checked) and the
        // reserved slots are defined too
        for (int i = kSavedStatus; i < FMBYM_SAVED; ++i) sv[i] = 0.f;
    }
}

// ------------------------------------------------------------------ stage 2

template <int N, int SEQ>
__global__ __launch_bounds__(256) void k_rows2(const float* __restrict__ f, const float* __restrict__ g,
                                               const float* __restrict__ mf, const float* __restrict__ mg,
                                               const float* __restrict__ hann,
                                               const float2* __restrict__ tw,
                                               const float* __restrict__ gr,
                                               float4* __restrict__ out, int win,
                                               const float* const* __restrict__ tab) {
    constexpr int L = pad2(N), E = kE2, T = L / E, LPB = 256 / T, H = L / 2, P2 = pitch_rows2(N);
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    // SEQ rows per line, one after the other: the next row's loads are in
    // flight during the current row's transform
    auto load = [&](int grow, float2 (&v)[E]) {
        const int b = grow / N, i = grow % N;
        const PairScans sc = pair_scans(tab, b, N, f, g, mf, mg);
        const float* grow_g = gr + (size_t)grow * N;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int x = t + m * T;
            if (m < 2 * E / 3) {   // x < n: data; the padding up to 3n/2 is zero
                const float a = scan_w(sc.f, sc.mf, hann, N, i, x, win);
                v[m] = make_float2(a, grow_g[x]);
            } else {
                v[m] = make_float2(0.f, 0.f);
            }
        }
    };
    const int grow0 = (blockIdx.x * SEQ) * LPB + line;
    float2 v[E];
    load(grow0, v);
#pragma unroll
    for (int it = 0; it < SEQ; ++it) {
        const int grow = grow0 + it * LPB;
        float2 nx[E];
        if (it + 1 < SEQ) load(grow + LPB, nx);
        fft_line<L, E>(v, lre[line], lim[line], fresh_index(t), tw);
        float2 mir[E];
        mirror_line<L, E>(v, mir, lre[line], lim[line], fresh_index(t));
        float4* o = out + (size_t)grow * P2;
#pragma unroll
        for (int m = 0; m <= E / 2; ++m) {
            const int k = t + m * T;
            if (k <= H) {
                const float2 X = split_x(v[m], mir[m]), Y = split_y(v[m], mir[m]);
                o[k] = make_float4(X.x, X.y, Y.x, Y.y);
            }
        }
        if (it + 1 < SEQ) {
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = nx[m];
        }
    }
}

// Rotate g_w into gr (and d g' / d theta into jac when not null).  A block
// owns a kRotTY x kRotTX tile of output pixels; the source positions of the
// tile lie in the rotated tile's bounding box, which is staged in LDS (windowed
// and masked, zeros outside the scan) with coalesced row reads, and every
// bilinear corner is then read from LDS.  The arithmetic (positions, weights,
// summation order) is that of rotate_sample / rotate_dtheta.

template <int N>
__global__ __launch_bounds__(256) void k_rotate(const float* __restrict__ g, const float* __restrict__ mg,
                                                const float* __restrict__ hann,
                                                const float* __restrict__ saved, float* __restrict__ gr,
                                                float* __restrict__ jac, int win,
                                                const float* const* __restrict__ tab) {
    static_assert(N % kRotTX == 0 && N % kRotTY == 0, "tiles cover the scan");
    constexpr int TPR = N / kRotTX, TPP = TPR * (N / kRotTY);   // tiles per tile row, per pair
    __shared__ float box[kRotBox * kRotBox];
    const int b = blockIdx.x / TPP, tile = blockIdx.x % TPP;
    const int i0 = (tile / TPR) * kRotTY, j0 = (tile % TPR) * kRotTX;
    const PairScans sc = pair_scans(tab, b, N, g, g, mg, mg);
    const float ct = saved[(size_t)b * FMBYM_SAVED + kSavedCos];
    const float st = saved[(size_t)b * FMBYM_SAVED + kSavedSin];
    // bounding box of the tile's source positions (corners of the tile map to its extremes)
    float ymin = 1e30f, ymax = -1e30f, xmin = 1e30f, xmax = -1e30f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float py, px;
        rot_src(N, i0 + (c & 1) * (kRotTY - 1), j0 + (c >> 1) * (kRotTX - 1), ct, st, py, px);
        ymin = fminf(ymin, py); ymax = fmaxf(ymax, py);
        xmin = fminf(xmin, px); xmax = fmaxf(xmax, px);
    }
    const int by0 = (int)floorf(ymin) - 1, bx0 = (int)floorf(xmin) - 1;
    const int bh = min(kRotBox, (int)floorf(ymax) + 3 - by0), bw = min(kRotBox, (int)floorf(xmax) + 3 - bx0);
    if (sc.mg) {
        if (win) stage_box<true, true>(box, sc.g, sc.mg, hann, N, by0, bx0, bh, bw);
        else stage_box<true, false>(box, sc.g, sc.mg, hann, N, by0, bx0, bh, bw);
    } else {
        if (win) stage_box<false, true>(box, sc.g, nullptr, hann, N, by0, bx0, bh, bw);
        else stage_box<false, false>(box, sc.g, nullptr, hann, N, by0, bx0, bh, bw);
    }
    __syncthreads();
    float* go = gr + (size_t)b * N * N;
    float* jo = jac ? jac + (size_t)b * N * N : nullptr;
#pragma unroll
    for (int k = 0; k < kRotTY * kRotTX / 256; ++k) {
        const int e = threadIdx.x + 256 * k;
        const int i = i0 + e / kRotTX, j = j0 + e % kRotTX;
        float py, px;
        rot_src(N, i, j, ct, st, py, px);
        const float fy = floorf(py), fx = floorf(px);
        const float wy = py - fy, wx = px - fx;
        const int y0 = (int)fy - by0, x0 = (int)fx - bx0;
        // the 2 x 2 cell lies inside the box (its margins cover the tile's
        // extreme sample positions); one check keeps every LDS read in it
        const bool inside = (unsigned)y0 <= (unsigned)(bh - 2) && (unsigned)x0 <= (unsigned)(bw - 2);
        const float* cell = box + (inside ? y0 * kRotBox + x0 : 0);
        const float s = inside ? 1.f : 0.f;
        float G[2][2];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) G[dy][dx] = s * cell[dy * kRotBox + dx];
        float acc = 0.f;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) acc += (dy ? wy : 1.f - wy) * (dx ? wx : 1.f - wx) * G[dy][dx];
        go[(size_t)i * N + j] = acc;
        if (jo) {
            const float gx = (1.f - wy) * (G[0][1] - G[0][0]) + wy * (G[1][1] - G[1][0]);
            const float gy = (1.f - wx) * (G[1][0] - G[0][0]) + wx * (G[1][1] - G[0][1]);
            const float yx = (float)(j - N / 2), yy = (float)(i - N / 2);
            jo[(size_t)i * N + j] = gx * (-st * yx - ct * yy) + gy * (ct * yx - st * yy);
        }
    }
}

// Column pass of stage 2 over columns 0 .. 3n/4 of the padded row spectra:
// forward column DFTs of F and G' (n data rows, n/2 zero rows), conj(F) G',
// inverse column DFT; the n lag rows of the window are kept.
template <int N, int C>
__global__ __launch_bounds__(C * pad2(N) / kE2) void k_cols2(const float4* __restrict__ in,
                                                             const float2* __restrict__ tw,
                                                             float2* __restrict__ out, int batch) {
    constexpr int L = pad2(N), E = kE2, T = L / E, H = L / 2, TILES = H / C + 1, P2 = pitch_rows2(N),
                  P3 = pitch_lag(N);
    __shared__ float lre[C][LdsCols<C>::words(L)];
    __shared__ float lim[C][LdsCols<C>::words(L)];
    const int total = batch * TILES;
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= total) return;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int tile = work % TILES, b = work / TILES;
    const int col = tile * C + c;
    const float4* src = in + (size_t)b * N * P2;
    float2 vf[E], vg[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if (m < 2 * E / 3) {
            const float4 q = src[(size_t)(t + m * T) * P2 + col];
            vf[m] = make_float2(q.x, q.y);
            vg[m] = make_float2(q.z, q.w);
        } else {
            vf[m] = vg[m] = make_float2(0.f, 0.f);
        }
    }
    fft_line<L, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
    fft_line<L, E, LdsCols<C>>(vg, lre[c], lim[c], fresh_index(t), tw);
#pragma unroll
    for (int m = 0; m < E; ++m) vf[m] = cmulcj(vf[m], vg[m]);
    ifft_line<L, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
    if (col > H) return;
    float2* dst = out + (size_t)b * N * P3;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int n = t + m * T;        // lag row s_y = n (n < N/2) or n - 3N/2 (n >= N)
        if (m < E / 3) dst[(size_t)(n + N / 2) * P3 + col] = vf[m];
        else if (m >= 2 * E / 3) dst[(size_t)(n - N) * P3 + col] = vf[m];
    }
}

// Entry k of the full L-point Hermitian spectrum of a lag row whose columns
// 0 .. L/2 are stored (the DC and Nyquist entries are real by symmetry).
// Branch-free: one load at the stored index, then conjugate / drop the
// imaginary part by selects, so a line's loads issue together.
__device__ __forceinline__ float2 herm_get(const float2* __restrict__ row, int L, int k) {
    const float2 a = row[k <= L / 2 ? k : L - k];
    const bool real = k == 0 || k == L / 2;
    return make_float2(a.x, real ? 0.f : (k < L / 2 ? a.y : -a.y));
}

template <int N>
__global__ __launch_bounds__(256) void k_rows3(const float2* __restrict__ in,
                                               const float2* __restrict__ tw,
                                               float* __restrict__ c_xy, float4* __restrict__ part,
                                               float temp) {
    constexpr int L = pad2(N), E = kE2, T = L / E, LPB = 256 / T, PPP = (N / 2) / LPB, P3 = pitch_lag(N);
    constexpr int K = 2 * E / 3;    // kept lags per thread
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    __shared__ float4 red[256];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int gl = blockIdx.x * LPB + line;       // row pair over the batch
    const int b = gl / (N / 2), q = gl % (N / 2);
    const float2* r1 = in + ((size_t)b * N + 2 * q) * P3;
    const float2* r2 = r1 + P3;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * T;
        const float2 h1 = herm_get(r1, L, k), h2 = herm_get(r2, L, k);
        v[m] = make_float2(h1.x - h2.y, h1.y + h2.x);   // h1 + i h2
    }
    ifft_line<L, E>(v, lre[line], lim[line], t, tw);
    const float scale = 1.f / ((float)L * (float)L);
    const float inv_t = 1.f / temp;
    // kept lags: n < N/2 (m < E/3) and n >= N (m >= 2E/3)
    float cv[2][K];
    int sx[K];
    float lmax = -INFINITY;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int m = j < E / 3 ? j : j + E / 3;
        const int n = t + m * T;
        const int col = n < N / 2 ? n + N / 2 : n - N;
        sx[j] = col - N / 2;
        cv[0][j] = v[m].x * scale;
        cv[1][j] = v[m].y * scale;
        lmax = fmaxf(lmax, fmaxf(cv[0][j], cv[1][j]));
        if (c_xy) {
            c_xy[((size_t)b * N + 2 * q) * N + col] = cv[0][j];
            c_xy[((size_t)b * N + 2 * q + 1) * N + col] = cv[1][j];
        }
    }
    const float sy0 = (float)(2 * q - N / 2), sy1 = sy0 + 1.f;
    float Z = 0.f, Sx = 0.f, Sy = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float e0 = expf((cv[0][j] - lmax) * inv_t);
        const float e1 = expf((cv[1][j] - lmax) * inv_t);
        Z += e0 + e1;
        Sx += (e0 + e1) * (float)sx[j];
        Sy += e0 * sy0 + e1 * sy1;
    }
    red[threadIdx.x] = make_float4(lmax, Z, Sx, Sy);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const float4 a = red[threadIdx.x], c = red[threadIdx.x + s];
            const float M = fmaxf(a.x, c.x);
            const float ea = expf((a.x - M) * inv_t), ec = expf((c.x - M) * inv_t);
            red[threadIdx.x] = make_float4(M, a.y * ea + c.y * ec, a.z * ea + c.z * ec, a.w * ea + c.w * ec);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)b * PPP + (blockIdx.x % PPP)] = red[0];
}

// Merge of the online-softmax partials of one pair: 64 threads, each folds a
// strided subset, then a fixed-order tree.
__global__ __launch_bounds__(64) void k_xy_fin(const float4* __restrict__ part, int ppp, float temp,
                                               float delta, float* __restrict__ pose,
                                               float* __restrict__ saved) {
    __shared__ float4 red[64];
    const int b = blockIdx.x, t = threadIdx.x;
    const float inv_t = 1.f / temp;
    const float4* p = part + (size_t)b * ppp;
    float4 acc = make_float4(-INFINITY, 0.f, 0.f, 0.f);
    for (int i = t; i < ppp; i += 64) acc = softmax_merge(acc, p[i], inv_t);
    red[t] = acc;
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
        if (t < s) red[t] = softmax_merge(red[t], red[t + s], inv_t);
        __syncthreads();
    }
    if (t == 0) {
        const float4 r = red[0];
        float* sv = saved + (size_t)b * FMBYM_SAVED;
        const float tpx = delta * (r.z / r.y), tpy = delta * (r.w / r.y);
        const float ct = sv[kSavedCos], st = sv[kSavedSin];
        pose[b * 3 + 1] = ct * tpx - st * tpy;
        pose[b * 3 + 2] = st * tpx + ct * tpy;
        sv[kSavedXyMax] = r.x;
        sv[kSavedXySum] = r.y;
        sv[kSavedTpx] = tpx;
        sv[kSavedTpy] = tpy;
    }
}

// The translation soft-argmax of a pair from its whole surface c_xy, for the
// readings that need the surface's own statistics first: standardised scores
// (kScoreZ: softmax of (c - max c) / (T sigma), sigma the standard deviation
// over the n^2 lags) and the hard argmax (kScoreHard: t' = the lag of the first
// maximum in row-major order).  One block of 1024 threads per pair; every sum
// runs in a fixed order (strided per thread, then a tree).
__global__ __launch_bounds__(1024) void k_xy_stats(const float* __restrict__ c_xy, int n, float temp, float delta,
                                                   int mode, float* __restrict__ pose, float* __restrict__ saved) {
    __shared__ float red[1024];
    __shared__ int redi[1024];
    const int b = blockIdx.x, t = threadIdx.x;
    const int nn = n * n, half = n / 2;
    const float* c = c_xy + (size_t)b * nn;
    float s1 = 0.f, lmax = -INFINITY;
    int larg = 0;
    for (int i = t; i < nn; i += 1024) {
        const float v = c[i];
        s1 += v;
        if (v > lmax) {   // i increases: the first maximum of the thread keeps the lowest index
            lmax = v;
            larg = i;
        }
    }
    float cmax;
    int imax;
    block_argmax(lmax, larg, red, redi, 1024, cmax, imax);
    float sigma = 1.f;
    if (mode & kScoreZ) {
        const float mean = block_sum(s1, red, 1024) / (float)nn;
        float s2 = 0.f;
        for (int i = t; i < nn; i += 1024) s2 += (c[i] - mean) * (c[i] - mean);
        sigma = sqrtf(block_sum(s2, red, 1024) / (float)nn);
    }
    const float inv_t = 1.f / (temp * sigma);
    float z = 0.f, sx = 0.f, sy = 0.f;
    for (int i = t; i < nn; i += 1024) {
        const float e = expf((c[i] - cmax) * inv_t);
        z += e;
        sx += e * (float)(i % n - half);
        sy += e * (float)(i / n - half);
    }
    const float Z = block_sum(z, red, 1024);
    const float SX = block_sum(sx, red, 1024);
    const float SY = block_sum(sy, red, 1024);
    if (t == 0) {
        float* sv = saved + (size_t)b * FMBYM_SAVED;
        const bool hard = (mode & kScoreHard) != 0;
        const float tpx = delta * (hard ? (float)(imax % n - half) : SX / Z);
        const float tpy = delta * (hard ? (float)(imax / n - half) : SY / Z);
        const float ct = sv[kSavedCos], st = sv[kSavedSin];
        pose[b * 3 + 1] = ct * tpx - st * tpy;
        pose[b * 3 + 2] = st * tpx + ct * tpy;
        sv[kSavedXyMax] = cmax;
        sv[kSavedXySum] = Z;
        sv[kSavedTpx] = tpx;
        sv[kSavedTpy] = tpy;
    }
}

// ---------------------------------------------------------------- launcher

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

FwdLayout fwd_layout(const fmbym_params& p, int batch) {
    const size_t n = p.n, B = batch;
    FwdLayout L{};
    if (odd_side(p.n)) {   // the odd path carves its own regions; only the size is shared
        L.total = odd_fwd_workspace(p, batch);
        return L;
    }
    size_t off = 0;
    L.r1r2 = off;
    const size_t r1 = B * n * (size_t)pitch_rows1(p.n) * sizeof(float4);
    const size_t r2 = B * n * (size_t)pitch_rows2(p.n) * sizeof(float4);
    off = align256(off + (r1 > r2 ? r1 : r2));
    L.mag_r3 = off;
    const size_t mag = B * n * (size_t)pitch_mag(p.n) * sizeof(float2);
    const size_t r3 = B * n * (size_t)pitch_lag(p.n) * sizeof(float2);
    off = align256(off + (mag > r3 ? mag : r3));
    L.ptheta = off;
    const size_t spectra = (p.flags & FMBYM_ANGLE_MARGINAL) ? 2 : 1;   // marginal: both profiles' spectra
    off = align256(off + B * (size_t)radius_blocks(p.n_r, p.n_theta) * (p.n_theta / 2 + 1) * spectra * sizeof(float2));
    L.pxy = off;
    off = align256(off + B * (size_t)xy_partials_per_pair(p.n) * sizeof(float4));
    L.saved = off;
    off = align256(off + B * FMBYM_SAVED * sizeof(float));
    L.grot = off;
    off = align256(off + B * n * n * sizeof(float));
    L.fin = off;
    off = align256(off + B * kFiniteSlices * sizeof(int));
    L.total = off;
    return L;
}

size_t keep_bytes(const fmbym_params& p, int batch) {
    const size_t n = p.n, B = batch;
    return align256(B * n * (size_t)pitch_rows1(p.n) * sizeof(float4)) +
           align256(B * (size_t)p.n_r * p.n_theta * sizeof(float2)) + 2 * align256(B * n * n * sizeof(float)) +
           align256(B * n * (size_t)pitch_rows2(p.n) * sizeof(float4));
}

Keep keep_pointers(const fmbym_params& p, int batch, void* state) {
    const size_t n = p.n, B = batch;
    char* c = (char*)state;
    Keep k;
    k.r1 = (float4*)c;
    c += align256(B * n * (size_t)pitch_rows1(p.n) * sizeof(float4));
    k.pspec = (float2*)c;
    c += align256(B * (size_t)p.n_r * p.n_theta * sizeof(float2));
    k.gr = (float*)c;
    c += align256(B * n * n * sizeof(float));
    k.jac = (float*)c;
    c += align256(B * n * n * sizeof(float));
    k.r2 = (float4*)c;
    return k;
}

Keep keep_slice(const Keep& k, const fmbym_params& p, int b0) {
    const size_t n = p.n, b = b0;
    Keep r;
    r.r1 = k.r1 + b * n * pitch_rows1(p.n);
    r.pspec = k.pspec + b * (size_t)p.n_r * p.n_theta;
    r.gr = k.gr + b * n * n;
    r.jac = k.jac + b * n * n;
    r.r2 = k.r2 + b * n * pitch_rows2(p.n);
    return r;
}

// Column-tile widths are the plan's tuning (fmbym_tuning: 4, 8 or 16 columns
// per block); every width gives the same arithmetic per column.  The radix
// plan of the stage-1 columns (elements per thread, 8 or 4) is tuned too; the
// two plans round differently.  Blocks stay within 1024 threads (tuning_ok).
template <int N, int C, int E>
static void launch_cols1_ce(const Plan& pl, int B, const float4* r1, float2* mag, hipStream_t s) {
    const int tiles1 = B * ((N / 2) / C + 1);
    if constexpr (C * N / E <= 1024)
        FMBYM_LAUNCH(kKCols1, (k_cols1<N, C, E>), dim3(((tiles1 + 7) / 8) * 8), dim3(C * N / E), s, r1, mag,
                     pl.twiddle, pl.band_on, pl.band_lo2, pl.band_hi2, B);
}

template <int N, int C>
static void launch_cols1_c(const Plan& pl, int B, const float4* r1, float2* mag, hipStream_t s) {
    if (pl.tune.radix1 == 4) launch_cols1_ce<N, C, 4>(pl, B, r1, mag, s);
    else launch_cols1_ce<N, C, 8>(pl, B, r1, mag, s);
}

template <int N>
static void launch_cols1(const Plan& pl, int B, const float4* r1, float2* mag, hipStream_t s) {
    switch (pl.tune.cols1) {
        case 4: launch_cols1_c<N, 4>(pl, B, r1, mag, s); break;
        case 8: launch_cols1_c<N, 8>(pl, B, r1, mag, s); break;
        default: launch_cols1_c<N, 16>(pl, B, r1, mag, s); break;
    }
}

template <int N, int C>
static void launch_cols2_c(const Plan& pl, int B, const float4* r2, float2* r3, hipStream_t s) {
    constexpr int T2 = pad2(N) / kE2;
    const int total2 = B * ((pad2(N) / 2) / C + 1);
    FMBYM_LAUNCH(kKCols2, (k_cols2<N, C>), dim3(((total2 + 7) / 8) * 8), dim3(C * T2), s, r2, pl.twiddle3,
                 r3, B);
}

template <int N>
static void launch_cols2(const Plan& pl, int B, const float4* r2, float2* r3, hipStream_t s) {
    switch (pl.tune.cols2) {
        case 4: launch_cols2_c<N, 4>(pl, B, r2, r3, s); break;
        case 8: launch_cols2_c<N, 8>(pl, B, r2, r3, s); break;
        default: launch_cols2_c<N, 16>(pl, B, r2, r3, s); break;
    }
}

template <int N>
static void launch_stage1_rows_cols(const Plan& pl, int B, const float* f, const float* g,
                                    const float* mf, const float* mg, float4* r1, float2* mag,
                                    hipStream_t s, const float* const* tab) {
    const int win = (pl.p.flags & FMBYM_HANN) ? 1 : 0;
    constexpr int T1 = N / kE, LPB1 = 256 / T1;
    // rows per line in sequence (1 or 2): the plan's tuning, the same arithmetic per row
    if (pl.tune.rows1 == 1)
        FMBYM_LAUNCH(kKRows1, (k_rows1<N, 1>), dim3(B * N / LPB1), dim3(256), s, f, g, mf, mg, pl.hann,
                     pl.twiddle, r1, win, tab);
    else
        FMBYM_LAUNCH(kKRows1, (k_rows1<N, 2>), dim3(B * N / (LPB1 * 2)), dim3(256), s, f, g, mf, mg, pl.hann,
                     pl.twiddle, r1, win, tab);
    launch_cols1<N>(pl, B, r1, mag, s);
}

void launch_stage1_spectra(const Plan& pl, int B, const float* f, const float* g, const float* mf,
                           const float* mg, float4* r1, float2* mag, hipStream_t s) {
    switch (pl.p.n) {
        case 128: launch_stage1_rows_cols<128>(pl, B, f, g, mf, mg, r1, mag, s, nullptr); break;
        case 256: launch_stage1_rows_cols<256>(pl, B, f, g, mf, mg, r1, mag, s, nullptr); break;
        case 512: launch_stage1_rows_cols<512>(pl, B, f, g, mf, mg, r1, mag, s, nullptr); break;
        default: break;
    }
}

// Score readings of the plan's flags for k_angle_fin / k_xy_stats.
static int score_mode(const Plan& pl) {
    return ((pl.p.flags & FMBYM_LOGIT_ZSCORE) ? kScoreZ : 0) | ((pl.p.flags & FMBYM_HARD_ARGMAX) ? kScoreHard : 0);
}

template <int N, int NT>
static void launch_polar(const Plan& pl, int B, const float2* mag, float2* pth, float* c_theta,
                         float* pose, float* saved, hipStream_t s, float2* spec_out) {
    const int nrb = radius_blocks(pl.p.n_r, pl.p.n_theta);
    const int total = B * nrb;
    const int grid = ((total + 7) / 8) * 8;
    const int mode = score_mode(pl);
    if (pl.p.flags & FMBYM_ANGLE_MARGINAL) {
        FMBYM_LAUNCH(kKPolar, (k_polar<NT, N, true>), dim3(grid), dim3(256), s, mag, pl.twiddle, pth, pl.p.n_r, B,
                     spec_out);
        FMBYM_LAUNCH(kKAngleFin, (k_angle_fin<NT, true>), dim3(B), dim3(kAngleGroups * NT / kE), s, pth,
                     pl.p.n_r, pl.twiddle, pl.p.temp_theta, c_theta, pose, saved, mode);
    } else {
        FMBYM_LAUNCH(kKPolar, (k_polar<NT, N, false>), dim3(grid), dim3(256), s, mag, pl.twiddle, pth, pl.p.n_r,
                     B, spec_out);
        FMBYM_LAUNCH(kKAngleFin, (k_angle_fin<NT, false>), dim3(B), dim3(kAngleGroups * NT / kE), s, pth,
                     pl.p.n_r, pl.twiddle, pl.p.temp_theta, c_theta, pose, saved, mode);
    }
}

template <int N>
static void launch_rows2_n(const Plan& pl, int B, const float* f, const float* g, const float* mf,
                           const float* mg, const float* gr, float4* r2, int win2, hipStream_t s,
                           const float* const* tab) {
    constexpr int LPB2 = rows2_lines(N);
    if (pl.tune.rows2 == 1)
        FMBYM_LAUNCH(kKRows2, (k_rows2<N, 1>), dim3(B * N / LPB2), dim3(256), s, f, g, mf, mg, pl.hann,
                     pl.twiddle3, gr, r2, win2, tab);
    else
        FMBYM_LAUNCH(kKRows2, (k_rows2<N, 2>), dim3(B * N / (LPB2 * 2)), dim3(256), s, f, g, mf, mg, pl.hann,
                     pl.twiddle3, gr, r2, win2, tab);
}

// Stage 2 up to the lag rows: Rotate, the 3n/2-point rows of f_w + i g', the
// column correlation and the inverse rows (c_xy and the softmax partials in
// the layout's pxy region).  The heading is read from saved[b].
template <int N>
static void stage2_n(const Plan& pl, int B, const float* f, const float* g, const float* mf,
                     const float* mg, const float* sv, float* c_xy, char* ws, hipStream_t s,
                     const float* const* tab, const Keep* keep) {
    const FwdLayout lay = fwd_layout(pl.p, B);
    const int win2 = ((pl.p.flags & FMBYM_HANN) && !(pl.p.flags & FMBYM_XY_UNWINDOWED)) ? 1 : 0;
    // without keep, stage-1 rows are dead after k_cols1 and magnitudes after k_polar
    float4* r2 = keep ? keep->r2 : (float4*)(ws + lay.r1r2);
    float2* r3 = (float2*)(ws + lay.mag_r3);
    float4* pxy = (float4*)(ws + lay.pxy);
    constexpr int T2 = pad2(N) / kE2, LPB2 = rows2_lines(N);
    float* gr = keep ? keep->gr : (float*)(ws + lay.grot);
    FMBYM_LAUNCH(kKRotate, k_rotate<N>, dim3(B * (N / kRotTY) * (N / kRotTX)), dim3(256), s, g, mg, pl.hann,
                 sv, gr, keep ? keep->jac : nullptr, win2, tab);
    launch_rows2_n<N>(pl, B, f, g, mf, mg, gr, r2, win2, s, tab);
    launch_cols2<N>(pl, B, r2, r3, s);
    FMBYM_LAUNCH(kKRows3, k_rows3<N>, dim3(B * (N / 2) / LPB2), dim3(256), s, r3, pl.twiddle3, c_xy,
                 pxy, pl.p.temp_xy);
}

// Input check (FMBYM_CHECK_FINITE): slice q of pair b counts the values of f,
// g (and the masks) in [q n^2 / S, (q + 1) n^2 / S) that are NaN or infinite;
// then one thread per pair adds the slices in order into saved[b].
__global__ __launch_bounds__(256) void k_finite_part(const float* __restrict__ f, const float* __restrict__ g,
                                                     const float* __restrict__ mf, const float* __restrict__ mg,
                                                     int n, int* __restrict__ counts,
                                                     const float* const* __restrict__ tab) {
    const int b = blockIdx.x / kFiniteSlices, q = blockIdx.x % kFiniteSlices;
    const PairScans sc = pair_scans(tab, b, n, f, g, mf, mg);
    const int n4 = n * n / 4, per = n4 / kFiniteSlices;   // n^2 / 4 float4 per scan, a multiple of 64
    const float4* arr[4] = {(const float4*)sc.f, (const float4*)sc.g, (const float4*)sc.mf, (const float4*)sc.mg};
    int bad = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (!arr[a]) continue;   // block-uniform
        for (int i = q * per + (int)threadIdx.x; i < (q + 1) * per; i += 256) {
            const float4 v = arr[a][i];
            bad += !isfinite(v.x) + !isfinite(v.y) + !isfinite(v.z) + !isfinite(v.w);
        }
    }
    __shared__ int red[256];
    red[threadIdx.x] = bad;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

__global__ void k_finite_fin(const int* __restrict__ counts, int batch, float* __restrict__ saved) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    long long c = 0;
    for (int q = 0; q < kFiniteSlices; ++q) c += counts[b * kFiniteSlices + q];
    saved[(size_t)b * FMBYM_SAVED + kSavedStatus] = (float)c;
}

template <int N>
static int launch_n(const Plan& pl, int B, const float* f, const float* g, const float* mf,
                    const float* mg, float* pose, float* c_theta, float* c_xy, float* saved,
                    char* ws, hipStream_t s, const float* const* tab, const Keep* keep) {
    const FwdLayout lay = fwd_layout(pl.p, B);
    float4* r1 = keep ? keep->r1 : (float4*)(ws + lay.r1r2);
    float2* mag = (float2*)(ws + lay.mag_r3);   // dead after k_polar (the adjoint keeps the polar spectra)
    float2* pth = (float2*)(ws + lay.ptheta);
    float4* pxy = (float4*)(ws + lay.pxy);
    float* sv = saved ? saved : (float*)(ws + lay.saved);
    launch_stage1_rows_cols<N>(pl, B, f, g, mf, mg, r1, mag, s, tab);
    switch (pl.p.n_theta) {
        case 16: launch_polar<N, 16>(pl, B, mag, pth, c_theta, pose, sv, s, keep ? keep->pspec : nullptr); break;
        case 32: launch_polar<N, 32>(pl, B, mag, pth, c_theta, pose, sv, s, keep ? keep->pspec : nullptr); break;
        case 64: launch_polar<N, 64>(pl, B, mag, pth, c_theta, pose, sv, s, keep ? keep->pspec : nullptr); break;
        case 128: launch_polar<N, 128>(pl, B, mag, pth, c_theta, pose, sv, s, keep ? keep->pspec : nullptr); break;
        case 256: launch_polar<N, 256>(pl, B, mag, pth, c_theta, pose, sv, s, keep ? keep->pspec : nullptr); break;
        case 512: launch_polar<N, 512>(pl, B, mag, pth, c_theta, pose, sv, s, keep ? keep->pspec : nullptr); break;
        case 1024: launch_polar<N, 1024>(pl, B, mag, pth, c_theta, pose, sv, s, keep ? keep->pspec : nullptr); break;
        default: return FMBYM_EUNSUPPORTED;
    }
    const int mode = score_mode(pl);
    // the readings that need the whole surface first keep c_xy in the workspace
    // when the caller does not want it (g' is dead by then)
    float* cxy = (mode && !c_xy) ? (float*)(ws + lay.grot) : c_xy;
    stage2_n<N>(pl, B, f, g, mf, mg, sv, cxy, ws, s, tab, keep);
    if (mode)
        FMBYM_LAUNCH(kKXyFin, k_xy_stats, dim3(B), dim3(1024), s, cxy, N, pl.p.temp_xy, pl.p.delta_xy, mode, pose,
                     sv);
    else
        FMBYM_LAUNCH(kKXyFin, k_xy_fin, dim3(B), dim3(64), s, pxy, xy_partials_per_pair(N), pl.p.temp_xy,
                     pl.p.delta_xy, pose, sv);
    if (pl.p.flags & FMBYM_CHECK_FINITE) {   // after k_angle_fin, which clears the status slot
        int* counts = (int*)(ws + lay.fin);
        FMBYM_LAUNCH(kKFinite, k_finite_part, dim3(B * kFiniteSlices), dim3(256), s, f, g, mf, mg, N, counts,
                     tab);
        FMBYM_LAUNCH(kKFinite, k_finite_fin, dim3((B + 63) / 64), dim3(64), s, counts, B, sv);
    }
    return FMBYM_OK;
}

void launch_stage2(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                   const float* mg, const float* saved, float* c_xy, char* ws, hipStream_t s,
                   const float* const* tab) {
    switch (pl.p.n) {
        case 128: stage2_n<128>(pl, batch, f, g, mf, mg, saved, c_xy, ws, s, tab, nullptr); break;
        case 256: stage2_n<256>(pl, batch, f, g, mf, mg, saved, c_xy, ws, s, tab, nullptr); break;
        case 512: stage2_n<512>(pl, batch, f, g, mf, mg, saved, c_xy, ws, s, tab, nullptr); break;
        default: break;
    }
}

void launch_rows2(const Plan& pl, int batch, const float* f, const float* g, const float* mf, const float* mg,
                  const float* gr, float4* out, int win2, hipStream_t s) {
    switch (pl.p.n) {
        case 128: launch_rows2_n<128>(pl, batch, f, g, mf, mg, gr, out, win2, s, nullptr); break;
        case 256: launch_rows2_n<256>(pl, batch, f, g, mf, mg, gr, out, win2, s, nullptr); break;
        case 512: launch_rows2_n<512>(pl, batch, f, g, mf, mg, gr, out, win2, s, nullptr); break;
        default: break;
    }
}

void launch_xy_fin_parts(const float4* part, int ppp, float temp_xy, float delta_xy, int batch, float* pose,
                         float* saved, hipStream_t s) {
    FMBYM_LAUNCH(kKXyFin, k_xy_fin, dim3(batch), dim3(64), s, part, ppp, temp_xy, delta_xy, pose, saved);
}

void launch_xy_fin(const Plan& pl, int batch, char* ws, float* pose, float* saved, hipStream_t s) {
    const FwdLayout lay = fwd_layout(pl.p, batch);
    FMBYM_LAUNCH(kKXyFin, k_xy_fin, dim3(batch), dim3(64), s, (const float4*)(ws + lay.pxy),
                 xy_partials_per_pair(pl.p.n), pl.p.temp_xy, pl.p.delta_xy, pose, saved);
}

void launch_rotate(const Plan& pl, int B, const float* g, const float* mg, const float* saved, float* gr,
                   float* jac, int win, hipStream_t s, const float* const* tab) {
    const int N = pl.p.n;
    switch (N) {
        case 128:
            FMBYM_LAUNCH(kKRotate, k_rotate<128>, dim3(B * (128 / kRotTY) * (128 / kRotTX)), dim3(256), s, g, mg,
                         pl.hann,
                         saved, gr, jac, win, tab);
            break;
        case 256:
            FMBYM_LAUNCH(kKRotate, k_rotate<256>, dim3(B * (256 / kRotTY) * (256 / kRotTX)), dim3(256), s, g, mg,
                         pl.hann,
                         saved, gr, jac, win, tab);
            break;
        case 512:
            FMBYM_LAUNCH(kKRotate, k_rotate<512>, dim3(B * (512 / kRotTY) * (512 / kRotTX)), dim3(256), s, g, mg,
                         pl.hann,
                         saved, gr, jac, win, tab);
            break;
        default: break;
    }
}

int launch_forward(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                   const float* mg, float* pose, float* c_theta, float* c_xy, float* saved,
                   char* ws, hipStream_t s, const float* const* tab, const Keep* keep) {
    if (odd_side(pl.p.n)) {   // forward only, packed batches
        if (tab || keep) return FMBYM_EUNSUPPORTED;
        return launch_forward_odd(pl, batch, f, g, mf, mg, pose, c_theta, c_xy, saved, ws, s);
    }
    switch (pl.p.n) {
        case 128: return launch_n<128>(pl, batch, f, g, mf, mg, pose, c_theta, c_xy, saved, ws, s, tab, keep);
        case 256: return launch_n<256>(pl, batch, f, g, mf, mg, pose, c_theta, c_xy, saved, ws, s, tab, keep);
        case 512: return launch_n<512>(pl, batch, f, g, mf, mg, pose, c_theta, c_xy, saved, ws, s, tab, keep);
        default: return FMBYM_EUNSUPPORTED;
    }
}

}  // namespace fmbym
