// Adjoint of the decoupled search (reverse mode through Algorithm 1), with the
// spectra recomputed rather than stored.  Given d_pose = dL/d(theta, t_x, t_y):
//
//   t = R(theta) t'               dt' = R^T dt,  dtheta_1 = dt . R'(theta) t'
//   t' = delta sum_s q_s s        dc_xy[s] = q_s ((delta s - t') . dt') / T_xy
//   c_xy = f2 * g' (linear corr.) df2 = dc (corr) g',  dg' = f2 (conv) dc
//                                 (three 2n-padded transforms, two inverses)
//   g' = Rotate(g2, theta)        dg2 = Rotate^T dg' (gather form, no atomics)
//                                 dtheta_2 = sum_y dg'[y] grad(g2)(p_y) . dp_y/dtheta
//   theta = sum_l p_l l dtheta    dc_theta[l] = p_l (l dtheta - theta) dtheta_total / T_theta
//   c_theta = polar correlation   dP_f = corr(dc, P_g) / n_r, dP_g = conv(P_f, dc) / n_r
//                                 (per radius, through the angular DFT)
//   P = Cart2Pol(A)               dA = Cart2Pol^T dP (gather over the polar samples
//                                 whose bilinear footprint covers each bin)
//   A = band |F|                  dF = band dA F / |F|   (0 where F = 0)
//   F = DFT2(f_w)                 df_w = Re(unnormalised inverse DFT2 of dF)
//   f_w = w f m                   df = w m df_w, dm = w f df_w
//
// Kernels, in launch order:
//   (k_rotate, k_rows2 of the forward again, unless the forward kept g', J and the rows)
//   kb_rows_fwd2   rows of dc_xy (3n/2-padded), paired complex FFTs
//   kb_cols_xy     column FFTs, conj(DC) G' and F DC, inverse columns (rows < n kept)
//                  (layouts as in the forward: interleaved spectra, all unique columns)
//   kb_rows_xy     inverse rows -> df2, dg'; partial sums of dtheta_2
//   kb_dtheta      dtheta_total -> dc_theta -> its angular DFT
//   k_rows1/k_cols1 (forward kernels) recompute the stage-1 row spectra and |F|
//   kb_polar       polar gather + angular FFT again, the angular adjoint -> dP
//   kb_dmag        transposed polar gather dA = Cart2Pol^T dP (plan's CSR table)
//   kb_cols_mag    column FFTs again, |F| adjoint, inverse column DFT (in place
//                  over the row spectra)
//   kb_rows_final  inverse row DFT -> df_w, dg_w; adds the translation-stage
//                  terms (Rotate^T gathered here); window and mask adjoints
#include "internal.hpp"
#include "profile.hpp"

namespace fmbym {

constexpr int kEb = 8;
constexpr float kPi = 3.14159265358979323846f;

// Translation-stage softmax adjoint of one lag, from the forward's c_xy and statistics.
struct XyAdj {
    float M, invZ, inv_t, delta, tpx, tpy, dtpx, dtpy, bias;
    __device__ __forceinline__ float operator()(float c, int sx, int sy) const {
        const float q = expf((c - M) * inv_t) * invZ;
        return q * inv_t * (delta * ((float)sx * dtpx + (float)sy * dtpy) - bias);
    }
};

__device__ __forceinline__ XyAdj make_xy_adj(const float* sv, const float* dp, float temp, float delta) {
    XyAdj a;
    a.M = sv[kSavedXyMax];
    a.invZ = 1.f / sv[kSavedXySum];
    a.inv_t = 1.f / temp;
    a.delta = delta;
    a.tpx = sv[kSavedTpx];
    a.tpy = sv[kSavedTpy];
    const float ct = sv[kSavedCos], st = sv[kSavedSin];
    a.dtpx = ct * dp[1] + st * dp[2];     // dt' = R^T dt
    a.dtpy = -st * dp[1] + ct * dp[2];
    a.bias = a.tpx * a.dtpx + a.tpy * a.dtpy;
    return a;
}

// ------------------------------------------------------ translation adjoint

// Pairs of dc_xy lag rows (the softmax adjoint of c_xy, zero-padded to 3n/2)
// as one complex FFT each -> rdc, columns 0 .. 3n/4 of both row spectra.  The
// stage-2 rows of f_w and g' come from the forward's k_rows2 (kept, or run
// again by the recomputing adjoint), so both adjoints read the same values.
template <int N>
__global__ __launch_bounds__(256) void kb_rows_fwd2(const float2* __restrict__ tw,
                                                    const float* __restrict__ saved,
                                                    const float* __restrict__ c_xy,
                                                    const float* __restrict__ d_pose,
                                                    float2* __restrict__ rdc, float temp, float delta) {
    constexpr int L = pad2(N), E = kE2, T = L / E, LPB = 256 / T, H = L / 2, P3 = pitch_lag(N);
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    float2 v[E];
    const int gl = (int)blockIdx.x * LPB + line;   // lag-row pair
    const int b = gl / (N / 2), q = gl % (N / 2);
    {
        const XyAdj adj = make_xy_adj(saved + (size_t)b * FMBYM_SAVED, d_pose + b * 3, temp, delta);
        const float* c1 = c_xy + ((size_t)b * N + 2 * q) * N;
        const float* c2 = c1 + N;
        const int sy1 = 2 * q - N / 2, sy2 = sy1 + 1;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int x = t + m * T;                 // padded position s_x mod 3n/2
            if (m < E / 3 || m >= 2 * E / 3) {
                const int sx = m < E / 3 ? x : x - L;
                const int j = sx + N / 2;
                v[m] = make_float2(adj(c1[j], sx, sy1), adj(c2[j], sx, sy2));
            } else {
                v[m] = make_float2(0.f, 0.f);
            }
        }
    }
    fft_line<L, E>(v, lre[line], lim[line], t, tw);
    float2 mir[E];
    mirror_line<L, E>(v, mir, lre[line], lim[line], t);
    float2* o = rdc + ((size_t)b * N + 2 * q) * P3;
#pragma unroll
    for (int m = 0; m <= E / 2; ++m) {
        const int k = t + m * T;
        if (k > H) continue;
        o[k] = split_x(v[m], mir[m]);
        o[P3 + k] = split_y(v[m], mir[m]);
    }
}

// Column pass of the translation adjoint over columns 0 .. 3n/4: forward
// 3n/2-point column DFTs of F, G' and DC, then X1 = conj(DC) G' and X2 = F DC,
// inverse column DFTs; the n data rows of (X1, X2) go to out (which may be rf).
template <int N, int C>
__global__ __launch_bounds__(C * pad2(N) / kE2) void kb_cols_xy(const float4* rf, float4* out,
                                                                const float2* __restrict__ rdc,
                                                                const float2* __restrict__ tw,
                                                                int batch) {
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
    const float4* sf = rf + (size_t)b * N * P2;   // may equal out: a block reads its columns first
    float4* so = out + (size_t)b * N * P2;
    const float2* sd = rdc + (size_t)b * N * P3;
    float2 vd[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int n = t + m * T;
        // dc lag row o holds s_y = o - n/2, placed at padded row s_y mod 3n/2
        if (m < E / 3) vd[m] = sd[(size_t)(n + N / 2) * P3 + col];
        else if (m >= 2 * E / 3) vd[m] = sd[(size_t)(n - N) * P3 + col];
        else vd[m] = make_float2(0.f, 0.f);
    }
    // F and G' too before the first transform, whose barriers loads cannot cross
    float2 vf[E], vg[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if (m < 2 * E / 3) {
            const float4 q = sf[(size_t)(t + m * T) * P2 + col];
            vf[m] = make_float2(q.x, q.y);
            vg[m] = make_float2(q.z, q.w);
        } else {
            vf[m] = vg[m] = make_float2(0.f, 0.f);
        }
    }
    fft_line<L, E, LdsCols<C>>(vd, lre[c], lim[c], fresh_index(t), tw);
    fft_line<L, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
#pragma unroll
    for (int m = 0; m < E; ++m) vf[m] = cmul(vf[m], vd[m]);          // X2 = F DC
    fft_line<L, E, LdsCols<C>>(vg, lre[c], lim[c], fresh_index(t), tw);
#pragma unroll
    for (int m = 0; m < E; ++m) vg[m] = cmulcj(vd[m], vg[m]);        // X1 = conj(DC) G'
    ifft_line<L, E, LdsCols<C>>(vg, lre[c], lim[c], fresh_index(t), tw);
    ifft_line<L, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
    if (col > H) return;
#pragma unroll
    for (int m = 0; m < 2 * E / 3; ++m)
        so[(size_t)(t + m * T) * P2 + col] = make_float4(vg[m].x, vg[m].y, vf[m].x, vf[m].y);
}

// Entry k of the full L-point Hermitian spectrum from stored columns 0 .. L/2.
// Branch-free (one load at the stored index, then selects), as herm_get.
__device__ __forceinline__ float2 herm_get2(float2 (*get)(const float4*, int), const float4* row,
                                            int L, int k) {
    const float2 a = get(row, k <= L / 2 ? k : L - k);
    const bool real = k == 0 || k == L / 2;
    return make_float2(a.x, real ? 0.f : (k < L / 2 ? a.y : -a.y));
}
__device__ __forceinline__ float2 get_lo(const float4* row, int k) { return make_float2(row[k].x, row[k].y); }
__device__ __forceinline__ float2 get_hi(const float4* row, int k) { return make_float2(row[k].z, row[k].w); }

// Inverse rows of the translation adjoint -> df2, dg' (rows < n, columns < n),
// and the Rotate-path heading gradient dtheta_2 summed per block.
template <int N>
__global__ __launch_bounds__(256) void kb_rows_xy(const float4* __restrict__ q12,
                                                  const float* __restrict__ jac,
                                                  const float2* __restrict__ tw,
                                                  float* __restrict__ df2, float* __restrict__ dgp,
                                                  float* __restrict__ dth_part) {
    constexpr int L = pad2(N), E = kE2, T = L / E, LPB = 256 / T, PPB = N / LPB, P2 = pitch_rows2(N);
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    __shared__ float red[256];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int grow = blockIdx.x * LPB + line;
    const int b = grow / N, i = grow % N;
    const float4* row = q12 + (size_t)grow * P2;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * T;
        const float2 h1 = herm_get2(get_lo, row, L, k), h2 = herm_get2(get_hi, row, L, k);
        v[m] = make_float2(h1.x - h2.y, h1.y + h2.x);
    }
    const size_t base = (size_t)b * N * N;
    float jv[2 * E / 3];   // loaded before the transform, whose barriers the loads cannot cross
#pragma unroll
    for (int m = 0; m < 2 * E / 3; ++m) jv[m] = jac[base + (size_t)i * N + t + m * T];
    ifft_line<L, E>(v, lre[line], lim[line], t, tw);
    const float scale = 1.f / ((float)L * (float)L);
    float dth = 0.f;
#pragma unroll
    for (int m = 0; m < 2 * E / 3; ++m) {
        const int x = t + m * T;
        const float a = v[m].x * scale, d = v[m].y * scale;
        const size_t o = base + (size_t)i * N + x;
        df2[o] = a;
        dgp[o] = d;
        dth += d * jv[m];   // d g'(i, x) / d theta through the bilinear sample position
    }
    red[threadIdx.x] = dth;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) dth_part[(size_t)b * PPB + (blockIdx.x % PPB)] = red[0];
}

// dtheta_total -> dc_theta -> DFT over the lag (index l mod n_theta); one block per pair.
template <int NT>
__global__ __launch_bounds__(NT / kEb) void kb_dtheta(const float* __restrict__ dth_part, int ppb,
                                                      const float* __restrict__ c_theta,
                                                      const float* __restrict__ saved,
                                                      const float* __restrict__ d_pose,
                                                      const float2* __restrict__ tw, float temp,
                                                      float2* __restrict__ dspec) {
    constexpr int L = NT, T = L / kEb;
    __shared__ float lre[LdsRows<L>::words(L)];
    __shared__ float lim[LdsRows<L>::words(L)];
    __shared__ float red[T];
    const int b = blockIdx.x, t = threadIdx.x;
    float s = 0.f;
    for (int i = t; i < ppb; i += T) s += dth_part[(size_t)b * ppb + i];
    red[t] = s;
    __syncthreads();
    for (int k = T / 2; k > 0; k >>= 1) {
        if (t < k) red[t] += red[t + k];
        __syncthreads();
    }
    const float dth2 = red[0];
    const float* sv = saved + (size_t)b * FMBYM_SAVED;
    const float* dp = d_pose + b * 3;
    const float ct = sv[kSavedCos], st = sv[kSavedSin];
    const float tpx = sv[kSavedTpx], tpy = sv[kSavedTpy];
    // dtheta_1 = dt . R'(theta) t'
    const float dth1 = dp[1] * (-st * tpx - ct * tpy) + dp[2] * (ct * tpx - st * tpy);
    const float dtot = dp[0] + dth1 + dth2;
    const float M = sv[kSavedThetaMax], invZ = 1.f / sv[kSavedThetaSum];
    const int lag_star = (int)sv[kSavedThetaArg];
    const float nu = sv[kSavedThetaNu];
    const float inv_t = 1.f / temp, dlt = kPi / (float)NT;
    float2 v[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) {
        const int n = t + m * T;                    // index = lag mod n_theta
        const int lag = n < NT / 2 ? n : n - NT;
        const float c = c_theta[(size_t)b * NT + lag + NT / 2];
        const float p = expf((c - M) * inv_t) * invZ;
        // l dtheta - theta = ((l - l*) - nu) dtheta: no cancellation at the peak
        v[m] = make_float2(p * inv_t * ((float)(lag - lag_star) - nu) * dlt * dtot, 0.f);
    }
    fft_line<L, kEb>(v, lre, lim, t, tw);
#pragma unroll
    for (int m = 0; m < kEb; ++m) dspec[(size_t)b * NT + t + m * T] = v[m];
}

// ---------------------------------------------------------- rotation adjoint

// Polar gather + angular DFT of both magnitude spectra (as in the forward),
// then the angular adjoint: dP_f = IDFT(conj(D) Pg^) / n_r, dP_g = IDFT(Pf^ D) / n_r,
// written interleaved per polar sample.
template <int NT, int N>
__global__ __launch_bounds__(256) void kb_polar(const float2* __restrict__ A,
                                                const float2* __restrict__ tw,
                                                const float2* __restrict__ dspec,
                                                float2* __restrict__ dpol, int n_r, int batch) {
    constexpr int L = NT, T = L / kEb, LPB = 256 / T, RPB = radii_per_block(NT), PASSES = (RPB + LPB - 1) / LPB;
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    const int nrb = (n_r + radii_per_block(NT) - 1) / radii_per_block(NT);
    const int total = batch * nrb;
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= total) return;
    const int b = work / nrb, rb = work % nrb;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const float2* Ab = A + (size_t)b * N * pitch_mag(N);
    float2 D[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) D[m] = dspec[(size_t)b * NT + t + m * T];
    const float scale = 1.f / ((float)n_r * (float)NT);
    for (int pass = 0; pass < PASSES; ++pass) {
        const int slot = pass * LPB + line;
        const int rad = rb * RPB + slot;
        const bool live = slot < RPB && rad < n_r;
        float2 v[kEb];
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            if (live) {
                float uy, ux;
                polar_uv(tw, N, n_r, NT, rad, t + m * T, uy, ux);
                v[m] = mag_sample(Ab, N, uy, ux);
            } else {
                v[m] = make_float2(0.f, 0.f);
            }
        }
        fft_line<L, kEb>(v, lre[line], lim[line], fresh_index(t), tw);
        float2 mir[kEb];
        mirror_line<L, kEb>(v, mir, lre[line], lim[line], fresh_index(t));
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            const float2 Pf = split_x(v[m], mir[m]), Pg = split_y(v[m], mir[m]);
            const float2 a = cmulcj(D[m], Pg);     // conj(D) Pg
            const float2 c = cmul(Pf, D[m]);
            v[m] = make_float2(a.x - c.y, a.y + c.x);   // a + i c
        }
        ifft_line<L, kEb>(v, lre[line], lim[line], fresh_index(t), tw);
        if (live) {   // (dP_f, dP_g) interleaved: the transpose gathers both at once
            float2* o = dpol + ((size_t)b * n_r + rad) * NT;
#pragma unroll
            for (int m = 0; m < kEb; ++m) o[t + m * T] = cscale(v[m], scale);
        }
    }
}

// kb_polar from the training forward's kept polar spectra: the angular DFT of
// each radius (X = DFT(P_f + i P_g)) is read instead of gathered and
// transformed again, the mirror X[-k] straight from the same row.
template <int NT, int N>
__global__ __launch_bounds__(256) void kb_polar_keep(const float2* __restrict__ pspec,
                                                     const float2* __restrict__ tw,
                                                     const float2* __restrict__ dspec,
                                                     float2* __restrict__ dpol, int n_r, int batch) {
    constexpr int L = NT, T = L / kEb, LPB = 256 / T, RPB = radii_per_block(NT), PASSES = (RPB + LPB - 1) / LPB;
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    const int nrb = (n_r + radii_per_block(NT) - 1) / radii_per_block(NT);
    const int total = batch * nrb;
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= total) return;
    const int b = work / nrb, rb = work % nrb;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    float2 D[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) D[m] = dspec[(size_t)b * NT + t + m * T];
    const float scale = 1.f / ((float)n_r * (float)NT);
    for (int pass = 0; pass < PASSES; ++pass) {
        const int slot = pass * LPB + line;
        const int rad = rb * RPB + slot;
        const bool live = slot < RPB && rad < n_r;
        const float2* X = pspec + ((size_t)b * n_r + (live ? rad : 0)) * NT;
        float2 v[kEb];
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            const int k = t + m * T;
            const float2 x = live ? X[k] : make_float2(0.f, 0.f);
            const float2 xm = live ? X[k == 0 ? 0 : NT - k] : make_float2(0.f, 0.f);
            const float2 Pf = split_x(x, xm), Pg = split_y(x, xm);
            const float2 a = cmulcj(D[m], Pg);     // conj(D) Pg
            const float2 c = cmul(Pf, D[m]);
            v[m] = make_float2(a.x - c.y, a.y + c.x);   // a + i c
        }
        ifft_line<L, kEb>(v, lre[line], lim[line], fresh_index(t), tw);
        if (live) {
            float2* o = dpol + ((size_t)b * n_r + rad) * NT;
#pragma unroll
            for (int m = 0; m < kEb; ++m) o[t + m * T] = cscale(v[m], scale);
        }
    }
}

// dA = Cart2Pol^T dP over the half-plane bins, from the plan's CSR transpose
// of the polar gather (rows of bins outside the band are empty, so they come
// out 0).  Block x owns the CSR rows [part[x], part[x+1]) (at most kDmagRows
// rows, about kDmagChunk entries: a balanced share of the entries, whatever
// the density of polar samples) and kDmagPairs pairs.  Every thread forms the
// products w * (dP_f, dP_g) of a strided set of entries for all the pairs at
// once (independent gathers, many in flight), then each row sums its own
// segment from LDS in entry order and lands at dst[row] of the magnitude
// plane.  A row longer than kDmagChunk is processed in chunks, still in order.
constexpr int kDmagPairs = 4;
constexpr int kDmagPer = kDmagChunk / 256;
static_assert(kDmagChunk % 256 == 0 && kDmagRows <= 256, "one row per thread, whole strides of entries");
__global__ __launch_bounds__(256) void kb_dmag(const int* __restrict__ ptr, const int* __restrict__ col,
                                               const float* __restrict__ val, const int* __restrict__ dst,
                                               const int* __restrict__ part,
                                               const float2* __restrict__ dpol, float2* __restrict__ dA,
                                               int n, int n_r, int n_theta, int batch, int nparts) {
    __shared__ float4 prod[kDmagChunk][kDmagPairs / 2];
    const int tid = threadIdx.x;
    // work item (run, pair group), runs fastest, in contiguous eighths per XCD:
    // neighbouring bins, whose polar samples overlap, share one XCD's L2
    const int groups = (batch + kDmagPairs - 1) / kDmagPairs, total = nparts * groups;
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= total) return;
    const int run = work % nparts, grp = work / nparts;
    // the block's entry range from two uniform reads: the entry loads need not
    // wait for the rows' bounds, which each thread reads for itself
    const int r0 = part[run], nrow = part[run + 1] - r0;
    const int e_begin = ptr[r0], e_end = ptr[r0 + nrow];
    const size_t pstride = (size_t)n_r * n_theta;
    const int p0 = grp * kDmagPairs, np = min(kDmagPairs, batch - p0);
    const float2* src = dpol + (size_t)p0 * pstride;
    const int my0 = tid < nrow ? ptr[r0 + tid] : 0, my1 = tid < nrow ? ptr[r0 + tid + 1] : 0;
    float2 acc[kDmagPairs];
#pragma unroll
    for (int p = 0; p < kDmagPairs; ++p) acc[p] = make_float2(0.f, 0.f);
    for (int c0 = e_begin; c0 < e_end; c0 += kDmagChunk) {
        const int c1 = min(e_end, c0 + kDmagChunk);
#pragma unroll
        for (int j = 0; j < kDmagPer; ++j) {
            const int e = c0 + tid + 256 * j;
            if (e >= c1) break;
            const int cc = col[e];
            const float w = val[e];
            float2 x[kDmagPairs];
#pragma unroll
            for (int p = 0; p < kDmagPairs; ++p)
                x[p] = p < np ? cscale(src[p * pstride + cc], w) : make_float2(0.f, 0.f);
#pragma unroll
            for (int h = 0; h < kDmagPairs / 2; ++h)
                prod[e - c0][h] = make_float4(x[2 * h].x, x[2 * h].y, x[2 * h + 1].x, x[2 * h + 1].y);
        }
        __syncthreads();
        // this thread's row segment within the chunk, summed by four interleaved
        // partial sums (entries e = a + 4 i + u into part u), then part 0 + 1 + 2 + 3:
        // a fixed order, with four independent LDS reads in flight for the long
        // rows near the spectrum's centre
        const int a = max(my0, c0), z = min(my1, c1);
        float2 part[4][kDmagPairs];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int p = 0; p < kDmagPairs; ++p) part[u][p] = make_float2(0.f, 0.f);
        int e = a;
        for (; e + 4 <= z; e += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int h = 0; h < kDmagPairs / 2; ++h) {
                    const float4 q = prod[e + u - c0][h];
                    part[u][2 * h] = cadd(part[u][2 * h], make_float2(q.x, q.y));
                    part[u][2 * h + 1] = cadd(part[u][2 * h + 1], make_float2(q.z, q.w));
                }
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            if (e + u < z) {
#pragma unroll
                for (int h = 0; h < kDmagPairs / 2; ++h) {
                    const float4 q = prod[e + u - c0][h];
                    part[u][2 * h] = cadd(part[u][2 * h], make_float2(q.x, q.y));
                    part[u][2 * h + 1] = cadd(part[u][2 * h + 1], make_float2(q.z, q.w));
                }
            }
        }
#pragma unroll
        for (int p = 0; p < kDmagPairs; ++p)
            acc[p] = cadd(acc[p], cadd(cadd(part[0][p], part[1][p]), cadd(part[2][p], part[3][p])));
        __syncthreads();
    }
    if (tid < nrow) {
        const int o = dst[r0 + tid];
        const size_t plane = (size_t)n * pitch_mag(n);
#pragma unroll
        for (int p = 0; p < kDmagPairs; ++p)
            if (p < np) dA[(p0 + p) * plane + o] = acc[p];
    }
}

__device__ __forceinline__ float2 mag_adjoint(float2 F, float dA) {
    const float a = sqrtf(F.x * F.x + F.y * F.y);
    if (!(a > 0.f)) return make_float2(0.f, 0.f);
    const float s = dA / a;
    return make_float2(F.x * s, F.y * s);
}


// Column pass of the rotation adjoint over columns 0 .. n/2, in place over the
// stage-1 row spectra: column DFTs again, dF = dA F / |F| (dA already
// carries the band gain), unnormalised inverse column DFT.  For columns 0 and
// n/2 the row pass uses only the real part of the result.
template <int N, int C, int E>
__global__ __launch_bounds__(C * N / E) void kb_cols_mag(const float4* r1, float4* out,
                                                           const float2* __restrict__ dA,
                                                           const float2* __restrict__ tw, int batch) {
    constexpr int L = N, T = L / E, H = N / 2, TILES = H / C + 1, P1 = pitch_rows1(N), PA = pitch_mag(N);
    __shared__ float lre[C][LdsCols<C>::words(L)];
    __shared__ float lim[C][LdsCols<C>::words(L)];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int total = gridDim.x, per_xcd = total / 8;   // grid is a multiple of 8
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;   // adjacent tiles on one XCD
    if (work >= batch * TILES) return;
    const int tile = work % TILES, b = work / TILES;
    const int col = tile * C + c;
    const float4* src = r1 + (size_t)b * N * P1;   // may equal out: a block reads its columns first
    float4* dst = out + (size_t)b * N * P1;
    const float2* da = dA + (size_t)b * N * PA;
    float2 vf[E], vg[E], d[E];
    const int cl = col <= H ? col : H;   // padding lanes of the last tile read a valid column, then use 0
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const float4 q = src[(size_t)(t + m * T) * P1 + col];
        vf[m] = make_float2(q.x, q.y);
        vg[m] = make_float2(q.z, q.w);
        d[m] = da[(t + m * T) * PA + cl];   // dA too before the transforms, whose barriers loads cannot cross
    }
    fft_line<L, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
    fft_line<L, E, LdsCols<C>>(vg, lre[c], lim[c], fresh_index(t), tw);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const float2 dm = col <= H ? d[m] : make_float2(0.f, 0.f);
        vf[m] = mag_adjoint(vf[m], dm.x);
        vg[m] = mag_adjoint(vg[m], dm.y);
    }
    ifft_line<L, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
    ifft_line<L, E, LdsCols<C>>(vg, lre[c], lim[c], fresh_index(t), tw);
    if (col > H) return;
#pragma unroll
    for (int m = 0; m < E; ++m)
        dst[(size_t)(t + m * T) * P1 + col] = make_float4(vf[m].x, vf[m].y, vg[m].x, vg[m].y);
}

// Rotate^T of dg' at scan pixel (qr, qc): sum over output pixels whose
// bilinear sample position p lies within the open unit box around it.
__device__ __forceinline__ float rotate_adjoint(const float* __restrict__ dgp, int N, int qr, int qc,
                                                float ct, float st) {
    const float ox = (float)(qc - N / 2), oy = (float)(qr - N / 2);
    const float cx = ct * ox + st * oy + (float)(N / 2);    // R^T (q - c) + c
    const float cy = -st * ox + ct * oy + (float)(N / 2);
    const float e = fabsf(ct) + fabsf(st) + 1e-3f;
    const int j0 = max(0, (int)ceilf(cx - e)), j1 = min(N - 1, (int)floorf(cx + e));
    const int i0 = max(0, (int)ceilf(cy - e)), i1 = min(N - 1, (int)floorf(cy + e));
    float acc = 0.f;
    for (int i = i0; i <= i1; ++i)
        for (int j = j0; j <= j1; ++j) {
            float py, px;
            rot_src(N, i, j, ct, st, py, px);
            const float ey = fabsf(py - (float)qr), ex = fabsf(px - (float)qc);
            if (ey < 1.f && ex < 1.f) acc += (1.f - ey) * (1.f - ex) * dgp[(size_t)i * N + j];
        }
    return acc;
}

// Rotate^T of dg' on its own, one scan pixel per thread (a gather over the few
// output pixels whose sample position falls within a unit box of it).
template <int N>
__global__ __launch_bounds__(256) void kb_rotate_adj(const float* __restrict__ dgp,
                                                     const float* __restrict__ saved,
                                                     float* __restrict__ dgr) {
    constexpr int TPR = N / kRotTX, TPP = TPR * (N / kRotTY);
    __shared__ float box[kRotBox * kRotBox];
    const int b = blockIdx.x / TPP, tile = blockIdx.x % TPP;
    const int q0 = (tile / TPR) * kRotTY, c0 = (tile % TPR) * kRotTX;
    const float* sv = saved + (size_t)b * FMBYM_SAVED;
    const float ct = sv[kSavedCos], st = sv[kSavedSin];
    const float e = fabsf(ct) + fabsf(st) + 1e-3f;
    // box of the output pixels that any scan pixel of the tile gathers from
    float ymin = 1e30f, ymax = -1e30f, xmin = 1e30f, xmax = -1e30f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float ox = (float)(c0 + (c >> 1) * (kRotTX - 1) - N / 2);
        const float oy = (float)(q0 + (c & 1) * (kRotTY - 1) - N / 2);
        const float cx = ct * ox + st * oy + (float)(N / 2);
        const float cy = -st * ox + ct * oy + (float)(N / 2);
        ymin = fminf(ymin, cy); ymax = fmaxf(ymax, cy);
        xmin = fminf(xmin, cx); xmax = fmaxf(xmax, cx);
    }
    const int by0 = (int)floorf(ymin - e) - 1, bx0 = (int)floorf(xmin - e) - 1;
    const int bh = min(kRotBox, (int)floorf(ymax + e) + 2 - by0), bw = min(kRotBox, (int)floorf(xmax + e) + 2 - bx0);
    stage_box<false, false>(box, dgp + (size_t)b * N * N, nullptr, nullptr, N, by0, bx0, bh, bw);
    __syncthreads();
    // sample-position offsets of the 3 x 3 window, the same for every pixel of the pair
    float ky[3][3], kx[3][3];
#pragma unroll
    for (int di = -1; di <= 1; ++di)
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
            ky[di + 1][dj + 1] = (float)di * ct + (float)dj * st;
            kx[di + 1][dj + 1] = (float)dj * ct - (float)di * st;
        }
#pragma unroll
    for (int k = 0; k < kRotTY * kRotTX / 256; ++k) {
        const int p = threadIdx.x + 256 * k;
        const int qr = q0 + p / kRotTX, qc = c0 + p % kRotTX;
        // the gather of rotate_adjoint, reading the box: every output pixel whose
        // sample position lies within the unit box of q is within one lattice step
        // of round(R^T (q - c) + c), so a fixed 3 x 3 window in row order visits
        // the same contributors in the same order.  The window lies inside the
        // box (its margins cover a rounding step and a lattice step), and the
        // box holds zeros for output positions outside the scan.
        const float ox = (float)(qc - N / 2), oy = (float)(qr - N / 2);
        const float cx = ct * ox + st * oy + (float)(N / 2);
        const float cy = -st * ox + ct * oy + (float)(N / 2);
        const int ic = (int)rintf(cy), jc = (int)rintf(cx);
        float py0, px0;
        rot_src(N, ic, jc, ct, st, py0, px0);
        py0 -= (float)qr;   // offsets of the window centre's sample position from q
        px0 -= (float)qc;
        const int r0 = ic - 1 - by0, c0w = jc - 1 - bx0;
        const bool inside = (unsigned)r0 <= (unsigned)(bh - 3) && (unsigned)c0w <= (unsigned)(bw - 3);
        const float* w = box + (inside ? r0 * kRotBox + c0w : 0);
        float acc = 0.f;
#pragma unroll
        for (int di = 0; di < 3; ++di)
#pragma unroll
            for (int dj = 0; dj < 3; ++dj) {
                // bilinear weight max(0, 1 - |e_y|) max(0, 1 - |e_x|): zero outside the unit box
                const float wy = fmaxf(0.f, 1.f - fabsf(py0 + ky[di][dj]));
                const float wx = fmaxf(0.f, 1.f - fabsf(px0 + kx[di][dj]));
                acc += wy * wx * w[di * kRotBox + dj];
            }
        if (!inside) acc = 0.f;   // unreachable by the box bounds; keeps every LDS read in the box
        dgr[(size_t)b * N * N + (size_t)qr * N + qc] = acc;
    }
}

// Inverse row DFT of the rotation adjoint: df_w[x] = Re sum_{k <= n/2} Q[k] e^{+2 pi i k x / n},
// formed as the inverse DFT of the Hermitian extension (Re Q at k = 0, n/2;
// Q/2 and conj(Q)/2 elsewhere), f and g paired in one transform.  Adds the
// translation-stage terms (Rotate^T gathered here), then the window and mask
// adjoints.
template <int N>
__global__ __launch_bounds__(256) void kb_rows_final(
    const float4* __restrict__ r1, const float* __restrict__ df2, const float* __restrict__ dgr,
    const float* __restrict__ f, const float* __restrict__ g, const float* __restrict__ mf,
    const float* __restrict__ mg, const float* __restrict__ hann, const float2* __restrict__ tw,
    const float* __restrict__ saved, float* __restrict__ d_f, float* __restrict__ d_g,
    float* __restrict__ d_mf, float* __restrict__ d_mg, int win, int win2) {
    constexpr int L = N, T = L / kEb, LPB = 256 / T, H = N / 2, P1 = pitch_rows1(N);
    __shared__ float lre[LPB][LdsRows<L>::words(L)];
    __shared__ float lim[LPB][LdsRows<L>::words(L)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int grow = blockIdx.x * LPB + line;
    const int b = grow / N, i = grow % N;
    const float4* q = r1 + (size_t)grow * P1;
    float2 v[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) {   // one load at the stored index, then selects (no branches)
        const int k = t + m * T;
        const float4 a = q[k <= H ? k : N - k];          // (Qf, Qg)
        float2 z;
        if (k == 0 || k == H) z = make_float2(a.x, a.z);
        else if (k < H) z = make_float2(0.5f * (a.x - a.w), 0.5f * (a.y + a.z));
        else z = make_float2(0.5f * (a.x + a.w), 0.5f * (a.z - a.y));
        v[m] = z;
    }
    const size_t base = (size_t)b * N * N;
    float s2fv[kEb], s2gv[kEb];   // loaded before the transform, whose barriers the loads cannot cross
#pragma unroll
    for (int m = 0; m < kEb; ++m) {
        const size_t o = base + (size_t)i * N + t + m * T;
        s2fv[m] = df2[o];
        s2gv[m] = dgr[o];
    }
    ifft_line<L, kEb>(v, lre[line], lim[line], t, tw);
    const float hi = win ? hann[i] : 1.f;
#pragma unroll
    for (int m = 0; m < kEb; ++m) {
        const int x = t + m * T;
        const size_t o = base + (size_t)i * N + x;
        const float w = win ? hi * hann[x] : 1.f;
        const float w2 = win2 ? w : 1.f;
        const float s2f = s2fv[m];
        const float s2g = s2gv[m];
        // stage 1 always sees the window; stage 2 sees it unless unwindowed
        const float dft = w * v[m].x + w2 * s2f;
        const float dgt = w * v[m].y + w2 * s2g;
        if (mf) {
            d_f[o] = mf[o] * dft;
            d_mf[o] = f[o] * dft;
        } else {
            d_f[o] = dft;
        }
        if (mg) {
            d_g[o] = mg[o] * dgt;
            d_mg[o] = g[o] * dgt;
        } else {
            d_g[o] = dgt;
        }
    }
}

// ------------------------------------------------------------------ launcher

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BwdLayout {
    size_t rf, rdc, df2, dgp, dpol, dth, dspec, jac, total;
};

// The stage-1 recomputation reuses the forward layout's first two regions;
// the adjoint's own buffers follow it.
static BwdLayout bwd_layout(const fmbym_params& p, int batch) {
    const size_t n = p.n, B = batch;
    const FwdLayout f = fwd_layout(p, batch);
    BwdLayout L{};
    size_t off = f.total;
    L.rf = off;
    off = al256(off + B * n * (size_t)pitch_rows2(p.n) * sizeof(float4));
    L.rdc = off;
    off = al256(off + B * n * (size_t)pitch_lag(p.n) * sizeof(float2));
    L.df2 = off;
    off = al256(off + B * n * n * sizeof(float));
    L.dgp = off;
    off = al256(off + B * n * n * sizeof(float));
    L.dpol = off;
    off = al256(off + B * (size_t)p.n_r * p.n_theta * sizeof(float2));
    L.dth = off;
    off = al256(off + B * n * sizeof(float));
    L.dspec = off;
    off = al256(off + B * (size_t)p.n_theta * sizeof(float2));
    L.jac = off;
    off = al256(off + B * n * n * sizeof(float));
    L.total = off;
    return L;
}

size_t bwd_workspace(const fmbym_params& p, int batch) { return bwd_layout(p, batch).total; }

template <int N, int NT>
static void launch_bwd_polar(const Plan& pl, int B, const float2* A, const float2* pspec, const float2* dspec,
                             float2* dpol, hipStream_t s) {
    const int nrb = radius_blocks(pl.p.n_r, pl.p.n_theta);
    const int total = B * nrb;
    if (pspec)
        FMBYM_LAUNCH(kKBPolar, (kb_polar_keep<NT, N>), dim3(((total + 7) / 8) * 8), dim3(256), s, pspec,
                     pl.twiddle, dspec, dpol, pl.p.n_r, B);
    else
        FMBYM_LAUNCH(kKBPolar, (kb_polar<NT, N>), dim3(((total + 7) / 8) * 8), dim3(256), s, A, pl.twiddle,
                     dspec, dpol, pl.p.n_r, B);
}

template <int NT>
static void launch_dtheta(const Plan& pl, int B, int ppb, const float* dth, const float* c_theta,
                          const float* saved, const float* d_pose, float2* dspec, hipStream_t s) {
    FMBYM_LAUNCH(kKBDtheta, kb_dtheta<NT>, dim3(B), dim3(NT / kEb), s, dth, ppb, c_theta, saved, d_pose,
                 pl.twiddle, pl.p.temp_theta, dspec);
}

// Column-tile widths from the plan's tuning (same arithmetic for every width).
template <int N, int C>
static void launch_cols_xy_c(const Plan& pl, int B, const float4* rows2, float4* rf, const float2* rdc,
                             hipStream_t s) {
    constexpr int T2 = pad2(N) / kE2;
    const int total2 = B * ((pad2(N) / 2) / C + 1);
    FMBYM_LAUNCH(kKBColsXy, (kb_cols_xy<N, C>), dim3(((total2 + 7) / 8) * 8), dim3(C * T2), s, rows2, rf,
                 rdc, pl.twiddle3, B);
}

template <int N>
static void launch_cols_xy(const Plan& pl, int B, const float4* rows2, float4* rf, const float2* rdc,
                           hipStream_t s) {
    switch (pl.tune.cols_xy) {
        case 4: launch_cols_xy_c<N, 4>(pl, B, rows2, rf, rdc, s); break;
        case 8: launch_cols_xy_c<N, 8>(pl, B, rows2, rf, rdc, s); break;
        default: launch_cols_xy_c<N, 16>(pl, B, rows2, rf, rdc, s); break;
    }
}

template <int N, int C, int E>
static void launch_cols_mag_ce(const Plan& pl, int B, const float4* r1, float4* out, const float2* dA,
                               hipStream_t s) {
    const int tiles_mag = B * ((N / 2) / C + 1);
    if constexpr (C * N / E <= 1024)
        FMBYM_LAUNCH(kKBColsMag, (kb_cols_mag<N, C, E>), dim3(((tiles_mag + 7) / 8) * 8), dim3(C * N / E), s, r1,
                     out, dA, pl.twiddle, B);
}

// The radix plan of these column lines (elements per thread, 8 or 4) is the plan's tuning.
template <int N, int C>
static void launch_cols_mag_c(const Plan& pl, int B, const float4* r1, float4* out, const float2* dA,
                              hipStream_t s) {
    if (pl.tune.radix_mag == 4) launch_cols_mag_ce<N, C, 4>(pl, B, r1, out, dA, s);
    else launch_cols_mag_ce<N, C, 8>(pl, B, r1, out, dA, s);
}

template <int N>
static void launch_cols_mag(const Plan& pl, int B, const float4* r1, float4* out, const float2* dA,
                            hipStream_t s) {
    switch (pl.tune.cols_mag) {
        case 4: launch_cols_mag_c<N, 4>(pl, B, r1, out, dA, s); break;
        case 8: launch_cols_mag_c<N, 8>(pl, B, r1, out, dA, s); break;
        default: launch_cols_mag_c<N, 16>(pl, B, r1, out, dA, s); break;
    }
}

template <int N>
static int launch_bwd_n(const Plan& pl, int B, const float* f, const float* g, const float* mf,
                        const float* mg, const float* c_theta, const float* c_xy, const float* saved,
                        const float* d_pose, float* d_f, float* d_g, float* d_mf, float* d_mg,
                        char* ws, hipStream_t s, const Keep* keep) {
    const FwdLayout fl = fwd_layout(pl.p, B);
    const BwdLayout bl = bwd_layout(pl.p, B);
    float4* rf = (float4*)(ws + bl.rf);
    float2* rdc = (float2*)(ws + bl.rdc);
    float* df2 = (float*)(ws + bl.df2);
    float* dgp = (float*)(ws + bl.dgp);
    float2* dpol = (float2*)(ws + bl.dpol);
    float* dth = (float*)(ws + bl.dth);
    float2* dspec = (float2*)(ws + bl.dspec);
    // With keep, the forward's g', J, stage-1 spectra and stage-2 rows are read
    // from the state (never written); otherwise they are recomputed into the
    // workspace.  Rotate^T dg', dA and the |F| adjoint's columns go to the workspace.
    float* jac = keep ? keep->jac : (float*)(ws + bl.jac);
    float* dgr = (float*)(ws + fl.grot);    // Rotate^T dg' (without keep, g' before it)
    const float* gr = keep ? keep->gr : dgr;
    float4* r1w = (float4*)(ws + fl.r1r2);
    const float4* r1 = keep ? keep->r1 : r1w;
    float2* magw = (float2*)(ws + fl.mag_r3);
    const float2* mag = magw;                 // recomputed |F| (unused with keep: kb_polar reads the spectra)
    const float4* rows2 = keep ? keep->r2 : rf;
    const int win = (pl.p.flags & FMBYM_HANN) ? 1 : 0;
    const int win2 = (win && !(pl.p.flags & FMBYM_XY_UNWINDOWED)) ? 1 : 0;

    // translation-stage adjoint
    constexpr int LPB2 = rows2_lines(N);
    const int dc_blocks = B * (N / 2) / LPB2;
    if (!keep) {
        // g' (and J) and the stage-2 rows again, by the forward's own kernels
        launch_rotate(pl, B, g, mg, saved, dgr, jac, win2, s, nullptr);
        launch_rows2(pl, B, f, g, mf, mg, dgr, rf, win2, s);
    }
    FMBYM_LAUNCH(kKBRowsFwd2, kb_rows_fwd2<N>, dim3(dc_blocks), dim3(256), s, pl.twiddle3, saved, c_xy,
                 d_pose, rdc, pl.p.temp_xy, pl.p.delta_xy);
    launch_cols_xy<N>(pl, B, rows2, rf, rdc, s);
    FMBYM_LAUNCH(kKBRowsXy, kb_rows_xy<N>, dim3(B * N / LPB2), dim3(256), s, rf, jac, pl.twiddle3, df2,
                 dgp, dth);
    const int ppb = N / LPB2;
    switch (pl.p.n_theta) {
        case 16: launch_dtheta<16>(pl, B, ppb, dth, c_theta, saved, d_pose, dspec, s); break;
        case 32: launch_dtheta<32>(pl, B, ppb, dth, c_theta, saved, d_pose, dspec, s); break;
        case 64: launch_dtheta<64>(pl, B, ppb, dth, c_theta, saved, d_pose, dspec, s); break;
        case 128: launch_dtheta<128>(pl, B, ppb, dth, c_theta, saved, d_pose, dspec, s); break;
        case 256: launch_dtheta<256>(pl, B, ppb, dth, c_theta, saved, d_pose, dspec, s); break;
        case 512: launch_dtheta<512>(pl, B, ppb, dth, c_theta, saved, d_pose, dspec, s); break;
        case 1024: launch_dtheta<1024>(pl, B, ppb, dth, c_theta, saved, d_pose, dspec, s); break;
        default: return FMBYM_EUNSUPPORTED;
    }

    // rotation-stage adjoint: recompute the stage-1 spectra, then transpose
    if (!keep) launch_stage1_spectra(pl, B, f, g, mf, mg, r1w, magw, s);
    switch (pl.p.n_theta) {
        case 16: launch_bwd_polar<N, 16>(pl, B, mag, keep ? keep->pspec : nullptr, dspec, dpol, s); break;
        case 32: launch_bwd_polar<N, 32>(pl, B, mag, keep ? keep->pspec : nullptr, dspec, dpol, s); break;
        case 64: launch_bwd_polar<N, 64>(pl, B, mag, keep ? keep->pspec : nullptr, dspec, dpol, s); break;
        case 128: launch_bwd_polar<N, 128>(pl, B, mag, keep ? keep->pspec : nullptr, dspec, dpol, s); break;
        case 256: launch_bwd_polar<N, 256>(pl, B, mag, keep ? keep->pspec : nullptr, dspec, dpol, s); break;
        case 512: launch_bwd_polar<N, 512>(pl, B, mag, keep ? keep->pspec : nullptr, dspec, dpol, s); break;
        case 1024: launch_bwd_polar<N, 1024>(pl, B, mag, keep ? keep->pspec : nullptr, dspec, dpol, s); break;
        default: return FMBYM_EUNSUPPORTED;
    }
    float2* dA = magw;                  // (recomputed magnitudes are dead after kb_polar)
    const int dmag_work = pl.dmag_nparts * ((B + kDmagPairs - 1) / kDmagPairs);
    FMBYM_LAUNCH(kKBDmag, kb_dmag, dim3(((dmag_work + 7) / 8) * 8), dim3(256), s, pl.csr_ptr, pl.csr_col,
                 pl.csr_val, pl.csr_dst, pl.dmag_part, dpol, dA, N, pl.p.n_r, pl.p.n_theta, B, pl.dmag_nparts);
    launch_cols_mag<N>(pl, B, r1, r1w, dA, s);
    FMBYM_LAUNCH(kKBRotateAdj, kb_rotate_adj<N>, dim3(B * (N / kRotTY) * (N / kRotTX)), dim3(256), s, dgp,
                 saved, dgr);
    constexpr int T1 = N / kEb, LPB1 = 256 / T1;
    FMBYM_LAUNCH(kKBRowsFinal, kb_rows_final<N>, dim3(B * N / LPB1), dim3(256), s, r1w, df2, dgr, f, g, mf,
                 mg, pl.hann, pl.twiddle, saved, d_f, d_g, d_mf, d_mg, win, win2);
    return FMBYM_OK;
}

int launch_backward(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                    const float* mg, const float* /*pose*/, const float* c_theta, const float* c_xy,
                    const float* saved, const float* d_pose, float* d_f, float* d_g, float* d_mf,
                    float* d_mg, char* ws, hipStream_t s, const Keep* keep) {
    switch (pl.p.n) {
        case 128:
            return launch_bwd_n<128>(pl, batch, f, g, mf, mg, c_theta, c_xy, saved, d_pose, d_f, d_g,
                                     d_mf, d_mg, ws, s, keep);
        case 256:
            return launch_bwd_n<256>(pl, batch, f, g, mf, mg, c_theta, c_xy, saved, d_pose, d_f, d_g,
                                     d_mf, d_mg, ws, s, keep);
        case 512:
            return launch_bwd_n<512>(pl, batch, f, g, mf, mg, c_theta, c_xy, saved, d_pose, d_f, d_g,
                                     d_mf, d_mg, ws, s, keep);
        default: return FMBYM_EUNSUPPORTED;
    }
}

}  // namespace fmbym
