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
//   kb_rows_fwd2   rows of f2 and g' (2n-padded) and of dc_xy, paired complex FFTs
//   kb_cols_xy     column FFTs, conj(DC) G' and F DC, inverse columns (rows < n kept)
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

// Blocks [0, B n / LPB) transform rows of f2 + i g'; the rest transform pairs
// of dc_xy lag rows.  Outputs are packed half spectra of the 2n-point rows.
template <int N>
__global__ __launch_bounds__(256) void kb_rows_fwd2(
    const float* __restrict__ f, const float* __restrict__ g, const float* __restrict__ mf,
    const float* __restrict__ mg, const float* __restrict__ hann, const float2* __restrict__ tw,
    const float* __restrict__ saved, const float* __restrict__ c_xy, const float* __restrict__ d_pose,
    float2* __restrict__ rf, float2* __restrict__ rg, float2* __restrict__ rdc, int win, int batch,
    float temp, float delta) {
    constexpr int L = 2 * N, T = L / kEb, LPB = 256 / T;
    __shared__ float lre[LPB][lds_line_words(L)];
    __shared__ float lim[LPB][lds_line_words(L)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int nscan_blocks = batch * N / LPB;
    float2 v[kEb];
    float2 *o1, *o2;
    if ((int)blockIdx.x < nscan_blocks) {
        const int grow = blockIdx.x * LPB + line;
        const int b = grow / N, i = grow % N;
        const size_t base = (size_t)b * N * N;
        const float* sv = saved + (size_t)b * FMBYM_SAVED;
        const float ct = sv[kSavedCos], st = sv[kSavedSin];
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            const int x = t + m * T;
            if (m < kEb / 2) {
                const float a = scan_w(f + base, mf ? mf + base : nullptr, hann, N, i, x, win);
                const float c = rotate_sample(g + base, mg ? mg + base : nullptr, hann, N, i, x, ct, st, win);
                v[m] = make_float2(a, c);
            } else {
                v[m] = make_float2(0.f, 0.f);
            }
        }
        o1 = rf + ((size_t)b * N + i) * N;
        o2 = rg + ((size_t)b * N + i) * N;
    } else {
        const int gl = (blockIdx.x - nscan_blocks) * LPB + line;   // lag-row pair
        const int b = gl / (N / 2), q = gl % (N / 2);
        const XyAdj adj = make_xy_adj(saved + (size_t)b * FMBYM_SAVED, d_pose + b * 3, temp, delta);
        const float* c1 = c_xy + ((size_t)b * N + 2 * q) * N;
        const float* c2 = c1 + N;
        const int sy1 = 2 * q - N / 2, sy2 = sy1 + 1;
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            const int x = t + m * T;                 // padded position s_x mod 2n
            if (m < kEb / 4 || m >= 3 * kEb / 4) {
                const int sx = m < kEb / 4 ? x : x - L;
                const int j = sx + N / 2;
                v[m] = make_float2(adj(c1[j], sx, sy1), adj(c2[j], sx, sy2));
            } else {
                v[m] = make_float2(0.f, 0.f);
            }
        }
        o1 = rdc + ((size_t)b * N + 2 * q) * N;
        o2 = o1 + N;
    }
    fft_line<L, kEb>(v, lre[line], lim[line], t, tw);
    float2 mir[kEb];
    mirror_line<L, kEb>(v, mir, lre[line], lim[line], t);
#pragma unroll
    for (int m = 0; m < kEb / 2; ++m) {
        const int k = t + m * T;
        float2 X = split_x(v[m], mir[m]);
        float2 Y = split_y(v[m], mir[m]);
        if (k == 0) {
            const float2 Xn = split_x(v[kEb / 2], mir[kEb / 2]);
            const float2 Yn = split_y(v[kEb / 2], mir[kEb / 2]);
            X = make_float2(X.x, Xn.x);
            Y = make_float2(Y.x, Yn.x);
        }
        o1[k] = X;
        o2[k] = Y;
    }
}

// Column pass of the translation adjoint.  Column col of the packed half
// spectra (2n-point transforms along the padded rows); writes the n data rows
// of the two inverse transforms in place of the F and G' inputs.
template <int N, int C>
__global__ __launch_bounds__(C * 2 * N / kEb) void kb_cols_xy(float2* __restrict__ rf,
                                                              float2* __restrict__ rg,
                                                              const float2* __restrict__ rdc,
                                                              const float2* __restrict__ tw,
                                                              int batch) {
    constexpr int L = 2 * N, T = L / kEb, TILES = N / C;
    __shared__ float lre[C][lds_line_words(L)];
    __shared__ float lim[C][lds_line_words(L)];
    const int total = batch * TILES;
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= total) return;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int tile = work % TILES, b = work / TILES;
    const int col = tile * C + c;
    float2* sf = rf + (size_t)b * N * N;
    float2* sg = rg + (size_t)b * N * N;
    const float2* sd = rdc + (size_t)b * N * N;
    float2 vf[kEb], vg[kEb], vd[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) {
        const int n = t + m * T;
        if (m < kEb / 2) {
            vf[m] = sf[(size_t)n * N + col];
            vg[m] = sg[(size_t)n * N + col];
        } else {
            vf[m] = vg[m] = make_float2(0.f, 0.f);
        }
        // dc lag row o holds s_y = o - n/2, placed at padded row s_y mod 2n
        if (m < kEb / 4) vd[m] = sd[(size_t)(n + N / 2) * N + col];
        else if (m >= 3 * kEb / 4) vd[m] = sd[(size_t)(n - 3 * N / 2) * N + col];
        else vd[m] = make_float2(0.f, 0.f);
    }
    fft_line<L, kEb>(vd, lre[c], lim[c], t, tw);
    fft_line<L, kEb>(vf, lre[c], lim[c], t, tw);
    fft_line<L, kEb>(vg, lre[c], lim[c], t, tw);
    float2 x1[kEb], x2[kEb];
    if (tile == 0) {   // packed DC / Nyquist column: split, multiply, repack
        float2 mf_[kEb], mg_[kEb], md_[kEb];
        mirror_line<L, kEb>(vf, mf_, lre[c], lim[c], t);
        mirror_line<L, kEb>(vg, mg_, lre[c], lim[c], t);
        mirror_line<L, kEb>(vd, md_, lre[c], lim[c], t);
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            if (c == 0) {
                const float2 f0 = split_x(vf[m], mf_[m]), fn = split_y(vf[m], mf_[m]);
                const float2 g0 = split_x(vg[m], mg_[m]), gn = split_y(vg[m], mg_[m]);
                const float2 d0 = split_x(vd[m], md_[m]), dn = split_y(vd[m], md_[m]);
                const float2 a0 = cmulcj(d0, g0), an = cmulcj(dn, gn);
                const float2 b0 = cmul(f0, d0), bn = cmul(fn, dn);
                x1[m] = make_float2(a0.x - an.y, a0.y + an.x);
                x2[m] = make_float2(b0.x - bn.y, b0.y + bn.x);
            } else {
                x1[m] = cmulcj(vd[m], vg[m]);
                x2[m] = cmul(vf[m], vd[m]);
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            x1[m] = cmulcj(vd[m], vg[m]);
            x2[m] = cmul(vf[m], vd[m]);
        }
    }
    ifft_line<L, kEb>(x1, lre[c], lim[c], t, tw);
    ifft_line<L, kEb>(x2, lre[c], lim[c], t, tw);
#pragma unroll
    for (int m = 0; m < kEb / 2; ++m) {
        const int n = t + m * T;
        sf[(size_t)n * N + col] = x1[m];
        sg[(size_t)n * N + col] = x2[m];
    }
}

__device__ __forceinline__ float2 herm_get2(const float2* __restrict__ row, int N, int k) {
    if (k == 0) return make_float2(row[0].x, 0.f);
    if (k == N) return make_float2(row[0].y, 0.f);
    if (k < N) return row[k];
    return cconj(row[2 * N - k]);
}

// Inverse rows of the translation adjoint -> df2, dg' (rows < n, columns < n),
// and the Rotate-path heading gradient dtheta_2 summed per block.
template <int N>
__global__ __launch_bounds__(256) void kb_rows_xy(const float2* __restrict__ q1,
                                                  const float2* __restrict__ q2,
                                                  const float* __restrict__ g,
                                                  const float* __restrict__ mg,
                                                  const float* __restrict__ hann,
                                                  const float2* __restrict__ tw,
                                                  const float* __restrict__ saved,
                                                  float* __restrict__ df2, float* __restrict__ dgp,
                                                  float* __restrict__ dth_part, int win) {
    constexpr int L = 2 * N, T = L / kEb, LPB = 256 / T, PPB = N / LPB;
    __shared__ float lre[LPB][lds_line_words(L)];
    __shared__ float lim[LPB][lds_line_words(L)];
    __shared__ float red[256];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int grow = blockIdx.x * LPB + line;
    const int b = grow / N, i = grow % N;
    const float2* r1 = q1 + ((size_t)b * N + i) * N;
    const float2* r2 = q2 + ((size_t)b * N + i) * N;
    float2 v[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) {
        const int k = t + m * T;
        const float2 h1 = herm_get2(r1, N, k), h2 = herm_get2(r2, N, k);
        v[m] = make_float2(h1.x - h2.y, h1.y + h2.x);
    }
    ifft_line<L, kEb>(v, lre[line], lim[line], t, tw);
    const float scale = 1.f / ((float)L * (float)L);
    const size_t base = (size_t)b * N * N;
    const float* sv = saved + (size_t)b * FMBYM_SAVED;
    const float ct = sv[kSavedCos], st = sv[kSavedSin];
    const float* gb = g + base;
    const float* mgb = mg ? mg + base : nullptr;
    float dth = 0.f;
#pragma unroll
    for (int m = 0; m < kEb / 2; ++m) {
        const int x = t + m * T;
        const float a = v[m].x * scale, d = v[m].y * scale;
        df2[base + (size_t)i * N + x] = a;
        dgp[base + (size_t)i * N + x] = d;
        // d g'(i, x) / d theta through the bilinear sample position
        float py, px;
        rot_src(N, i, x, ct, st, py, px);
        const float fy = floorf(py), fx = floorf(px);
        const float wy = py - fy, wx = px - fx;
        const int y0 = (int)fy, x0 = (int)fx;
        float G[2][2];
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int r = y0 + dy, cc = x0 + dx;
                G[dy][dx] = (r >= 0 && r < N && cc >= 0 && cc < N) ? scan_w(gb, mgb, hann, N, r, cc, win) : 0.f;
            }
        const float gx = (1.f - wy) * (G[0][1] - G[0][0]) + wy * (G[1][1] - G[1][0]);
        const float gy = (1.f - wx) * (G[1][0] - G[0][0]) + wx * (G[1][1] - G[0][1]);
        const float yx = (float)(x - N / 2), yy = (float)(i - N / 2);
        dth += d * (gx * (-st * yx - ct * yy) + gy * (ct * yx - st * yy));
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
    __shared__ float lre[lds_line_words(L)];
    __shared__ float lim[lds_line_words(L)];
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
// then the angular adjoint: dP_f = IDFT(conj(D) Pg^) / n_r, dP_g = IDFT(Pf^ D) / n_r.
template <int NT, int N>
__global__ __launch_bounds__(256) void kb_polar(const float* __restrict__ A,
                                                const float2* __restrict__ tw,
                                                const float2* __restrict__ dspec,
                                                float* __restrict__ dpol, int n_r, int batch) {
    constexpr int L = NT, T = L / kEb, LPB = 256 / T, PASSES = (kRadiiPerBlock + LPB - 1) / LPB;
    __shared__ float lre[LPB][lds_line_words(L)];
    __shared__ float lim[LPB][lds_line_words(L)];
    const int nrb = (n_r + kRadiiPerBlock - 1) / kRadiiPerBlock;
    const int total = batch * nrb;
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= total) return;
    const int b = work / nrb, rb = work % nrb;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const float* Af = A + (size_t)(b * 2 + 0) * N * mag_pitch(N);
    const float* Ag = A + (size_t)(b * 2 + 1) * N * mag_pitch(N);
    float2 D[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) D[m] = dspec[(size_t)b * NT + t + m * T];
    const float scale = 1.f / ((float)n_r * (float)NT);
    for (int pass = 0; pass < PASSES; ++pass) {
        const int slot = pass * LPB + line;
        const int rad = rb * kRadiiPerBlock + slot;
        const bool live = slot < kRadiiPerBlock && rad < n_r;
        float2 v[kEb];
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            if (live) {
                float uy, ux;
                polar_uv(tw, N, n_r, NT, rad, t + m * T, uy, ux);
                v[m] = make_float2(mag_sample(Af, N, uy, ux), mag_sample(Ag, N, uy, ux));
            } else {
                v[m] = make_float2(0.f, 0.f);
            }
        }
        fft_line<L, kEb>(v, lre[line], lim[line], t, tw);
        float2 mir[kEb];
        mirror_line<L, kEb>(v, mir, lre[line], lim[line], t);
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            const float2 Pf = split_x(v[m], mir[m]), Pg = split_y(v[m], mir[m]);
            const float2 a = cmulcj(D[m], Pg);     // conj(D) Pg
            const float2 c = cmul(Pf, D[m]);
            v[m] = make_float2(a.x - c.y, a.y + c.x);   // a + i c
        }
        ifft_line<L, kEb>(v, lre[line], lim[line], t, tw);
        if (live) {
            float* of = dpol + ((size_t)(b * 2 + 0) * n_r + rad) * NT;
            float* og = dpol + ((size_t)(b * 2 + 1) * n_r + rad) * NT;
#pragma unroll
            for (int m = 0; m < kEb; ++m) {
                of[t + m * T] = v[m].x * scale;
                og[t + m * T] = v[m].y * scale;
            }
        }
    }
}

// dA = band * Cart2Pol^T dP over the half-plane bins, from the plan's CSR
// transpose of the polar gather.  Bins outside the band get 0 without a gather.
// blockIdx.y walks groups of kDmagGroup (pair, scan) planes that share the
// block's CSR rows through the cache.
constexpr int kDmagGroup = 8;
__global__ __launch_bounds__(256) void kb_dmag(const int* __restrict__ ptr, const int* __restrict__ col,
                                               const float* __restrict__ val,
                                               const float* __restrict__ dpol, float* __restrict__ dA,
                                               int n, int n_r, int n_theta, int planes, int band_on,
                                               int lo2, int hi2) {
    const int h1 = n / 2 + 1;
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    if (bin >= n * h1) return;
    const int ky = bin / h1, kx = bin % h1;
    const int kys = ky < n / 2 ? ky : ky - n;
    const int r2 = kys * kys + kx * kx;
    const bool in_band = !band_on || (r2 >= lo2 && r2 <= hi2);
    const int e0 = ptr[bin], e1 = ptr[bin + 1];
    const size_t pstride = (size_t)n_r * n_theta;
    const int p0 = blockIdx.y * kDmagGroup, p1 = min(planes, p0 + kDmagGroup);
    for (int ps = p0; ps < p1; ++ps) {
        float acc = 0.f;
        if (in_band) {
            const float* src = dpol + (size_t)ps * pstride;
            for (int e = e0; e < e1; ++e) acc += val[e] * src[col[e]];
        }
        dA[((size_t)ps * n + ky) * mag_pitch(n) + kx] = acc;
    }
}

__device__ __forceinline__ float2 mag_adjoint(float2 F, float dA) {
    const float a = sqrtf(F.x * F.x + F.y * F.y);
    if (!(a > 0.f)) return make_float2(0.f, 0.f);
    const float s = dA / a;
    return make_float2(F.x * s, F.y * s);
}


// Column pass of the rotation adjoint, in place over the stage-1 row spectra:
// column DFTs again, dF = dA F / |F| (dA already carries the band gain), and
// the unnormalised inverse column DFT.  For the packed DC/Nyquist column only
// the real parts of the inverse are needed: the inverse of the Hermitian part
// of each, both through one transform.
template <int N, int C>
__global__ __launch_bounds__(C * N / kEb) void kb_cols_mag(float2* __restrict__ r1,
                                                           const float* __restrict__ dA,
                                                           const float2* __restrict__ tw) {
    constexpr int L = N, T = L / kEb, H = N / 2, TILES = H / C, P = mag_pitch(N);
    __shared__ float lre[C][lds_line_words(L)];
    __shared__ float lim[C][lds_line_words(L)];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int tile = blockIdx.x % TILES, bs = blockIdx.x / TILES;
    const int col = tile * C + c;
    float2* src = r1 + (size_t)bs * N * H;
    const float* da = dA + (size_t)bs * N * P;
    float2 v[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) v[m] = src[(size_t)(t + m * T) * H + col];
    fft_line<L, kEb>(v, lre[c], lim[c], t, tw);
    if (tile == 0) {
        float2 mir[kEb];
        mirror_line<L, kEb>(v, mir, lre[c], lim[c], t);
        float2 d0[kEb], dn[kEb];
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            const int ky = t + m * T;
            if (c == 0) {
                d0[m] = mag_adjoint(split_x(v[m], mir[m]), da[ky * P + 0]);
                dn[m] = mag_adjoint(split_y(v[m], mir[m]), da[ky * P + H]);
            } else {
                d0[m] = mag_adjoint(v[m], da[ky * P + col]);
                dn[m] = make_float2(0.f, 0.f);
            }
        }
        float2 m0[kEb], mn[kEb];
        mirror_line<L, kEb>(d0, m0, lre[c], lim[c], t);
        mirror_line<L, kEb>(dn, mn, lre[c], lim[c], t);
#pragma unroll
        for (int m = 0; m < kEb; ++m) {
            if (c == 0) {
                const float2 s0 = make_float2(0.5f * (d0[m].x + m0[m].x), 0.5f * (d0[m].y - m0[m].y));
                const float2 sn = make_float2(0.5f * (dn[m].x + mn[m].x), 0.5f * (dn[m].y - mn[m].y));
                v[m] = make_float2(s0.x - sn.y, s0.y + sn.x);
            } else {
                v[m] = d0[m];
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < kEb; ++m) v[m] = mag_adjoint(v[m], da[(t + m * T) * P + col]);
    }
    ifft_line<L, kEb>(v, lre[c], lim[c], t, tw);
#pragma unroll
    for (int m = 0; m < kEb; ++m) src[(size_t)(t + m * T) * H + col] = v[m];
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

// Inverse row DFT of the rotation adjoint (Re part via the Hermitian
// extension, f and g paired), plus the translation-stage terms, then the
// window and mask adjoints.
template <int N>
__global__ __launch_bounds__(256) void kb_rows_final(
    const float2* __restrict__ r1, const float* __restrict__ df2, const float* __restrict__ dgp,
    const float* __restrict__ f, const float* __restrict__ g, const float* __restrict__ mf,
    const float* __restrict__ mg, const float* __restrict__ hann, const float2* __restrict__ tw,
    const float* __restrict__ saved, float* __restrict__ d_f, float* __restrict__ d_g,
    float* __restrict__ d_mf, float* __restrict__ d_mg, int win, int win2) {
    constexpr int L = N, T = L / kEb, LPB = 256 / T, H = N / 2;
    __shared__ float lre[LPB][lds_line_words(L)];
    __shared__ float lim[LPB][lds_line_words(L)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int grow = blockIdx.x * LPB + line;
    const int b = grow / N, i = grow % N;
    const float2* qf = r1 + ((size_t)(b * 2 + 0) * N + i) * H;
    const float2* qg = r1 + ((size_t)(b * 2 + 1) * N + i) * H;
    float2 v[kEb];
#pragma unroll
    for (int m = 0; m < kEb; ++m) {
        const int k = t + m * T;
        float2 z;
        if (k == 0) z = make_float2(qf[0].x, qg[0].x);
        else if (k == H) z = make_float2(qf[0].y, qg[0].y);
        else if (k < H) {
            const float2 a = qf[k], c = qg[k];
            z = make_float2(0.5f * (a.x - c.y), 0.5f * (a.y + c.x));
        } else {
            const float2 a = qf[N - k], c = qg[N - k];
            z = make_float2(0.5f * (a.x + c.y), 0.5f * (c.x - a.y));
        }
        v[m] = z;
    }
    ifft_line<L, kEb>(v, lre[line], lim[line], t, tw);
    const size_t base = (size_t)b * N * N;
    const float* sv = saved + (size_t)b * FMBYM_SAVED;
    const float ct = sv[kSavedCos], st = sv[kSavedSin];
    const float hi = win ? hann[i] : 1.f;
#pragma unroll
    for (int m = 0; m < kEb; ++m) {
        const int x = t + m * T;
        const size_t o = base + (size_t)i * N + x;
        const float w = win ? hi * hann[x] : 1.f;
        const float w2 = win2 ? w : 1.f;
        const float s2f = df2[o];
        const float s2g = rotate_adjoint(dgp + base, N, i, x, ct, st);
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
    size_t fwd_end;   // stage-1 recomputation reuses the forward layout's first regions
    size_t rf, rg, rdc, df2, dgp, dpol, dth, dspec, total;
};

static BwdLayout bwd_layout(const fmbym_params& p, int batch) {
    const size_t n = p.n, B = batch;
    const FwdLayout f = fwd_layout(p, batch);
    BwdLayout L{};
    size_t off = f.total;
    L.fwd_end = off;
    L.rf = off;
    off = al256(off + B * n * n * sizeof(float2));
    L.rg = off;
    off = al256(off + B * n * n * sizeof(float2));
    L.rdc = off;
    off = al256(off + B * n * n * sizeof(float2));
    L.df2 = off;
    off = al256(off + B * n * n * sizeof(float));
    L.dgp = off;
    off = al256(off + B * n * n * sizeof(float));
    L.dpol = off;
    off = al256(off + B * 2 * (size_t)p.n_r * p.n_theta * sizeof(float));
    L.dth = off;
    off = al256(off + B * n * sizeof(float));
    L.dspec = off;
    off = al256(off + B * (size_t)p.n_theta * sizeof(float2));
    L.total = off;
    return L;
}

size_t bwd_workspace(const fmbym_params& p, int batch) { return bwd_layout(p, batch).total; }

template <int N, int NT>
static void launch_bwd_polar(const Plan& pl, int B, const float* A, const float2* dspec, float* dpol,
                             hipStream_t s) {
    const int nrb = radius_blocks(pl.p.n_r);
    const int total = B * nrb;
    FMBYM_LAUNCH(kKBPolar, (kb_polar<NT, N>), dim3(((total + 7) / 8) * 8), dim3(256), s, A, pl.twiddle,
                 dspec, dpol, pl.p.n_r, B);
}

template <int NT>
static void launch_dtheta(const Plan& pl, int B, int ppb, const float* dth, const float* c_theta,
                          const float* saved, const float* d_pose, float2* dspec, hipStream_t s) {
    FMBYM_LAUNCH(kKBDtheta, kb_dtheta<NT>, dim3(B), dim3(NT / kEb), s, dth, ppb, c_theta, saved, d_pose,
                 pl.twiddle, pl.p.temp_theta, dspec);
}

template <int N>
static int launch_bwd_n(const Plan& pl, int B, const float* f, const float* g, const float* mf,
                        const float* mg, const float* c_theta, const float* c_xy, const float* saved,
                        const float* d_pose, float* d_f, float* d_g, float* d_mf, float* d_mg,
                        char* ws, hipStream_t s) {
    const FwdLayout fl = fwd_layout(pl.p, B);
    const BwdLayout bl = bwd_layout(pl.p, B);
    float2* rf = (float2*)(ws + bl.rf);
    float2* rg = (float2*)(ws + bl.rg);
    float2* rdc = (float2*)(ws + bl.rdc);
    float* df2 = (float*)(ws + bl.df2);
    float* dgp = (float*)(ws + bl.dgp);
    float* dpol = (float*)(ws + bl.dpol);
    float* dth = (float*)(ws + bl.dth);
    float2* dspec = (float2*)(ws + bl.dspec);
    float2* r1 = (float2*)(ws + fl.r1r2);
    float* mag = (float*)(ws + fl.mag_r3);
    const int win = (pl.p.flags & FMBYM_HANN) ? 1 : 0;
    const int win2 = (win && !(pl.p.flags & FMBYM_XY_UNWINDOWED)) ? 1 : 0;

    // translation-stage adjoint
    constexpr int T2 = 2 * N / kEb, LPB2 = 256 / T2;
    const int scan_blocks = B * N / LPB2, dc_blocks = B * (N / 2) / LPB2;
    FMBYM_LAUNCH(kKBRowsFwd2, kb_rows_fwd2<N>, dim3(scan_blocks + dc_blocks), dim3(256), s, f, g, mf, mg,
                 pl.hann, pl.twiddle, saved, c_xy, d_pose, rf, rg, rdc, win2, B, pl.p.temp_xy,
                 pl.p.delta_xy);
    // 512-thread blocks: the three transforms per column need more than the
    // 128 registers a 1024-thread block leaves each lane
    constexpr int C2 = N >= 512 ? 4 : (N >= 256 ? 8 : 16);
    const int total2 = B * (N / C2);
    FMBYM_LAUNCH(kKBColsXy, (kb_cols_xy<N, C2>), dim3(((total2 + 7) / 8) * 8), dim3(C2 * 2 * N / kEb), s,
                 rf, rg, rdc, pl.twiddle, B);
    FMBYM_LAUNCH(kKBRowsXy, kb_rows_xy<N>, dim3(B * N / LPB2), dim3(256), s, rf, rg, g, mg, pl.hann,
                 pl.twiddle, saved, df2, dgp, dth, win2);
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
    launch_stage1_spectra(pl, B, f, g, mf, mg, r1, mag, s);
    switch (pl.p.n_theta) {
        case 16: launch_bwd_polar<N, 16>(pl, B, mag, dspec, dpol, s); break;
        case 32: launch_bwd_polar<N, 32>(pl, B, mag, dspec, dpol, s); break;
        case 64: launch_bwd_polar<N, 64>(pl, B, mag, dspec, dpol, s); break;
        case 128: launch_bwd_polar<N, 128>(pl, B, mag, dspec, dpol, s); break;
        case 256: launch_bwd_polar<N, 256>(pl, B, mag, dspec, dpol, s); break;
        case 512: launch_bwd_polar<N, 512>(pl, B, mag, dspec, dpol, s); break;
        case 1024: launch_bwd_polar<N, 1024>(pl, B, mag, dspec, dpol, s); break;
        default: return FMBYM_EUNSUPPORTED;
    }
    float* dA = mag;                    // the recomputed magnitudes are dead after kb_polar
    const int nbins = N * (N / 2 + 1);
    FMBYM_LAUNCH(kKBDmag, kb_dmag, dim3((nbins + 255) / 256, (2 * B + kDmagGroup - 1) / kDmagGroup),
                 dim3(256), s, pl.csr_ptr, pl.csr_col, pl.csr_val, dpol, dA, N, pl.p.n_r, pl.p.n_theta,
                 2 * B, pl.band_on, pl.band_lo2, pl.band_hi2);
    constexpr int C = 16;
    FMBYM_LAUNCH(kKBColsMag, (kb_cols_mag<N, C>), dim3(B * 2 * (N / 2) / C), dim3(C * N / kEb), s, r1, dA,
                 pl.twiddle);
    constexpr int T1 = N / kEb, LPB1 = 256 / T1;
    FMBYM_LAUNCH(kKBRowsFinal, kb_rows_final<N>, dim3(B * N / LPB1), dim3(256), s, r1, df2, dgp, f, g, mf, mg,
                 pl.hann, pl.twiddle, saved, d_f, d_g, d_mf, d_mg, win, win2);
    return FMBYM_OK;
}

int launch_backward(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                    const float* mg, const float* /*pose*/, const float* c_theta, const float* c_xy,
                    const float* saved, const float* d_pose, float* d_f, float* d_g, float* d_mf,
                    float* d_mg, char* ws, hipStream_t s) {
    switch (pl.p.n) {
        case 128:
            return launch_bwd_n<128>(pl, batch, f, g, mf, mg, c_theta, c_xy, saved, d_pose, d_f, d_g,
                                     d_mf, d_mg, ws, s);
        case 256:
            return launch_bwd_n<256>(pl, batch, f, g, mf, mg, c_theta, c_xy, saved, d_pose, d_f, d_g,
                                     d_mf, d_mg, ws, s);
        case 512:
            return launch_bwd_n<512>(pl, batch, f, g, mf, mg, c_theta, c_xy, saved, d_pose, d_f, d_g,
                                     d_mf, d_mg, ws, s);
        default: return FMBYM_EUNSUPPORTED;
    }
}

}  // namespace fmbym
