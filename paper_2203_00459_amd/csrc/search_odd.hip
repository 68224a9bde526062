// Forward decoupled search (Algorithm 1) at odd scan sides, the paper's
// measured 127, 255 and 511 px (Section IV-C), with any number of heading
// bins (its default 733).  The origin pixel is c = (n - 1)/2; lags run over
// -(n-1)/2 .. (n-1)/2 on both translation axes and -floor(n_theta/2) ..
// n_theta - 1 - floor(n_theta/2) in heading.
//
// Stage 1 (Eq. 5-8)
//   ko_rows1     window (and mask), then the n-point DFT of f + i g per row by
//                Bluestein's chirp transform over a power-of-two line of
//                M1 >= 2n - 1 points; the two spectra split by the mirror
//                X[(n - k) mod n], columns 0 .. (n-1)/2 kept.
//   ko_cols1     n-point column DFTs (Bluestein) of both spectra, band-pass,
//                magnitude.
//   ko_polar     bilinear polar gather of both magnitude spectra; each radius
//                centred by its angular mean; the linear correlation along
//                angle through one LT-point DFT of the zero-padded pair
//                (LT >= 2 n_theta - 1), summed over a block of radii.
//   ko_angle_sum sum over radius blocks, one spectrum bin per thread.
//   ko_angle_fin inverse DFT, the circular correlation folded back from the
//                linear one
//                (c[l] = lin[l mod n_theta] + lin[(l mod n_theta) - n_theta]),
//                softmax and soft-argmax -> theta.
// Stage 2 (Eq. 9)
//   ko_rotate    g' = Rotate(g_w, theta) about the origin pixel, per pixel.
//   ko_rows2     f_w + i g' zero-padded to M2 = 3 2^b >= n + (n-1)/2 (the
//                circular correlation at that length is the linear one on the
//                lag window), row DFTs, columns 0 .. M2/2.
//   ko_cols2     column DFTs of both, conj(F) G', inverse; the n lag rows kept.
//   ko_rows3     inverse row DFTs of two lag rows at a time -> c_xy and
//                online-softmax partials, merged by k_xy_fin.
// All reductions run in a fixed order; results are bitwise reproducible.
#include "internal.hpp"
#include "profile.hpp"

namespace fmbym {

namespace {

constexpr int kOddPasses = 4;   // radii per line of a heading-correlation block (in sequence)
constexpr int kOddE1 = 8;       // elements per thread of the Bluestein lines

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Elements per thread and radii per block of the heading correlation over LT points.
__host__ __device__ constexpr int odd_lt_e(int lt) { return (lt & (lt - 1)) == 0 ? 8 : 12; }
__host__ __device__ constexpr int odd_radii(int lt) { return (256 / (lt / odd_lt_e(lt))) * kOddPasses; }
__host__ __device__ constexpr int odd_radius_blocks(int n_r, int lt) { return (n_r + odd_radii(lt) - 1) / odd_radii(lt); }

// Pitches (elements) of the odd path's row arrays.
constexpr int odd_u(int n) { return (n + 1) / 2; }          // stage-1 unique columns (a power of two)
constexpr int odd_p2(int m2) { return m2 / 2 + 16; }        // stage-2 columns 0 .. M2/2 plus a tile's room

struct OddLayout {
    size_t r12, alag, pth, pthm, pxy, saved, grot, total;
};

OddLayout odd_layout(const fmbym_params& p, int batch) {
    const size_t n = p.n, B = batch, U = odd_u(p.n), P2 = odd_p2(odd_m2(p.n));
    const int lt = odd_lt(p.n_theta), nrb = odd_radius_blocks(p.n_r, lt);
    OddLayout L{};
    size_t off = 0;
    L.r12 = off;   // stage-1 row spectra, then the stage-2 row spectra
    const size_t r1 = B * n * U * sizeof(float4), r2 = B * n * P2 * sizeof(float4);
    off = al256(off + (r1 > r2 ? r1 : r2));
    L.alag = off;  // magnitudes, then the stage-2 lag rows
    const size_t a = B * n * U * sizeof(float2), lag = B * n * P2 * sizeof(float2);
    off = al256(off + (a > lag ? a : lag));
    L.pth = off;
    off = al256(off + B * (size_t)nrb * (lt / 2 + 1) * sizeof(float2));
    L.pthm = off;
    off = al256(off + B * (size_t)nrb * sizeof(float));
    L.pxy = off;
    off = al256(off + B * n * sizeof(float4));   // at most one partial per lag row
    L.saved = off;
    off = al256(off + B * FMBYM_SAVED * sizeof(float));
    L.grot = off;
    off = al256(off + B * n * n * sizeof(float));
    L.total = off;
    return L;
}

// Bluestein's chirp transform of one line: on entry v holds x[j] at
// j = t + m T (j < n; entries past n are ignored), on exit X[k] at k = t + m T
// for k < n (entries past n are unused values).  With c_j = exp(i pi j^2 / n),
// jk = (j^2 + k^2 - (k - j)^2) / 2 gives X[k] = conj(c_k) sum_j (x_j conj(c_j))
// c_{k - j}: a circular convolution over M >= 2n - 1 points, whose filter
// spectrum (DFT_M of c_m for |m| < n, wrapped, divided by M) is bspec.
template <int M, int E, class Lay>
__device__ __forceinline__ void bluestein(float2 (&v)[E], float* re, float* im, int t,
                                          const float2* __restrict__ tw, const float2* __restrict__ chirp,
                                          const float2* __restrict__ bspec, int n) {
    constexpr int T = M / E;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int j = t + m * T;
        const float2 c = chirp[j < n ? j : 0];
        v[m] = j < n ? cmulcj(c, v[m]) : make_float2(0.f, 0.f);
    }
    fft_line<M, E, Lay>(v, re, im, fresh_index(t), tw);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cmul(v[m], bspec[t + m * T]);
    ifft_line<M, E, Lay>(v, re, im, fresh_index(t), tw);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * T;
        v[m] = cmulcj(chirp[k < n ? k : 0], v[m]);
    }
}

__device__ __forceinline__ float odd_band(int ky_signed, int kx, int on, int lo2, int hi2) {
    if (!on) return 1.f;
    const int r2 = ky_signed * ky_signed + kx * kx;
    return (r2 >= lo2 && r2 <= hi2) ? 1.f : 0.f;
}

// ------------------------------------------------------------------ stage 1

template <int N, int M>
__global__ __launch_bounds__(256) void ko_rows1(const float* __restrict__ f, const float* __restrict__ g,
                                                const float* __restrict__ mf, const float* __restrict__ mg,
                                                const float* __restrict__ hann, const float2* __restrict__ tw,
                                                const float2* __restrict__ chirp, const float2* __restrict__ bspec,
                                                float4* __restrict__ out, int win, int batch) {
    constexpr int E = kOddE1, T = M / E, LPB = 256 / T, U = odd_u(N);
    __shared__ float lre[LPB][LdsRows<M>::words(M)];
    __shared__ float lim[LPB][LdsRows<M>::words(M)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int grow = blockIdx.x * LPB + line;      // row over the batch
    const bool live = grow < batch * N;
    const int i = live ? grow % N : 0;
    const size_t off = live ? (size_t)grow * N : 0;
    const float hi = hann[i];
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + m * T;
        if (live && x < N) {
            const float w = win ? hi * hann[x] : 1.f;
            const float a = f[off + x] * (mf ? mf[off + x] : 1.f);
            const float c = g[off + x] * (mg ? mg[off + x] : 1.f);
            v[m] = make_float2(a * w, c * w);
        } else {
            v[m] = make_float2(0.f, 0.f);
        }
    }
    bluestein<M, E, LdsRows<M>>(v, lre[line], lim[line], t, tw, chirp, bspec, N);
    // split the two real rows' spectra with the mirror X[(n - k) mod n]
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * T;
        if (k < N) {
            lre[line][LdsRows<M>::at(k)] = v[m].x;
            lim[line][LdsRows<M>::at(k)] = v[m].y;
        }
    }
    __syncthreads();
    if (!live) return;   // no barriers follow
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * T;
        if (k < U) {
            const int km = LdsRows<M>::at(k == 0 ? 0 : N - k);
            const float2 mir = make_float2(lre[line][km], lim[line][km]);
            const float2 X = split_x(v[m], mir), Y = split_y(v[m], mir);
            out[(size_t)grow * U + k] = make_float4(X.x, X.y, Y.x, Y.y);
        }
    }
}

// Column DFTs (Bluestein) of both stage-1 spectra, band-pass and magnitude:
// C columns per block, all (n + 1)/2 columns in whole tiles.
template <int N, int M, int C>
__global__ __launch_bounds__(C * M / kOddE1) void ko_cols1(const float4* __restrict__ in, float2* __restrict__ A,
                                                           const float2* __restrict__ tw,
                                                           const float2* __restrict__ chirp,
                                                           const float2* __restrict__ bspec, int band_on,
                                                           int lo2, int hi2, int batch) {
    constexpr int E = kOddE1, T = M / E, U = odd_u(N), H = N / 2, TILES = U / C;
    static_assert(U % C == 0, "whole tiles");
    __shared__ float lre[C][LdsCols<C>::words(M)];
    __shared__ float lim[C][LdsCols<C>::words(M)];
    const int per_xcd = gridDim.x / 8;   // grid is a multiple of 8
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;   // a pair's tiles on one XCD
    if (work >= batch * TILES) return;   // block-uniform
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int tile = work % TILES, b = work / TILES;
    const int col = tile * C + c;
    const float4* src = in + (size_t)b * N * U;
    float2 vf[E], vg[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int r = t + m * T;
        const float4 q = r < N ? src[(size_t)r * U + col] : make_float4(0.f, 0.f, 0.f, 0.f);
        vf[m] = make_float2(q.x, q.y);
        vg[m] = make_float2(q.z, q.w);
    }
    bluestein<M, E, LdsCols<C>>(vf, lre[c], lim[c], t, tw, chirp, bspec, N);
    bluestein<M, E, LdsCols<C>>(vg, lre[c], lim[c], t, tw, chirp, bspec, N);
    float2* dst = A + (size_t)b * N * U;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int ky = t + m * T;
        if (ky < N) {
            const float gain = odd_band(ky <= H ? ky : ky - N, col, band_on, lo2, hi2);
            dst[(size_t)ky * U + col] = make_float2(sqrtf(vf[m].x * vf[m].x + vf[m].y * vf[m].y) * gain,
                                                    sqrtf(vg[m].x * vg[m].x + vg[m].y * vg[m].y) * gain);
        }
    }
}

// Bilinear read of both magnitude spectra at frequency (uy, ux) in bins, with
// indices modulo n and |F(-k)| = |F(k)| for columns past (n - 1)/2.  The polar
// grid has 0 <= uy < n/2 and |ux| < n/2, so every corner index lies in
// [-(n+1)/2, (n+1)/2] and one conditional add reduces it modulo n.
__device__ __forceinline__ float2 odd_mag_sample(const float2* __restrict__ A, int n, float uy, float ux) {
    const int U = (n + 1) / 2;
    const float fy = floorf(uy), fx = floorf(ux);
    const float wy = uy - fy, wx = ux - fx;
    const int y0 = (int)fy, x0 = (int)fx;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            int ky = y0 + dy, kx = x0 + dx;
            ky = ky < 0 ? ky + n : ky;
            kx = kx < 0 ? kx + n : kx;
            if (kx >= U) {
                kx = n - kx;
                ky = ky == 0 ? 0 : n - ky;
            }
            const float w = (dy ? wy : 1.f - wy) * (dx ? wx : 1.f - wx);
            const float2 a = A[(size_t)ky * U + kx];
            acc.x += w * a.x;
            acc.y += w * a.y;
        }
    }
    return acc;
}

// Heading correlation over odd_radii(LT) radii per block (kOddPasses per
// line, one after the other).  Radius b samples
// rho = (n/2) b / n_r bins at the plan's angles; each radius's profiles are
// centred by their angular means (sum_a (P_f - mu_f)(P_g - mu_g)(. + l) is the
// circular correlation minus S_f S_g / n_theta, its mean over the lags), then
// zero-padded to LT and transformed as one complex line.  The block writes the
// sum over its radii of conj(A_f) A_g (bins 0 .. LT/2) and of S_f S_g.
template <int LT, int E>
__global__ __launch_bounds__(256) void ko_polar(const float2* __restrict__ A, int n,
                                                const float2* __restrict__ cs, int n_theta, int n_r,
                                                const float2* __restrict__ tw, float2* __restrict__ part,
                                                float* __restrict__ partm, int batch) {
    constexpr int T = LT / E, LPB = 256 / T, PASSES = kOddPasses, HK = LT / 2 + 1, RPB = LPB * PASSES;
    static_assert(T % 64 == 0, "a line is whole wavefronts");
    __shared__ float lre[LPB][LdsRows<LT>::words(LT)];
    __shared__ float lim[LPB][LdsRows<LT>::words(LT)];
    __shared__ float2 red[4];   // per-wavefront angular sums (S_f, S_g)
    const int nrb = (n_r + RPB - 1) / RPB;
    const int total = batch * nrb;
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;   // a pair's blocks on one XCD
    if (work >= total) return;   // block-uniform
    const int b = work / nrb, rb = work % nrb;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const float2* Ab = A + (size_t)b * n * odd_u(n);
    float2 acc[E / 2 + 1];
#pragma unroll
    for (int m = 0; m <= E / 2; ++m) acc[m] = make_float2(0.f, 0.f);
    float accm = 0.f;
    for (int pass = 0; pass < PASSES; ++pass) {
        const int rad = rb * RPB + pass * LPB + line;
        const bool live = rad < n_r;
        const float rho = 0.5f * (float)n * (float)rad / (float)n_r;
        float2 v[E];
        float sf = 0.f, sg = 0.f;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int a = t + m * T;
            if (live && a < n_theta) {
                const float2 w = cs[a];
                v[m] = odd_mag_sample(Ab, n, rho * w.y, rho * w.x);
            } else {
                v[m] = make_float2(0.f, 0.f);
            }
            sf += v[m].x;
            sg += v[m].y;
        }
        // angular sums of this radius: a butterfly within each wavefront whose
        // lane-0 value every lane takes (one rounding order for all), then the
        // line's wavefronts added in order
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sf += __shfl_xor(sf, off);
            sg += __shfl_xor(sg, off);
        }
        sf = __shfl(sf, 0);
        sg = __shfl(sg, 0);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_float2(sf, sg);
        __syncthreads();
        float Sf = 0.f, Sg = 0.f;
#pragma unroll
        for (int w = 0; w < T / 64; ++w) {
            const float2 r = red[line * (T / 64) + w];
            Sf += r.x;
            Sg += r.y;
        }
        const float muf = Sf / (float)n_theta, mug = Sg / (float)n_theta;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (t + m * T < n_theta) v[m] = make_float2(v[m].x - muf, v[m].y - mug);
        }
        accm += Sf * Sg;
        fft_line<LT, E>(v, lre[line], lim[line], fresh_index(t), tw);
        float2 mir[E];
        mirror_line<LT, E>(v, mir, lre[line], lim[line], fresh_index(t));
#pragma unroll
        for (int m = 0; m <= E / 2; ++m) acc[m] = cadd(acc[m], cmulcj(split_x(v[m], mir[m]), split_y(v[m], mir[m])));
    }
    // fixed-order sum over the lines of the block, through LDS
    __syncthreads();
    float* sre = &lre[0][0];
    float* sim = &lim[0][0];
#pragma unroll
    for (int m = 0; m <= E / 2; ++m) {
        const int k = t + m * T;
        if (k < HK) {
            sre[line * HK + k] = acc[m].x;
            sim[line * HK + k] = acc[m].y;
        }
    }
    __shared__ float redm[LPB];
    if (t == 0) redm[line] = accm;
    __syncthreads();
    float2* dst = part + ((size_t)b * nrb + rb) * HK;
    for (int k = threadIdx.x; k < HK; k += 256) {
        float2 s = make_float2(0.f, 0.f);
        for (int l = 0; l < LPB; ++l) s = cadd(s, make_float2(sre[l * HK + k], sim[l * HK + k]));
        dst[k] = s;
    }
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int l = 0; l < LPB; ++l) s += redm[l];
        partm[(size_t)b * nrb + rb] = s;
    }
}

// Sum over radius blocks, inverse DFT to the linear correlation lin[d] of the
// centred profiles (d mod LT), the circular correlation folded back from it,
// then the softmax and the soft-argmax as for even sides:
// theta = (l* + nu) pi / n_theta with nu = sum_l p_l (l - l*).
// Sum over the radius blocks of a pair, in block order, for one spectrum bin
// per thread (and, by one thread, of the S_f S_g partials): the totals replace
// radius block 0 of the partials (a thread reads and writes only its bin).
template <int LT>
__global__ __launch_bounds__(256) void ko_angle_sum(float2* __restrict__ part, float* __restrict__ partm, int n_r) {
    constexpr int HK = LT / 2 + 1;
    const int b = blockIdx.y, k = blockIdx.x * 256 + threadIdx.x;
    const int nrb = odd_radius_blocks(n_r, LT);
    float2* src = part + (size_t)b * nrb * HK;
    if (k < HK) {
        float2 s = make_float2(0.f, 0.f);
        int r = 0;
        for (; r + 8 <= nrb; r += 8) {   // eight loads in flight, then added in order
            float2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src[(size_t)(r + u) * HK + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) s = cadd(s, v[u]);
        }
        for (; r < nrb; ++r) s = cadd(s, src[(size_t)r * HK + k]);
        src[k] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float m = 0.f;
        for (int r = 0; r < nrb; ++r) m += partm[(size_t)b * nrb + r];
        partm[(size_t)b * nrb] = m;
    }
}

template <int LT, int E>
__global__ __launch_bounds__(LT / E) void ko_angle_fin(const float2* __restrict__ part,
                                                       const float* __restrict__ partm, int n_r, int n_theta,
                                                       const float2* __restrict__ tw, float temp,
                                                       float* __restrict__ c_theta, float* __restrict__ pose,
                                                       float* __restrict__ saved) {
    constexpr int T = LT / E, HK = LT / 2 + 1, J = E / 2 + 1;   // n_theta <= (LT + 1) / 2 lags
    __shared__ float lre[LdsRows<LT>::words(LT)];
    __shared__ float lim[LdsRows<LT>::words(LT)];
    __shared__ float lin[LT];
    __shared__ float red[T];
    __shared__ int redi[T];
    const int b = blockIdx.x, t = threadIdx.x;
    const int nrb = odd_radius_blocks(n_r, LT);
    const float2* psum = part + (size_t)b * nrb * HK;   // block 0 holds the totals (ko_angle_sum)
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * T;
        const float2 s = psum[k < HK ? k : LT - k];
        v[m] = k < HK ? s : cconj(s);
    }
    ifft_line<LT, E>(v, lre, lim, t, tw);
#pragma unroll
    for (int m = 0; m < E; ++m) lin[t + m * T] = v[m].x;
    __syncthreads();
    const float scale = 1.f / ((float)LT * (float)n_r);
    const int half = n_theta / 2;
    float c[J];
    float lmax = -INFINITY;
    int larg = 0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int k = t + j * T;   // storage index: lag k - half
        if (k < n_theta) {
            const int l = k - half;
            const int lp = l < 0 ? l + n_theta : l;   // l mod n_theta
            c[j] = (lin[lp] + lin[lp - n_theta + LT]) * scale;
            if (c[j] > lmax) {   // k increases with j: the first maximum keeps the lowest index
                lmax = c[j];
                larg = k;
            }
        } else {
            c[j] = -INFINITY;
        }
    }
    float cmax;
    int kmax;
    block_argmax(lmax, larg, red, redi, T, cmax, kmax);
    const int lag_star = kmax - half;
    const float inv_t = 1.f / temp;
    float se = 0.f, sn = 0.f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int k = t + j * T;
        if (k < n_theta) {
            const float e = expf((c[j] - cmax) * inv_t);
            se += e;
            sn += e * (float)(k - half - lag_star);
            if (c_theta) c_theta[(size_t)b * n_theta + k] = c[j];
        }
    }
    const float Z = block_sum(se, red, T);
    const float SN = block_sum(sn, red, T);
    if (t == 0) {
        const float mean = partm[(size_t)b * nrb];   // the total (ko_angle_sum)
        const float nu = SN / Z;
        const float theta = ((float)lag_star + nu) * (3.14159265358979323846f / (float)n_theta);
        pose[b * 3 + 0] = theta;
        float* sv = saved + (size_t)b * FMBYM_SAVED;
        sv[kSavedTheta] = theta;
        float snt, cst;
        sincosf(theta, &snt, &cst);
        sv[kSavedCos] = cst;
        sv[kSavedSin] = snt;
        sv[kSavedThetaMax] = cmax;
        sv[kSavedThetaSum] = Z;
        sv[kSavedThetaMean] = mean / ((float)n_theta * (float)n_r);
        sv[kSavedThetaArg] = (float)lag_star;
        sv[kSavedThetaNu] = nu;
        for (int i = kSavedStatus; i < FMBYM_SAVED; ++i) sv[i] = 0.f;
    }
}

// ------------------------------------------------------------------ stage 2

template <int N>
__global__ __launch_bounds__(256) void ko_rotate(const float* __restrict__ g, const float* __restrict__ mg,
                                                 const float* __restrict__ hann, const float* __restrict__ saved,
                                                 float* __restrict__ gr, int win, int batch) {
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= (long long)batch * N * N) return;
    const int b = (int)(p / (N * N)), q = (int)(p % (N * N));
    const float* sv = saved + (size_t)b * FMBYM_SAVED;
    const size_t o = (size_t)b * N * N;
    gr[p] = rotate_sample(g + o, mg ? mg + o : nullptr, hann, N, q / N, q % N, sv[kSavedCos], sv[kSavedSin],
                          win != 0);
}

template <int N, int M2>
__global__ __launch_bounds__(256) void ko_rows2(const float* __restrict__ f, const float* __restrict__ mf,
                                                const float* __restrict__ hann, const float* __restrict__ gr,
                                                const float2* __restrict__ tw, float4* __restrict__ out, int win2,
                                                int batch) {
    constexpr int E = kE2, T = M2 / E, LPB = 256 / T, H2 = M2 / 2, P2 = odd_p2(M2);
    __shared__ float lre[LPB][LdsRows<M2>::words(M2)];
    __shared__ float lim[LPB][LdsRows<M2>::words(M2)];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int grow = blockIdx.x * LPB + line;
    const bool live = grow < batch * N;
    const int b = live ? grow / N : 0, i = live ? grow % N : 0;
    const size_t o = (size_t)b * N * N;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + m * T;
        v[m] = (live && x < N) ? make_float2(scan_w(f + o, mf ? mf + o : nullptr, hann, N, i, x, win2 != 0),
                                             gr[(size_t)grow * N + x])
                               : make_float2(0.f, 0.f);
    }
    fft_line<M2, E>(v, lre[line], lim[line], fresh_index(t), tw);
    float2 mir[E];
    mirror_line<M2, E>(v, mir, lre[line], lim[line], fresh_index(t));
    if (!live) return;
#pragma unroll
    for (int m = 0; m <= E / 2; ++m) {
        const int k = t + m * T;
        if (k <= H2) {
            const float2 X = split_x(v[m], mir[m]), Y = split_y(v[m], mir[m]);
            out[(size_t)grow * P2 + k] = make_float4(X.x, X.y, Y.x, Y.y);
        }
    }
}

// Column pass of stage 2 over columns 0 .. M2/2: forward DFTs of F and G'
// (n data rows, zeros after), conj(F) G', inverse; lag rows -(n-1)/2 ..
// (n-1)/2 kept in that order.
template <int N, int M2, int C>
__global__ __launch_bounds__(C * M2 / kE2) void ko_cols2(const float4* __restrict__ in,
                                                        const float2* __restrict__ tw, float2* __restrict__ out,
                                                        int batch) {
    constexpr int E = kE2, T = M2 / E, H2 = M2 / 2, TILES = H2 / C + 1, P2 = odd_p2(M2), H = N / 2;
    __shared__ float lre[C][LdsCols<C>::words(M2)];
    __shared__ float lim[C][LdsCols<C>::words(M2)];
    const int total = batch * TILES;
    const int per_xcd = (total + 7) / 8;
    const int work = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (work >= total) return;   // block-uniform
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int tile = work % TILES, b = work / TILES;
    const int col = tile * C + c;   // < P2: the last tile's spare columns are computed, not stored
    const float4* src = in + (size_t)b * N * P2;
    float2 vf[E], vg[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int r = t + m * T;
        const float4 q = r < N ? src[(size_t)r * P2 + col] : make_float4(0.f, 0.f, 0.f, 0.f);
        vf[m] = make_float2(q.x, q.y);
        vg[m] = make_float2(q.z, q.w);
    }
    fft_line<M2, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
    fft_line<M2, E, LdsCols<C>>(vg, lre[c], lim[c], fresh_index(t), tw);
#pragma unroll
    for (int m = 0; m < E; ++m) vf[m] = cmulcj(vf[m], vg[m]);
    ifft_line<M2, E, LdsCols<C>>(vf, lre[c], lim[c], fresh_index(t), tw);
    if (col > H2) return;
    float2* dst = out + (size_t)b * N * P2;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int r = t + m * T;        // lag s_y = r (r <= H) or r - M2 (r >= M2 - H)
        if (r <= H) dst[(size_t)(r + H) * P2 + col] = vf[m];
        else if (r >= M2 - H) dst[(size_t)(r - M2 + H) * P2 + col] = vf[m];
    }
}

// Entry k of the M-point Hermitian spectrum of a lag row storing columns 0 .. M/2.
__device__ __forceinline__ float2 odd_herm(const float2* __restrict__ row, int M, int k) {
    const float2 a = row[k <= M / 2 ? k : M - k];
    const bool real = k == 0 || k == M / 2;
    return make_float2(a.x, real ? 0.f : (k < M / 2 ? a.y : -a.y));
}

// Inverse rows of lag rows 2q and 2q + 1 in one complex line (the second is
// absent for q = (n - 1)/2), c_xy of the kept lags, and one online-softmax
// partial (max, sum of exp, sum of exp s_x, sum of exp s_y) per block.
template <int N, int M2>
__global__ __launch_bounds__(256) void ko_rows3(const float2* __restrict__ in, const float2* __restrict__ tw,
                                                float* __restrict__ c_xy, float4* __restrict__ part, float temp,
                                                int batch) {
    constexpr int E = kE2, T = M2 / E, LPB = 256 / T, NP = (N + 1) / 2, P2 = odd_p2(M2), H = N / 2;
    static_assert(NP % LPB == 0, "a block's lines belong to one pair");
    __shared__ float lre[LPB][LdsRows<M2>::words(M2)];
    __shared__ float lim[LPB][LdsRows<M2>::words(M2)];
    __shared__ float4 red[256];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int gl = blockIdx.x * LPB + line;   // row pair over the batch (the grid covers them exactly)
    const int b = gl / NP, q = gl % NP;
    const int r0 = 2 * q, r1 = 2 * q + 1;
    const bool two = r1 < N;
    const float2* row0 = in + ((size_t)b * N + r0) * P2;
    const float2* row1 = in + ((size_t)b * N + (two ? r1 : r0)) * P2;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * T;
        const float2 h1 = odd_herm(row0, M2, k);
        const float2 h2 = two ? odd_herm(row1, M2, k) : make_float2(0.f, 0.f);
        v[m] = make_float2(h1.x - h2.y, h1.y + h2.x);   // h1 + i h2
    }
    ifft_line<M2, E>(v, lre[line], lim[line], t, tw);
    const float scale = 1.f / ((float)M2 * (float)M2);
    const float inv_t = 1.f / temp;
    const float sy0 = (float)(r0 - H), sy1 = (float)(r1 - H);
    float lmax = -INFINITY;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int nn = t + m * T;
        const bool kept = nn <= H || nn >= M2 - H;
        if (kept) {
            const int col = nn <= H ? nn + H : nn - M2 + H;
            const float c0 = v[m].x * scale, c1 = v[m].y * scale;
            if (c_xy) c_xy[((size_t)b * N + r0) * N + col] = c0;
            lmax = fmaxf(lmax, c0);
            if (two) {
                if (c_xy) c_xy[((size_t)b * N + r1) * N + col] = c1;
                lmax = fmaxf(lmax, c1);
            }
        }
    }
    float Z = 0.f, Sx = 0.f, Sy = 0.f;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int nn = t + m * T;
        if (nn <= H || nn >= M2 - H) {
            const float sx = (float)(nn <= H ? nn : nn - M2);
            const float e0 = expf((v[m].x * scale - lmax) * inv_t);
            const float e1 = two ? expf((v[m].y * scale - lmax) * inv_t) : 0.f;
            Z += e0 + e1;
            Sx += (e0 + e1) * sx;
            Sy += e0 * sy0 + e1 * sy1;
        }
    }
    red[threadIdx.x] = make_float4(lmax, Z, Sx, Sy);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = softmax_merge(red[threadIdx.x], red[threadIdx.x + s], inv_t);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- launchers

template <int LT>
void launch_angle(const Plan& pl, int B, const float2* A, float2* pth, float* pthm, float* c_theta, float* pose,
                  float* sv, hipStream_t s) {
    constexpr int E = (LT & (LT - 1)) == 0 ? 8 : 12;
    const float2* tw = (LT & (LT - 1)) == 0 ? pl.twiddle : pl.twiddle3;
    const int nrb = odd_radius_blocks(pl.p.n_r, LT);
    const int total = B * nrb;
    FMBYM_LAUNCH(kOPolar, (ko_polar<LT, E>), dim3(((total + 7) / 8) * 8), dim3(256), s, A, pl.p.n, pl.polar_cs,
                 pl.p.n_theta, pl.p.n_r, tw, pth, pthm, B);
    FMBYM_LAUNCH(kOAngleFin, ko_angle_sum<LT>, dim3((LT / 2 + 1 + 255) / 256, B), dim3(256), s, pth, pthm,
                 pl.p.n_r);
    FMBYM_LAUNCH(kOAngleFin, (ko_angle_fin<LT, E>), dim3(B), dim3(LT / E), s, pth, pthm, pl.p.n_r, pl.p.n_theta,
                 tw, pl.p.temp_theta, c_theta, pose, sv);
}

template <int N>
int launch_odd_n(const Plan& pl, int B, const float* f, const float* g, const float* mf, const float* mg,
                 float* pose, float* c_theta, float* c_xy, float* saved, char* ws, hipStream_t s) {
    constexpr int M1 = N == 127 ? 256 : N == 255 ? 512 : 1024;
    constexpr int M2 = N == 127 ? 192 : N == 255 ? 384 : 768;
    constexpr int T1 = M1 / kOddE1, C1 = 256 / T1, U = odd_u(N);
    constexpr int T2 = M2 / kE2, C2 = 256 / T2, LPB2 = 256 / T2, NP = (N + 1) / 2;
    const OddLayout L = odd_layout(pl.p, B);
    float4* r1 = (float4*)(ws + L.r12);
    float4* r2 = (float4*)(ws + L.r12);      // stage-1 rows are dead after ko_cols1
    float2* A = (float2*)(ws + L.alag);
    float2* lag = (float2*)(ws + L.alag);    // magnitudes are dead after ko_polar
    float2* pth = (float2*)(ws + L.pth);
    float* pthm = (float*)(ws + L.pthm);
    float4* pxy = (float4*)(ws + L.pxy);
    float* sv = saved ? saved : (float*)(ws + L.saved);
    float* gr = (float*)(ws + L.grot);
    const int win = (pl.p.flags & FMBYM_HANN) ? 1 : 0;
    const int win2 = (win && !(pl.p.flags & FMBYM_XY_UNWINDOWED)) ? 1 : 0;
    const int rows = B * N;
    FMBYM_LAUNCH(kORows1, (ko_rows1<N, M1>), dim3((rows + (256 / T1) - 1) / (256 / T1)), dim3(256), s, f, g, mf,
                 mg, pl.hann, pl.twiddle, pl.chirp, pl.bspec, r1, win, B);
    const int tiles1 = B * (U / C1);
    FMBYM_LAUNCH(kOCols1, (ko_cols1<N, M1, C1>), dim3(((tiles1 + 7) / 8) * 8), dim3(C1 * T1), s, r1, A,
                 pl.twiddle, pl.chirp, pl.bspec, pl.band_on, pl.band_lo2, pl.band_hi2, B);
    switch (odd_lt(pl.p.n_theta)) {
        case 512: launch_angle<512>(pl, B, A, pth, pthm, c_theta, pose, sv, s); break;
        case 768: launch_angle<768>(pl, B, A, pth, pthm, c_theta, pose, sv, s); break;
        case 1024: launch_angle<1024>(pl, B, A, pth, pthm, c_theta, pose, sv, s); break;
        case 1536: launch_angle<1536>(pl, B, A, pth, pthm, c_theta, pose, sv, s); break;
        case 2048: launch_angle<2048>(pl, B, A, pth, pthm, c_theta, pose, sv, s); break;
        default: return FMBYM_EUNSUPPORTED;
    }
    const long long px = (long long)B * N * N;
    FMBYM_LAUNCH(kORotate, ko_rotate<N>, dim3((unsigned)((px + 255) / 256)), dim3(256), s, g, mg, pl.hann, sv, gr,
                 win2, B);
    FMBYM_LAUNCH(kORows2, (ko_rows2<N, M2>), dim3((rows + LPB2 - 1) / LPB2), dim3(256), s, f, mf, pl.hann, gr,
                 pl.twiddle3, r2, win2, B);
    const int tiles2 = B * ((M2 / 2) / C2 + 1);
    FMBYM_LAUNCH(kOCols2, (ko_cols2<N, M2, C2>), dim3(((tiles2 + 7) / 8) * 8), dim3(C2 * T2), s, r2,
                 pl.twiddle3, lag, B);
    constexpr int PPP = NP / LPB2;   // softmax partials per pair
    FMBYM_LAUNCH(kORows3, (ko_rows3<N, M2>), dim3(B * PPP), dim3(256), s, lag, pl.twiddle3, c_xy, pxy,
                 pl.p.temp_xy, B);
    launch_xy_fin_parts(pxy, PPP, pl.p.temp_xy, pl.p.delta_xy, B, pose, sv, s);
    return FMBYM_OK;
}

}  // namespace

size_t odd_fwd_workspace(const fmbym_params& p, int batch) { return odd_layout(p, batch).total; }

int launch_forward_odd(const Plan& pl, int batch, const float* f, const float* g, const float* mf,
                       const float* mg, float* pose, float* c_theta, float* c_xy, float* saved, char* ws,
                       hipStream_t s) {
    switch (pl.p.n) {
        case 127: return launch_odd_n<127>(pl, batch, f, g, mf, mg, pose, c_theta, c_xy, saved, ws, s);
        case 255: return launch_odd_n<255>(pl, batch, f, g, mf, mg, pose, c_theta, c_xy, saved, ws, s);
        case 511: return launch_odd_n<511>(pl, batch, f, g, mf, mg, pose, c_theta, c_xy, saved, ws, s);
        default: return FMBYM_EUNSUPPORTED;
    }
}

}  // namespace fmbym
