// Device-side building blocks of the search kernels: complex helpers, radix-2/3/4/6/8/12
// butterflies and a Stockham autosort FFT over one "line" of L = 2^a or 3 2^a
// points held cooperatively by T threads, each owning E = L/T elements in
// registers.  Lines exchange data between stages through a padded LDS buffer
// (separate re/im planes).
//
// Register layout, on entry and on exit: thread t holds element t + m*T in v[m].
// This is the layout of a coalesced global load/store of the line, so row
// kernels load and store directly from/to registers and column kernels only
// need the LDS transpose that the FFT stages already perform.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmbym {

// Twiddle tables: W_2048^m for lines of 2^a points and W_3072^m for lines of
// 3 2^a points (each small enough to stay in the vector L1 cache).
constexpr int kTwiddleLen = 2048;
constexpr int kTwiddleLen3 = 3072;
template <int L>
constexpr int twiddle_len() { return (L & (L - 1)) == 0 ? kTwiddleLen : kTwiddleLen3; }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulcj(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 mul_negi(float2 a) { return make_float2(a.y, -a.x); }   // a * (-i)

// Forward butterflies, X[k] = sum_n v[n] exp(-2 pi i k n / R), in place.
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
    float2 a0 = cadd(v0, v2), a1 = csub(v0, v2);
    float2 a2 = cadd(v1, v3), a3 = mul_negi(csub(v1, v3));
    v0 = cadd(a0, a2);
    v2 = csub(a0, a2);
    v1 = cadd(a1, a3);
    v3 = csub(a1, a3);
}

__device__ __forceinline__ void dft8(float2 (&v)[8]) {
    const float c = 0.70710678118654752440f;
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    // o_k *= W8^k
    float2 w1 = make_float2(c * (o1.x + o1.y), c * (o1.y - o1.x));
    float2 w2 = mul_negi(o2);
    float2 w3 = make_float2(c * (o3.y - o3.x), -c * (o3.x + o3.y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1);
    v[5] = csub(e1, w1);
    v[2] = cadd(e2, w2);
    v[6] = csub(e2, w2);
    v[3] = cadd(e3, w3);
    v[7] = csub(e3, w3);
}

// X1 = a + W b + W^2 c, X2 = a + W^2 b + W c with W = exp(-2 pi i / 3).
__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
    const float h = 0.86602540378443864676f;   // sqrt(3) / 2
    const float2 s = cadd(b, c);
    const float2 m = make_float2(a.x - 0.5f * s.x, a.y - 0.5f * s.y);
    const float2 d = csub(b, c);
    const float2 r = make_float2(h * d.y, -h * d.x);   // -i (sqrt(3)/2) (b - c)
    a = cadd(a, s);
    b = cadd(m, r);
    c = csub(m, r);
}

// 12 = 4 x 3: DFT4 over n1 of v[3 n1 + n2] for each n2, twiddles W12^(n2 k1),
// then DFT3 over n2 for each k1 gives X[k1 + 4 k2].
__device__ __forceinline__ void dft12(float2 (&v)[12]) {
    const float h = 0.86602540378443864676f;   // sqrt(3) / 2
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) dft4(v[n2], v[3 + n2], v[6 + n2], v[9 + n2]);
    // row n2 = 1: W12^1, W12^2, W12^3 = -i; row n2 = 2: W12^2, W12^4, W12^6 = -1
    const float2 w1 = make_float2(h, -0.5f), w2 = make_float2(0.5f, -h), w4 = make_float2(-0.5f, -h);
    v[4] = cmul(v[4], w1);
    v[7] = cmul(v[7], w2);
    v[10] = mul_negi(v[10]);
    v[5] = cmul(v[5], w2);
    v[8] = cmul(v[8], w4);
    v[11] = make_float2(-v[11].x, -v[11].y);
    float2 x[12];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 a = v[3 * k1], b = v[3 * k1 + 1], c = v[3 * k1 + 2];
        dft3(a, b, c);
        x[k1] = a;
        x[k1 + 4] = b;
        x[k1 + 8] = c;
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = x[k];
}

// 6 = 3 x 2: DFT3 over n1 of v[2 n1 + n2] for each n2, twiddles W6^(n2 k1), then
// DFT2 over n2 for each k1 gives X[k1 + 3 k2].
__device__ __forceinline__ void dft6(float2 (&v)[6]) {
    const float h = 0.86602540378443864676f;
    dft3(v[0], v[2], v[4]);
    dft3(v[1], v[3], v[5]);
    v[3] = cmul(v[3], make_float2(0.5f, -h));
    v[5] = cmul(v[5], make_float2(-0.5f, -h));
    float2 x[6];
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        x[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
        x[k1 + 3] = csub(v[2 * k1], v[2 * k1 + 1]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = x[k];
}

template <int R>
__device__ __forceinline__ void dft_r(float2 (&v)[R]);
template <>
__device__ __forceinline__ void dft_r<3>(float2 (&v)[3]) { dft3(v[0], v[1], v[2]); }
template <>
__device__ __forceinline__ void dft_r<2>(float2 (&v)[2]) { dft2(v[0], v[1]); }
template <>
__device__ __forceinline__ void dft_r<4>(float2 (&v)[4]) { dft4(v[0], v[1], v[2], v[3]); }
template <>
__device__ __forceinline__ void dft_r<8>(float2 (&v)[8]) { dft8(v); }
template <>
__device__ __forceinline__ void dft_r<6>(float2 (&v)[6]) { dft6(v); }
template <>
__device__ __forceinline__ void dft_r<12>(float2 (&v)[12]) { dft12(v); }

// LDS layouts of a line (separate re/im planes, 32 banks of 4 bytes).  The
// Stockham stages read unit-stride and write stride-Ns patterns, the mirror
// reads reversed; these layouts keep those patterns near one cycle per
// half-wave access (chosen with a bank simulator of exactly these patterns),
// and both are paddings, at(i) = i + p (i >> s): a stage's addresses are then
// one per-thread base plus constants (LDS immediate offsets), at(b + c) =
// at(b) + at(c), which lds_layout_linear() below proves for every access of
// every instantiated transform.
//   rows (one line per T threads, lanes vary the element): three spare words
//     per 32 elements (per 16 for lines shorter than 256), short lines spaced
//     by a measured stride;
//   column tiles (lanes vary the column fastest, C columns per tile): one
//     spare word per 8 elements and a line stride of 32/C words mod 32.
template <int L>
struct LdsRows {
    static constexpr bool kLinear = true;
    static constexpr int kShift = L >= 256 ? 5 : 4;
    __host__ __device__ static constexpr int lin(int c) { return c + 3 * (c >> kShift); }
    __host__ __device__ static constexpr int at(int i) { return i + 3 * (i >> kShift); }
    __host__ __device__ static constexpr int spacing() {
        return L >= 256 ? 0 : L == 192 ? 15 : L == 128 ? 27 : L == 64 ? 15 : L == 32 ? 1 : 2;
    }
    __host__ __device__ static constexpr int words(int) { return at(L - 1) + 1 + spacing(); }
};
template <int C>
struct LdsCols {
    static constexpr bool kLinear = true;
    __host__ __device__ static constexpr int lin(int c) { return c + (c >> 3); }
    __host__ __device__ static constexpr int at(int i) { return i + (i >> 3); }
    __host__ __device__ static constexpr int words(int L) {
        return L + L / 8 + ((32 / C - (L + L / 8)) % 32 + 32) % 32;
    }
};

// Power-of-two factor of x = 2^a or 3 2^a.
constexpr int pow2_part(int x) { return (x & (x - 1)) == 0 ? x : pow2_part(x / 3); }
// Largest power-of-two radix (at most 8) that divides the per-thread count E.
constexpr int max_pow2_radix(int E) { return E % 8 == 0 ? 8 : (E % 4 == 0 ? 4 : 2); }

// Radix plan of a length-L line with E elements per thread: power-of-two
// stages of radix min(max_pow2_radix(E), what is left of 2^a); for lengths
// 3 2^a the last stage takes the factor 3 together with what is left of 2^a
// when that is 6 or 12 and E allows it (one LDS exchange fewer than a separate
// radix-3 stage), else a radix-3 stage of its own.  Every radix divides E.
constexpr int stage_radix(int left, int E) {
    return (left == 6 || left == 12) && E % left == 0
               ? left
               : (pow2_part(left) > 1 ? (pow2_part(left) < max_pow2_radix(E) ? pow2_part(left) : max_pow2_radix(E))
                                      : left);
}
template <int L, int E, int S>
struct StageRadix {
    static constexpr int done = StageRadix<L, E, S - 1>::done * StageRadix<L, E, S - 1>::R;
    static constexpr int left = L / done;
    static constexpr int R = stage_radix(left, E);
};
template <int L, int E>
struct StageRadix<L, E, 0> {
    static constexpr int done = 1;
    static constexpr int left = L;
    static constexpr int R = stage_radix(L, E);
};
template <int L, int E, int S = 0, bool END = (StageRadix<L, E, S>::done == L)>
struct NumStagesFrom {
    static constexpr int value = 1 + NumStagesFrom<L, E, S + 1>::value;
};
template <int L, int E, int S>
struct NumStagesFrom<L, E, S, true> {
    static constexpr int value = 0;
};
template <int L, int E>
struct NumStages {
    static constexpr int value = NumStagesFrom<L, E>::value;
};

// LDS word of line element i = b + c (b per thread, c a compile-time constant
// after unrolling): at(b) + lin(c) for layouts that allow it, else at(i).
template <class Lay>
__device__ __forceinline__ int lds_index(int b, int i, int c) {
    if constexpr (Lay::kLinear) return Lay::at(b) + Lay::lin(c);
    else return Lay::at(i);
}

// One Stockham stage.  FIRST reads the inputs from registers, LAST writes the
// outputs to registers; otherwise they go through the LDS line (re, im).
template <int L, int E, int S, bool FIRST, bool LAST, class Lay>
__device__ __forceinline__ void fft_stage(float2 (&v)[E], float* re, float* im, int t,
                                          const float2* __restrict__ tw) {
    constexpr int T = L / E;
    constexpr int R = StageRadix<L, E, S>::R;
    constexpr int Ns = StageRadix<L, E, S>::done;
    constexpr int Q = E / R;          // butterflies per thread
    constexpr int LR = L / R;
    static_assert(E % R == 0 && (Ns & (Ns - 1)) == 0, "radix divides E; the radix-3 stage comes last");
    float2 out[Q][R];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = t + q * T;
        float2 x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (FIRST) {
                x[r] = v[q + r * Q];
            } else {
                const int idx = lds_index<Lay>(t, j + r * LR, q * T + r * LR);
                x[r] = make_float2(re[idx], im[idx]);
            }
        }
        if (Ns > 1) {   // W^r for r < R from one table read, products at most 3 deep
            const int k = j & (Ns - 1);
            constexpr int step = twiddle_len<L>() / (Ns * R);
            float2 w[R];
            w[1] = tw[k * step];
#pragma unroll
            for (int r = 2; r < R; ++r) w[r] = cmul(w[r / 2], w[r - r / 2]);
#pragma unroll
            for (int r = 1; r < R; ++r) x[r] = cmul(x[r], w[r]);
        }
        dft_r<R>(x);
#pragma unroll
        for (int r = 0; r < R; ++r) out[q][r] = x[r];
    }
    if (!LAST) {
        __syncthreads();   // every read of this stage is done before the line is overwritten
        // write index (j / Ns) Ns R + (j mod Ns) + r Ns with j = t + q T, as a
        // per-thread base w0 plus a constant: for Ns <= T (Ns | T) it is
        // w0 = (t / Ns) Ns R + (t mod Ns) plus q T R + r Ns; for Ns > T (T | Ns)
        // it is t plus (q T / Ns) Ns R + (q T mod Ns) + r Ns.  In both cases
        // (w0 mod 8) + (constant mod 8) < 8, so LdsCols stays linear.
        constexpr bool small = Ns <= T;
        const int w0 = small ? (t / Ns) * Ns * R + (t & (Ns - 1)) : t;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j = t + q * T;
            const int k = j & (Ns - 1);
            const int base = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int c = small ? q * T * R + r * Ns : (q * T / Ns) * Ns * R + (q * T) % Ns + r * Ns;
                const int idx = lds_index<Lay>(w0, base + r * Ns, c);
                re[idx] = out[q][r].x;
                im[idx] = out[q][r].y;
            }
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) v[q + r * Q] = out[q][r];
    }
}

template <int L, int E, int S, int NS, class Lay>
struct FFTStages {
    __device__ __forceinline__ static void run(float2 (&v)[E], float* re, float* im, int t,
                                               const float2* tw) {
        fft_stage<L, E, S, S == 0, S == NS - 1, Lay>(v, re, im, t, tw);
        FFTStages<L, E, S + 1, NS, Lay>::run(v, re, im, t, tw);
    }
};
template <int L, int E, int NS, class Lay>
struct FFTStages<L, E, NS, NS, Lay> {
    __device__ __forceinline__ static void run(float2 (&)[E], float*, float*, int, const float2*) {}
};

// The thread index under a fresh name.  Kernels that run several transforms
// pass each one its own fresh index: the LDS addresses of a transform are
// functions of t alone, and when transforms share them the compiler computes
// them once and keeps them all live in registers from the first transform to
// the last (about 80 VGPRs for 12 elements per thread).  With a fresh index
// they are recomputed per transform, a few integer instructions per stage.
__device__ __forceinline__ int fresh_index(int t) {
    asm volatile("" : "+v"(t));
    return t & 1023;   // restores the known range (t < 1024): unsigned index arithmetic
}

// Forward DFT of one line, in registers.  All threads of the block must call
// it (it contains block barriers) even if their line is padding.  tw is the
// table of twiddle_len<L>() entries.
// Compile-time proof that the base-plus-constant addresses of fft_stage equal
// the layout function for every thread, butterfly, radix index and stage.
template <int L, int E, class Lay, int S = 0, bool END = (S == NumStages<L, E>::value)>
struct LayoutCheck {
    static constexpr bool ok() {
        constexpr int T = L / E, R = StageRadix<L, E, S>::R, Ns = StageRadix<L, E, S>::done, Q = E / R;
        constexpr int LR = L / R, NS = NumStages<L, E>::value;
        constexpr bool small = Ns <= T;
        for (int t = 0; t < T; ++t)
            for (int q = 0; q < Q; ++q)
                for (int r = 0; r < R; ++r) {
                    const int j = t + q * T;
                    if (S > 0 && Lay::at(t) + Lay::lin(q * T + r * LR) != Lay::at(j + r * LR)) return false;
                    if (S < NS - 1) {
                        const int w0 = small ? (t / Ns) * Ns * R + (t & (Ns - 1)) : t;
                        const int c = small ? q * T * R + r * Ns : (q * T / Ns) * Ns * R + (q * T) % Ns + r * Ns;
                        const int i = (j / Ns) * Ns * R + (j & (Ns - 1)) + r * Ns;
                        if (Lay::at(w0) + Lay::lin(c) != Lay::at(i)) return false;
                    }
                }
        return LayoutCheck<L, E, Lay, S + 1>::ok();
    }
};
template <int L, int E, class Lay, int S>
struct LayoutCheck<L, E, Lay, S, true> {
    static constexpr bool ok() { return true; }
};

template <int L, int E, class Lay = LdsRows<L>>
__device__ __forceinline__ void fft_line(float2 (&v)[E], float* re, float* im, int t,
                                         const float2* __restrict__ tw) {
    static_assert(!Lay::kLinear || LayoutCheck<L, E, Lay>::ok(), "linear LDS addresses equal the layout");
    static_assert(pow2_part(L) * (pow2_part(L) == L ? 1 : 3) == L && L >= 2 && twiddle_len<L>() % L == 0,
                  "length 2^a or 3 2^a dividing its twiddle table");
    static_assert(E == 2 || E == 4 || E == 8 || E == 12 || E == 24, "elements per thread");
    FFTStages<L, E, 0, NumStages<L, E>::value, Lay>::run(v, re, im, t, tw);
}

// Inverse (unnormalised) DFT: conj(DFT(conj(x))).
template <int L, int E, class Lay = LdsRows<L>>
__device__ __forceinline__ void ifft_line(float2 (&v)[E], float* re, float* im, int t,
                                          const float2* __restrict__ tw) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m].y = -v[m].y;
    fft_line<L, E, Lay>(v, re, im, t, tw);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m].y = -v[m].y;
}

// Store the register line to LDS in natural order / read the mirror element
// X[(L - k) mod L] of each held X[k].  Used to split the transforms of two real
// sequences packed as x + i y.  Barriers included.
template <int L, int E, class Lay = LdsRows<L>>
__device__ __forceinline__ void mirror_line(const float2 (&v)[E], float2 (&mir)[E], float* re,
                                            float* im, int t) {
    constexpr int T = L / E;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int idx = Lay::at(t + m * T);
        re[idx] = v[m].x;
        im[idx] = v[m].y;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int k = t + m * T;
        const int idx = Lay::at(k == 0 ? 0 : L - k);
        mir[m] = make_float2(re[idx], im[idx]);
    }
}

// Z = DFT(x + i y) with x, y real: X[k] = (Z[k] + conj Z[-k]) / 2, Y[k] = (Z[k] - conj Z[-k]) / 2i.
__device__ __forceinline__ float2 split_x(float2 z, float2 zm) {
    return make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
}
__device__ __forceinline__ float2 split_y(float2 z, float2 zm) {
    return make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
}

}  // namespace fmbym
