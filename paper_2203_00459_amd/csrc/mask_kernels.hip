// Kernels of the mask network: BF16 matrix-core 3x3 convolutions (forward,
// data gradient through the same kernel with flipped weights, weight gradient)
// and the FP32 element-wise layers (batch norm, ReLU, pooling, upsampling,
// head, optimiser, loss).  Every reduction runs in a fixed order, so results
// are bitwise reproducible.
//
// Matrix-core operand layout (v_mfma_f32_16x16x32_bf16): lane l holds
// A[l % 16][8 (l / 16) .. + 7], B[8 (l / 16) .. + 7][l % 16] and receives
// D[4 (l / 16) + r][l % 16], r < 4.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "mask_kernels.hpp"
#include "profile.hpp"

namespace fmbym {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

// Input channels staged per pass: all of them up to 32, else 32 or 24 at a time.
__host__ __device__ constexpr int chunk_ch(int cin) { return cin <= 32 ? cin : (cin % 32 == 0 ? 32 : 24); }

// Threads of a convolution, weight-gradient or head weight-gradient block (its
// launch bounds; a compile-time stride keeps the block-size load, and the wait
// for every load in flight it brings, out of the staging loops).
constexpr int kConvThreads = 256;

// Convolution tiles are 16 x 16 pixels (sides S >= 16): the input patch with
// its one-pixel halo is 18 x 18, 1.27 reads per output pixel where a
// 256-pixel row strip reads 3.
constexpr int kConvSide = 16;
static_assert(kConvSide * kConvSide == kConvTile, "one conv tile per block");

// Pixels of a conv tile's input patch, (rows + 2) x (cols + 2).
__host__ __device__ constexpr int patch_pixels(int /*S*/) { return (kConvSide + 2) * (kConvSide + 2); }

// Pixel pitch of the staged patch in 16-byte groups: the smallest odd count that
// holds the pixel's G groups, so that eight lanes reading eight consecutive
// pixels at a stride of an odd number of 16-byte slots touch eight different
// slots of every 128 bytes of banks.
__host__ __device__ constexpr int patch_pitch(int G) { return G | 1; }

constexpr size_t kLdsLimit = 64 * 1024;

// The convolution's output tile (256 pixels x the chunk's channels) is staged
// in LDS when it fits in kOutStageLimit bytes, so that each thread writes whole
// 16-byte groups of a pixel's channels to HBM instead of single elements: pixel
// p of the tile at element p * out_pitch.  The pitch keeps rows 16-byte aligned
// and shifts the four pixel groups of a store instruction across banks.
constexpr size_t kOutStageLimit = 40 * 1024;
__host__ __device__ constexpr int out_pitch(int co, int elem) { return co + 16 / elem; }
__host__ __device__ constexpr size_t out_tile_bytes(int co, int elem) {
    return (size_t)kConvTile * out_pitch(co, elem) * elem;
}
__host__ __device__ constexpr bool out_staged(int co, int elem) { return out_tile_bytes(co, elem) <= kOutStageLimit; }

// The weights of a block's output channels are staged in LDS, once per block,
// when the input is staged in one pass (cin <= 32) and they take at most
// kWStageLimit bytes: the B fragments then come from LDS, and no global load
// in the tile loop waits behind the next tile's patch loads (the vector-memory
// counter is in order).  Rows of cin 9 weights at a pitch of an odd number of
// 16-byte slots.
constexpr size_t kWStageLimit = 28 * 1024;
__host__ __device__ constexpr int w_pitch(int cin) { return (9 * cin * 2 / 16) % 2 == 0 ? 9 * cin + 8 : 9 * cin; }
__host__ __device__ constexpr size_t w_stage_bytes(int cin, int co) {
    return cin <= 32 && (size_t)co * w_pitch(cin) * 2 <= kWStageLimit ? (size_t)co * w_pitch(cin) * 2 : 0;
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), as_bf16x8(b), c, 0, 0, 0);
}

// Output tile of conv block `blk`: image, first row/column, rows x cols.
struct TileGeo {
    int img, y0, x0, pr, pc;
};

// The convolution's tile: 16 x 16 pixels, tiles row-major within the image.
__device__ __forceinline__ TileGeo conv_tile_geo(int blk, int S) {
    TileGeo t;
    const int per_row = S / kConvSide, per_img = per_row * per_row;
    t.img = blk / per_img;
    const int k = blk % per_img;
    t.pr = t.pc = kConvSide;
    t.y0 = (k / per_row) * kConvSide;
    t.x0 = (k % per_row) * kConvSide;
    return t;
}

// 1-D taps of the half-pixel bilinear x2 upsampling at output o of a length-n input.
__device__ __forceinline__ void up_taps(int o, int n, int& i0, int& i1, float& w1) {
    const float s = fmaxf(0.f, 0.5f * (float)o - 0.25f);
    i0 = (int)s;
    w1 = s - (float)i0;
    i1 = min(i0 + 1, n - 1);
}

// Side of the low-resolution region an up-concat tile interpolates from: the
// patch rows y0 - 1 .. y0 + 16 fall between low-resolution rows y0/2 - 1 and
// y0/2 + 8 (the same for columns).
constexpr int kUpSide = kConvSide / 2 + 2;

// Dynamic LDS bytes of a convolution's staged input: the patch at a pitch of
// patch_pitch(G) 16-byte groups per pixel, and for the up-concat input the
// low-resolution entries after it.
__host__ __device__ constexpr size_t conv_in_bytes(int cin, int src) {
    return (size_t)patch_pixels(0) * patch_pitch(chunk_ch(cin) / 8) * 16 +
           (src == kSrcUpCat ? (size_t)kUpSide * kUpSide * (chunk_ch(cin) / 8) * 16 : 0);
}

// Bytes of the region before a convolution's staged weights: the staged input
// or, when it is staged, the output tile (elem bytes per value), in 16-byte units.
__host__ __device__ constexpr size_t conv_lds_region(int cin, int src, int co, int elem) {
    return ((conv_in_bytes(cin, src) > (out_staged(co, elem) ? out_tile_bytes(co, elem) : 0)
                 ? conv_in_bytes(cin, src)
                 : (out_staged(co, elem) ? out_tile_bytes(co, elem) : 0)) +
            15) / 16 * 16;
}

// Channel groups of the chunk starting at channel c0 that come from the
// upsampled deeper activation (the first 2 CIN / 3 channels of an up-concat
// input); the chunk's remaining groups come from the skip activation.
template <int CIN, int SRC>
__device__ __forceinline__ int up_groups(int c0, int G) {
    if constexpr (SRC != kSrcUpCat) {
        return 0;
    } else {
        const int d = 2 * CIN / 3 / 8 - c0 / 8;
        return d < 0 ? 0 : (d > G ? G : d);
    }
}

// Entries of a tile's staged input for a chunk of G groups of 8 channels, dg
// of them upsampled: plain and up-concat skip entries are (patch pixel, group)
// pairs, scan entries one patch pixel each, and the up-concat input adds the
// deeper activation's dg groups at the kUpSide^2 low-resolution pixels.
template <int SRC>
__host__ __device__ constexpr int stage_entries(int G, int dg) {
    return SRC == kSrcScan ? (kConvSide + 2) * (kConvSide + 2)
                           : (kConvSide + 2) * (kConvSide + 2) * (G - dg) + kUpSide * kUpSide * dg;
}

// Entry `it` of the staged input of the chunk at channel c0 (zeros outside
// the image):
//   plain: pixel it / G of the patch, group it % G of the input;
//   scans: pixel it of the patch, the scan planes' values as FP32 bits in the
//          first lanes (rounded to BF16 when stored, as channels 0 and 1);
//   up-concat: first pixel q, group dg + k of the chunk from the skip
//          activation for it = q (G - dg) + k, then the deeper activation's
//          groups k < dg at low-resolution pixel q of the kUpSide^2 region.
template <int CIN, int SRC>
__device__ __forceinline__ u32x4 fetch_entry(const ConvSrc& src, const TileGeo& t, int S, int c0, int G, int dg,
                                             int it) {
    constexpr int W = kConvSide + 2;
    u32x4 v = {0u, 0u, 0u, 0u};
    if constexpr (SRC == kSrcPlain) {
        const int q = it / G, cg = it % G;
        const int y = t.y0 - 1 + q / W, x = t.x0 - 1 + q % W;
        if (y >= 0 && y < S && x >= 0 && x < S)
            v = *(const u32x4*)(src.in + (((size_t)t.img * S + y) * S + x) * CIN + c0 + 8 * cg);
    } else if constexpr (SRC == kSrcScan) {
        const int y = t.y0 - 1 + it / W, x = t.x0 - 1 + it % W;
        if (y >= 0 && y < S && x >= 0 && x < S) {
            const size_t p = (size_t)y * S + x;
            if (src.x_tab) {
                v[0] = __float_as_uint(src.x_tab[t.img][p]);
            } else {
                const size_t pi = (size_t)t.img * S * S + p;
                v[0] = __float_as_uint(src.x[pi]);
                if (src.ch > 1) v[1] = __float_as_uint(src.x[src.plane + pi]);
            }
        }
    } else {
        constexpr int CD = 2 * CIN / 3, CE = CIN - CD;
        const int sg = G - dg, nskip = W * W * sg;
        if (it < nskip) {
            const int q = it / sg, k = it % sg;
            const int y = t.y0 - 1 + q / W, x = t.x0 - 1 + q % W;
            if (y >= 0 && y < S && x >= 0 && x < S)
                v = *(const u32x4*)(src.skip + (((size_t)t.img * S + y) * S + x) * CE + c0 + 8 * (dg + k) - CD);
        } else {
            const int j = it - nskip, q = j / dg, k = j % dg, H = S / 2;
            const int ly = t.y0 / 2 - 1 + q / kUpSide, lx = t.x0 / 2 - 1 + q % kUpSide;
            if (ly >= 0 && ly < H && lx >= 0 && lx < H)
                v = *(const u32x4*)(src.in + (((size_t)t.img * H + ly) * H + lx) * CD + c0 + 8 * k);
        }
    }
    return v;
}

// Write entry `it` to LDS: patch pixel q at patch[q * pitch + group]; the
// up-concat input's low-resolution entries after the patch.
template <int SRC>
__device__ __forceinline__ void put_entry(u32x4* patch, int pitch, int G, int dg, int it, u32x4 v) {
    constexpr int W = kConvSide + 2;
    if constexpr (SRC == kSrcPlain) {
        patch[(it / G) * pitch + it % G] = v;
    } else if constexpr (SRC == kSrcScan) {
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = (bf16)0.f;
        o[0] = (bf16)__uint_as_float(v[0]);
        o[1] = (bf16)__uint_as_float(v[1]);
        patch[it * pitch] = __builtin_bit_cast(u32x4, o);
    } else {
        const int sg = G - dg, nskip = W * W * sg;
        if (it < nskip)
            patch[(it / sg) * pitch + dg + it % sg] = v;
        else
            patch[W * W * pitch + (it - nskip)] = v;
    }
}

// The up-concat input's first dg groups of every patch pixel: the bilinear x2
// upsampling of the low-resolution entries staged after the patch (the
// arithmetic of the upsampling layer, rounded to BF16).
__device__ __forceinline__ void up_interp(u32x4* patch, int pitch, int dg, const TileGeo& t, int S) {
    constexpr int W = kConvSide + 2;
    const u32x4* lr = patch + W * W * pitch;
    const int H = S / 2, ly0 = t.y0 / 2 - 1, lx0 = t.x0 / 2 - 1;
    for (int it = threadIdx.x; it < W * W * dg; it += kConvThreads) {
        const int q = it / dg, k = it % dg;
        const int y = t.y0 - 1 + q / W, x = t.x0 - 1 + q % W;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (y >= 0 && y < S && x >= 0 && x < S) {
            int y0, y1, x0, x1;
            float wy, wx;
            up_taps(y, H, y0, y1, wy);
            up_taps(x, H, x0, x1, wx);
            const bf16x8 a = as_bf16x8(lr[((y0 - ly0) * kUpSide + x0 - lx0) * dg + k]);
            const bf16x8 b = as_bf16x8(lr[((y0 - ly0) * kUpSide + x1 - lx0) * dg + k]);
            const bf16x8 c = as_bf16x8(lr[((y1 - ly0) * kUpSide + x0 - lx0) * dg + k]);
            const bf16x8 d = as_bf16x8(lr[((y1 - ly0) * kUpSide + x1 - lx0) * dg + k]);
            bf16x8 o;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float top = (1.f - wx) * (float)a[j] + wx * (float)b[j];
                const float bot = (1.f - wx) * (float)c[j] + wx * (float)d[j];
                o[j] = (bf16)((1.f - wy) * top + wy * bot);
            }
            v = __builtin_bit_cast(u32x4, o);
        }
        patch[q * pitch + k] = v;
    }
}

// ------------------------------------------------------------ convolution

// out = conv3x3(in, w) over one 16 x 16-pixel tile per block (blockIdx.x) and
// one chunk of output channels (blockIdx.y): all of them up to 96, else 64 at
// a time, so that the accumulators stay within 96 registers.  K runs over (tap, input
// channel) in groups of 8; every 32-wide K step is one matrix-core instruction
// per (16-pixel M-tile, 16-channel N-tile).  Each wave owns 4 M-tiles; A comes
// from the LDS patch, B from the packed weights.
// MODE kConvDgrad: out is FP32 (the data gradient).  kConvTrain: out = z in
// BF16 and the block's sums of the stored z and z^2 go to part.  kConvInfer:
// out = relu(z scale + shift) in BF16 with the running statistics' scale and
// shift (inference; no z, no partials).
__host__ __device__ constexpr int co_chunk(int cout) { return cout > 96 ? 64 : cout; }
// A launch with few tiles (the deep levels) takes its output channels in
// smaller chunks, half or a quarter of co_chunk down to 16, until it has at
// least kConvMinBlocks blocks: more blocks to fill the GPU, each staging the
// same input patch.
constexpr int kConvMinBlocks = 512;
inline int conv_chunk(int cout, int blocks) {
    int co = co_chunk(cout);
    for (int k = 0; k < 2 && co % 32 == 0 && blocks * (cout / co) < kConvMinBlocks; ++k) co /= 2;
    return co;
}

// Waves per SIMD the compiler must leave room for, where measured faster than
// its own register choice (1: no constraint): the 24- and 48-channel up-concat
// inference convolutions at 4 (361 against 403 us and 212 against 238 us at
// 64 x 512^2; the 48-channel one spills 8 bytes) and the 8-channel pooling one
// at 6 (154 against 165 us).  Others lost time or spilled more at a higher count.
constexpr int conv_waves(int cin, int mode, int src, bool pool) {
    return mode != kConvInfer ? 1 : (src == kSrcUpCat && (cin == 24 || cin == 48) ? 4 : (pool && cin == 8 ? 6 : 1));
}

template <int CIN, int COUT, int MODE, int CO_ = co_chunk(COUT), int SRC = kSrcPlain, bool POOL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(conv_waves(CIN, MODE, SRC, POOL)))) void
k_conv3x3(ConvSrc src, const bf16* __restrict__ w,
                                                 void* __restrict__ outv, float* __restrict__ part,
                                                 bf16* __restrict__ pool, int S, BnInfer bn, int tpb, int tiles) {
    using OutT = typename std::conditional<MODE == kConvDgrad, float, bf16>::type;
    OutT* __restrict__ out = static_cast<OutT*>(outv);
    constexpr bool STATS = MODE == kConvTrain;
    constexpr int CC = chunk_ch(CIN), NCH = CIN / CC, G = CC / 8, NQ = 9 * G, NS = (NQ + 3) / 4;
    constexpr int CO = CO_, NT = pad16(CO) / 16, K = 9 * CIN;
    static_assert(COUT % CO == 0, "whole output-channel chunks");
    const int co0 = blockIdx.y * CO;
    static_assert(CIN % 8 == 0 && CIN % CC == 0, "input channels in groups of 8");
    static_assert(SRC == kSrcPlain || MODE == kConvInfer, "fused inputs in inference only");
    static_assert(SRC != kSrcScan || CIN == 8, "scans feed the 8-channel first convolution");
    static_assert(SRC != kSrcUpCat || CIN % 24 == 0, "up-concat input: 2 CIN / 3 upsampled, CIN / 3 skip channels");
    static_assert(!POOL || (MODE == kConvInfer && out_staged(CO_, 2)), "pooling from the staged output tile");
    constexpr int PITCH = patch_pitch(G);
    // LDS: the staged input (conv_in_bytes) or output tile, then the weights
    constexpr size_t R0 = conv_lds_region(CIN, SRC, CO_, (int)sizeof(OutT));
    constexpr int KP = w_pitch(CIN);
    constexpr bool WLDS = w_stage_bytes(CIN, CO_) > 0;
    extern __shared__ u32x4 patch[];
    bf16* wl = reinterpret_cast<bf16*>(reinterpret_cast<char*>(patch) + R0);
    if constexpr (WLDS) {
        // read by the compute only after the first tile's barriers
        for (int it = threadIdx.x; it < CO_ * (K / 8); it += kConvThreads) {
            const int co = it / (K / 8), kg = it % (K / 8);
            *(u32x4*)(wl + co * KP + 8 * kg) = *(const u32x4*)(w + (size_t)(co0 + co) * K + 8 * kg);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    constexpr int W = kConvSide + 2;
    int prow[4], pcol[4];
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        const int p = (wave + 4 * mi) * 16 + r16;
        prow[mi] = p / kConvSide;
        pcol[mi] = p % kConvSide;
    }
    // With the whole patch in one pass (CIN <= 32), the patches of the next PD
    // tiles are loaded into registers while the current one is computed: two
    // tiles ahead when a patch takes at most three loads per thread (the small
    // layers, whose compute is too short to cover one load's latency), else one.
    constexpr bool PREF = NCH == 1;
    constexpr int DG0 = SRC == kSrcUpCat ? (2 * CIN / 3 / 8 < G ? 2 * CIN / 3 / 8 : G) : 0;
    constexpr int NE = stage_entries<SRC>(G, DG0);   // entries of the one chunk (c0 = 0)
    constexpr int PLOADS = (NE + 255) / 256;
    constexpr int PD = 1;
    constexpr int NPRE = PREF ? PLOADS : 1;
    u32x4 preA[NPRE], preB[NPRE];
    const int tile0 = blockIdx.x * tpb, tile1 = min(tiles, tile0 + tpb);
    auto prefetch = [&](u32x4 (&pre)[NPRE], int tile) {
        const TileGeo tn = conv_tile_geo(tile, S);
#pragma unroll
        for (int k = 0; k < PLOADS; ++k) {
            const int it = threadIdx.x + 256 * k;
            pre[k] = it < NE ? fetch_entry<CIN, SRC>(src, tn, S, 0, G, DG0, it) : u32x4{0u, 0u, 0u, 0u};
        }
    };
    if constexpr (PREF) {
        prefetch(preA, tile0);
        if constexpr (PD == 2)
            if (tile0 + 1 < tile1) prefetch(preB, tile0 + 1);
    }
    // inference: batch norm on the running statistics and ReLU on the BF16-rounded
    // output, the arithmetic of the training pass's statistics and BN + ReLU passes
    float csc[NT], csh[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        csc[nt] = csh[nt] = 0.f;
        if constexpr (MODE == kConvInfer) {
            const int c = co0 + nt * 16 + r16;
            if (nt * 16 + r16 < CO) {
                const double mean = bn.run_mean[c], var = bn.run_var[c];
                const double inv = 1.0 / sqrt(var + (double)bn.eps);
                const double sc = (double)bn.gamma[c] * inv;
                csc[nt] = (float)sc;
                csh[nt] = (float)((double)bn.beta[c] - mean * sc);
            }
        }
    }
    float s1[NT], s2[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) s1[nt] = s2[nt] = 0.f;
    auto body = [&](int tile, u32x4 (&pre)[NPRE]) {
        const TileGeo t = conv_tile_geo(tile, S);
        f32x4 acc[4][NT];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mi][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        const u32x4 zero = {0u, 0u, 0u, 0u};
        for (int ch = 0; ch < NCH; ++ch) {
            const int c0 = ch * CC;
            __syncthreads();   // the previous patch (or staged output) has been read
            const int dg = up_groups<CIN, SRC>(c0, G);
            if constexpr (PREF) {
#pragma unroll
                for (int k = 0; k < PLOADS; ++k) {
                    const int it = threadIdx.x + 256 * k;
                    if (it < NE) put_entry<SRC>(patch, PITCH, G, DG0, it, pre[k]);
                }
                if (tile + PD < tile1) prefetch(pre, tile + PD);
            } else {
                const int ne = stage_entries<SRC>(G, dg);
                for (int it = threadIdx.x; it < ne; it += kConvThreads)
                    put_entry<SRC>(patch, PITCH, G, dg, it, fetch_entry<CIN, SRC>(src, t, S, c0, G, dg, it));
            }
            if constexpr (SRC == kSrcUpCat) {
                __syncthreads();
                up_interp(patch, PITCH, dg, t, S);
            }
            __syncthreads();
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                const int q = 4 * st + g;
                const bool valid = q < NQ;
                const int tap = valid ? q / G : 0, cg = q % G;
                const int ky = tap / 3, kx = tap % 3;
                u32x4 a[4], b[NT];
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
                    a[mi] = valid ? patch[((prow[mi] + ky) * W + pcol[mi] + kx) * PITCH + cg] : zero;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int co = nt * 16 + r16;
                    if constexpr (WLDS)
                        b[nt] = (valid && co < CO) ? *(const u32x4*)(wl + co * KP + tap * CIN + c0 + 8 * cg) : zero;
                    else
                        b[nt] = (valid && co < CO)
                                    ? *(const u32x4*)(w + (size_t)(co0 + co) * K + tap * CIN + c0 + 8 * cg)
                                    : zero;
                }
#pragma unroll
                for (int mi = 0; mi < 4; ++mi)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[mi][nt] = mfma(a[mi], b[nt], acc[mi][nt]);
            }
        }
        const size_t img_base = (size_t)t.img * S * S;
        constexpr int ELEM = (int)sizeof(OutT), TP = out_pitch(CO, ELEM);
        constexpr bool STAGED = out_staged(CO, ELEM);
        OutT* stage = reinterpret_cast<OutT*>(patch);
        if constexpr (STAGED) __syncthreads();   // every wave is done with the patch
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = (wave + 4 * mi) * 16 + 4 * g + r;
                const size_t pix = img_base + (size_t)(t.y0 + p / t.pc) * S + t.x0 + p % t.pc;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int co = nt * 16 + r16;
                    if (co >= CO) continue;
                    const float v = acc[mi][nt][r];
                    OutT o;
                    if constexpr (STATS) {
                        const bf16 h = (bf16)v;
                        o = h;
                        const float hv = (float)h;
                        s1[nt] += hv;
                        s2[nt] += hv * hv;
                    } else if constexpr (MODE == kConvInfer) {
                        o = (bf16)fmaxf(fmaf((float)(bf16)v, csc[nt], csh[nt]), 0.f);
                    } else {
                        o = v;
                    }
                    if constexpr (STAGED) stage[p * TP + co] = o;
                    else out[pix * COUT + co0 + co] = o;
                }
            }
        if constexpr (STAGED) {
            __syncthreads();
            constexpr int VEC = 16 / ELEM, VPP = CO / VEC;   // 16-byte groups per pixel
            static_assert(CO % VEC == 0, "whole 16-byte groups per pixel");
            for (int it = threadIdx.x; it < kConvTile * VPP; it += kConvThreads) {
                const int p = it / VPP, q = it % VPP;
                const size_t pix = img_base + (size_t)(t.y0 + p / t.pc) * S + t.x0 + p % t.pc;
                *(u32x4*)(out + pix * COUT + co0 + q * VEC) = *(const u32x4*)(stage + p * TP + q * VEC);
            }
            if constexpr (POOL) {
                // 2 x 2 max pooling of the tile into the next level's input [I][S/2][S/2][COUT]
                const int H = S / 2;
                for (int it = threadIdx.x; it < kConvTile / 4 * VPP; it += kConvThreads) {
                    const int pp = it / VPP, q = it % VPP;
                    const int py = pp / (kConvSide / 2), px = pp % (kConvSide / 2);
                    const int p00 = 2 * py * kConvSide + 2 * px;
                    const bf16x8 v00 = as_bf16x8(*(const u32x4*)(stage + p00 * TP + q * VEC));
                    const bf16x8 v01 = as_bf16x8(*(const u32x4*)(stage + (p00 + 1) * TP + q * VEC));
                    const bf16x8 v10 = as_bf16x8(*(const u32x4*)(stage + (p00 + kConvSide) * TP + q * VEC));
                    const bf16x8 v11 = as_bf16x8(*(const u32x4*)(stage + (p00 + kConvSide + 1) * TP + q * VEC));
                    bf16x8 o;
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        o[j] = (bf16)fmaxf(fmaxf((float)v00[j], (float)v01[j]), fmaxf((float)v10[j], (float)v11[j]));
                    const size_t pq = ((size_t)t.img * H + t.y0 / 2 + py) * H + t.x0 / 2 + px;
                    *(u32x4*)(pool + pq * COUT + co0 + q * VEC) = __builtin_bit_cast(u32x4, o);
                }
            }
        }
    };
    if constexpr (PD == 2) {
        for (int tile = tile0; tile < tile1; tile += 2) {
            body(tile, preA);
            if (tile + 1 < tile1) body(tile + 1, preB);
        }
    } else {
        for (int tile = tile0; tile < tile1; ++tile) body(tile, preA);
    }
    if constexpr (STATS) {
        __shared__ float red[4][2][NT * 16];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            s1[nt] += __shfl_xor(s1[nt], 16);
            s1[nt] += __shfl_xor(s1[nt], 32);
            s2[nt] += __shfl_xor(s2[nt], 16);
            s2[nt] += __shfl_xor(s2[nt], 32);
            if (g == 0) {
                red[wave][0][nt * 16 + r16] = s1[nt];
                red[wave][1][nt * 16 + r16] = s2[nt];
            }
        }
        __syncthreads();
        for (int c = threadIdx.x; c < CO; c += kConvThreads) {
            float a = 0.f, b = 0.f;
#pragma unroll
            for (int wv = 0; wv < 4; ++wv) {
                a += red[wv][0][c];
                b += red[wv][1][c];
            }
            part[(size_t)blockIdx.x * 2 * COUT + co0 + c] = a;
            part[(size_t)blockIdx.x * 2 * COUT + COUT + co0 + c] = b;
        }
    }
}

// Weight-gradient geometry.  N runs over base columns (ky, ci) of one channel
// chunk, in groups of 16; each group feeds three N-tiles, one per kx, whose B
// fragments come from the same two aligned LDS reads (the kx shift is a
// 16-bit funnel shift).  With fewer than 4 groups the 4 waves split the
// pixel steps instead and their accumulators are summed in wave order.
template <int CIN, int COUT, int CO_ = co_chunk(COUT)>
struct WgradGeo {
    static constexpr int CC = chunk_ch(CIN), NCH = CIN / CC;
    static constexpr int CO = CO_;   // output channels per block (blockIdx.y chunks)
    static constexpr int MT = pad16(CO) / 16, NB = 3 * CC, NG = (NB + 15) / 16;
    static constexpr int WG = NG >= 4 ? 4 : 1;            // waves across groups
    static constexpr int GPW = (NG + WG - 1) / WG;        // groups per wave
    static constexpr int KPW = (kConvTile / 32) * WG / 4; // pixel steps per wave
    static constexpr size_t red_bytes = WG == 1 ? (size_t)MT * GPW * 3 * 64 * 16 : 0;
};

// The input patch of a 16 x 16 tile, transposed: 18 rows at a pitch of 24
// (a B fragment reads 10 pixels from an 8-pixel-aligned column, 16-byte aligned).
__host__ __device__ constexpr int wg_pitch(int /*S*/) { return kConvSide + 8; }
__host__ __device__ constexpr int wg_rows(int /*S*/) { return kConvSide + 2; }
// LDS strides of the weight gradient's staged operands, in bf16 elements: the
// dz tile's channel rows and the patch's channel planes are padded to an odd
// number of 16-byte slots, so that the lanes of a fragment read (consecutive
// channels) fall on different slots of every 128 bytes of banks.
constexpr int kDztPitch = kConvTile + 8;
__host__ __device__ constexpr int wg_plane(int S) { return wg_rows(S) * wg_pitch(S) + 8; }

// Weight gradient over `tpb` consecutive tiles per block (blockIdx.x) for the
// output channels of chunk blockIdx.y:
// part[block][co][tap CIN + ci] = sum over the tiles' pixels of dz[p][co] in[p + tap][ci].
// M = output channels, K = pixels (8 per lane: one tile row), N = (tap, ci).
// Input-channel chunks (blockIdx.z of gridDim.z) write disjoint columns, so
// launches with few tiles spread them over blocks with the same sums.
// LDS: the chunk's dz tile transposed [CO][kDztPitch], the input patch transposed
// per channel [CC][rows][pitch] (pixels contiguous), and the wave-reduction area.
template <int CIN, int COUT, int CO_ = co_chunk(COUT)>
__global__ __launch_bounds__(256) void k_wgrad(const bf16* __restrict__ dz, const bf16* __restrict__ in,
                                               float* __restrict__ part, int S, int tpb, int tiles) {
    using Geo = WgradGeo<CIN, COUT, CO_>;
    constexpr int CC = Geo::CC, CO = Geo::CO, MT = Geo::MT, NB = Geo::NB, NG = Geo::NG, WG = Geo::WG,
                  GPW = Geo::GPW, KPW = Geo::KPW;
    constexpr int K = 9 * CIN;
    static_assert(COUT % CO == 0 && CO % 8 == 0, "whole output-channel chunks of 8-channel groups");
    const int co0 = blockIdx.y * CO;
    extern __shared__ u32x4 smem[];
    bf16* dzt = reinterpret_cast<bf16*>(smem);                       // [CO][kDztPitch]
    bf16* pt = dzt + CO * kDztPitch;                                 // [CC][plane: rows x pitch]
    const int PW = wg_pitch(S), PRW = wg_rows(S), PL = wg_plane(S);
    f32x4* red = reinterpret_cast<f32x4*>(pt + (size_t)CC * PL);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const u32x4 zero = {0u, 0u, 0u, 0u};
    const int nch = Geo::NCH / gridDim.z;   // the launcher makes it divide
    for (int ch = blockIdx.z * nch; ch < (blockIdx.z + 1) * nch; ++ch) {
        const int c0 = ch * CC;
        f32x4 acc[MT][GPW][3];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int gi = 0; gi < GPW; ++gi)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) acc[mt][gi][kx] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k = 0; k < tpb; ++k) {
            const int tile = blockIdx.x * tpb + k;
            if (tile >= tiles) break;
            const TileGeo t = conv_tile_geo(tile, S);
            const size_t img_base = (size_t)t.img * S * S;
            __syncthreads();
            // the chunk's dz tile, transposed
            for (int it = threadIdx.x; it < kConvTile * CO / 8; it += kConvThreads) {
                const int p = it / (CO / 8), cg = it % (CO / 8);
                const size_t pix = img_base + (size_t)(t.y0 + p / t.pc) * S + t.x0 + p % t.pc;
                const bf16x8 v = __builtin_bit_cast(bf16x8, *(const u32x4*)(dz + pix * COUT + co0 + 8 * cg));
#pragma unroll
                for (int j = 0; j < 8; ++j) dzt[(8 * cg + j) * kDztPitch + p] = v[j];
            }
            // input patch of the chunk, transposed per channel
            {
                const int W = t.pc + 2, npix = (t.pr + 2) * W;
                const bf16* base = in + (size_t)t.img * S * S * CIN;
                for (int it = threadIdx.x; it < npix * (CC / 8); it += kConvThreads) {
                    const int q = it / (CC / 8), cg = it % (CC / 8);
                    const int r = q / W, c = q % W;
                    const int y = t.y0 - 1 + r, x = t.x0 - 1 + c;
                    u32x4 u = zero;
                    if (y >= 0 && y < S && x >= 0 && x < S)
                        u = *(const u32x4*)(base + ((size_t)y * S + x) * CIN + c0 + 8 * cg);
                    const bf16x8 v = __builtin_bit_cast(bf16x8, u);
#pragma unroll
                    for (int j = 0; j < 8; ++j) pt[(size_t)(8 * cg + j) * PL + r * PW + c] = v[j];
                }
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KPW; ++kk) {
                const int st = WG == 4 ? kk : wave * KPW + kk;
                const int p0 = 32 * st + 8 * g;
                const int row = p0 / t.pc, col = p0 % t.pc;
                u32x4 a[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int co = mt * 16 + r16;
                    a[mt] = co < CO ? *(const u32x4*)(dzt + co * kDztPitch + p0) : zero;
                }
#pragma unroll
                for (int gi = 0; gi < GPW; ++gi) {
                    const int gp = WG == 4 ? wave + 4 * gi : gi;
                    if (gp >= NG) break;
                    const int bc = gp * 16 + r16;
                    u32x4 b0 = zero, b1 = zero, b2 = zero;
                    if (bc < NB) {
                        const int ky = bc / CC, ci = bc % CC;
                        const bf16* src = pt + (size_t)ci * PL + (row + ky) * PW + col;
                        const u32x4 w = *(const u32x4*)src;
                        const unsigned w4 = *(const unsigned*)(src + 8);
                        b0 = w;
                        b1 = u32x4{__builtin_amdgcn_alignbyte(w[1], w[0], 2), __builtin_amdgcn_alignbyte(w[2], w[1], 2),
                                   __builtin_amdgcn_alignbyte(w[3], w[2], 2), __builtin_amdgcn_alignbyte(w4, w[3], 2)};
                        b2 = u32x4{w[1], w[2], w[3], w4};
                    }
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        acc[mt][gi][0] = mfma(a[mt], b0, acc[mt][gi][0]);
                        acc[mt][gi][1] = mfma(a[mt], b1, acc[mt][gi][1]);
                        acc[mt][gi][2] = mfma(a[mt], b2, acc[mt][gi][2]);
                    }
                }
            }
        }
        if constexpr (WG == 1) {
            // waves hold partial sums over their pixel steps: add them in wave order
            for (int wv = 0; wv < 4; ++wv) {
                __syncthreads();
                if (wave == wv) {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int gi = 0; gi < GPW; ++gi)
#pragma unroll
                            for (int kx = 0; kx < 3; ++kx) {
                                f32x4& r = red[((mt * GPW + gi) * 3 + kx) * 64 + lane];
                                if (wv == 0)
                                    r = acc[mt][gi][kx];
                                else
                                    r = r + acc[mt][gi][kx];
                                acc[mt][gi][kx] = r;
                            }
                }
            }
            if (wave != 3) continue;   // wave 3 now holds the block's sums (block-uniform per wave)
        }
        float* pb = part + (size_t)blockIdx.x * COUT * K;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int gi = 0; gi < GPW; ++gi) {
                const int gp = WG == 4 ? wave + 4 * gi : gi;
                if (gp >= NG) break;
                const int bc = gp * 16 + r16;
                if (bc >= NB) continue;
                const int ky = bc / CC, ci = bc % CC;
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int kg = (ky * 3 + kx) * CIN + c0 + ci;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int co = mt * 16 + 4 * g + r;
                        if (co < CO) pb[(size_t)(co0 + co) * K + kg] = acc[mt][gi][kx][r];
                    }
                }
            }
    }
}

// Column sums of a [nb][stride] partial array, in two fixed-order stages so
// that both read coalesced rows: stage 1 gives tmp[c][j] = sum over the rows of
// chunk c (`per` rows, 4 interleaved lanes added in lane order), stage 2 adds
// the chunks in order (in double precision).
constexpr int kColChunks = 64;

__global__ __launch_bounds__(256) void k_colsum1(const float* __restrict__ part, int nb, long long stride,
                                                 int n, int per, float* __restrict__ tmp) {
    const int t = threadIdx.x & 63, bl = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + t;
    const int b0 = blockIdx.y * per, b1 = min(nb, b0 + per);
    float s = 0.f;
    if (j < n) {
        // eight loads in flight, then added in row order (the same sums as one at a time)
        int b = b0 + bl;
        for (; b + 28 < b1; b += 32) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(b + 4 * u) * stride + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; b < b1; b += 4) s += part[(size_t)b * stride + j];
    }
    __shared__ float r[4][64];
    r[bl][t] = s;
    __syncthreads();
    if (bl == 0 && j < n) tmp[(size_t)blockIdx.y * n + j] = ((r[0][t] + r[1][t]) + r[2][t]) + r[3][t];
}

// With cink > 0 the columns are a weight gradient in the packed K order
// [co][tap][ci < cink] and land in the parameter layout [co][ci][tap] (ci < cin;
// the padding channels are dropped); otherwise out[j] is column j0 + j.
__global__ void k_colsum2(const float* __restrict__ tmp, int nbc, int n, int j0, int count,
                          float* __restrict__ out, int cin, int cink) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    int dest = j;
    if (cink > 0) {
        const int co = j / (9 * cink), k = j % (9 * cink), tap = k / cink, ci = k % cink;
        if (ci >= cin) return;
        dest = (co * cin + ci) * 9 + tap;
    }
    double s = 0.0;
    int c = 0;
    for (; c + 8 <= nbc; c += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = tmp[(size_t)(c + u) * n + j0 + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nbc; ++c) s += tmp[(size_t)c * n + j0 + j];
    out[dest] = (float)s;
}

// The head's second stage: column j = o (9 C + 1) + r of tmp is dw[o][r] for
// r < 9 C (the [ch][C][3][3] layout) and db[o] for r = 9 C; each a sum of the
// chunks in order in double precision, as k_colsum2 adds them.
__global__ void k_head_colsum2(const float* __restrict__ tmp, int nbc, int n, float* __restrict__ dw,
                               float* __restrict__ db) {
    constexpr int NW = 9 * 8 + 1;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    int c = 0;
    for (; c + 8 <= nbc; c += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = tmp[(size_t)(c + u) * n + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nbc; ++c) s += tmp[(size_t)c * n + j];
    const int o = j / NW, r = j % NW;
    if (r < NW - 1)
        dw[o * (NW - 1) + r] = (float)s;
    else
        db[o] = (float)s;
}

// ------------------------------------------------------------ element-wise

// Scan -> 8-channel BF16 input; image i is x + i S^2, or x_tab[i] for a table of scans.
// Channel c of pixel p is plane c of x (x + c npix + p) for the dual-input network.
__global__ void k_input8(const float* __restrict__ x, const float* const* __restrict__ x_tab,
                         bf16* __restrict__ x8, long long npix, int S2, int ch) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (bf16)0.f;
    if (x_tab) {
        v[0] = (bf16)x_tab[p / S2][p % S2];
    } else {
        v[0] = (bf16)x[p];
        if (ch > 1) v[1] = (bf16)x[npix + p];
    }
    *(u32x4*)(x8 + p * 8) = __builtin_bit_cast(u32x4, v);
}

// d x of the network input (plane ci of ch): the first convolution's adjoint
// in FP32, one pixel per thread, taps and channels summed in a fixed order
// (ky, kx, c); w is the FP32 weight [C][ch][3][3].
__global__ void k_input_grad(const bf16* __restrict__ dz, const float* __restrict__ w, float* __restrict__ dx,
                             long long npix, int S, int C, int ch) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npix * ch) return;
    const int ci = (int)(q / npix);
    const long long p = q % npix;
    const int S2 = S * S;
    const long long img = p / S2;
    const int i = (int)(p % S2) / S, j = (int)(p % S2) % S;
    float acc = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
        const int y = i + 1 - ky;           // forward: z[y][x] reads in[y + ky - 1][x + kx - 1]
        if (y < 0 || y >= S) continue;
        for (int kx = 0; kx < 3; ++kx) {
            const int x = j + 1 - kx;
            if (x < 0 || x >= S) continue;
            const bf16* d = dz + ((img * S2) + (long long)y * S + x) * C;
            for (int c = 0; c < C; ++c) acc += w[(c * ch + ci) * 9 + ky * 3 + kx] * (float)d[c];
        }
    }
    dx[q] = acc;
}

// Per-thread sums of one channel's partial pairs over the blocks k = t, t + 256, ...
// (in that order): eight blocks' loads in flight, then added in order.
__device__ __forceinline__ void bn_part_sums(const float* __restrict__ part, int nb, int C, int c,
                                             double& a, double& b) {
    const int bd = blockDim.x;
    int k = threadIdx.x;
    for (; k + 7 * bd < nb; k += 8 * bd) {
        float va[8], vb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            va[u] = part[(size_t)(k + u * bd) * 2 * C + c];
            vb[u] = part[(size_t)(k + u * bd) * 2 * C + C + c];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a += va[u];
            b += vb[u];
        }
    }
    for (; k < nb; k += bd) {
        a += part[(size_t)k * 2 * C + c];
        b += part[(size_t)k * 2 * C + C + c];
    }
}

// Batch-norm statistics from the conv partials (double-precision sums in block order).
__global__ void k_bn_stats(const float* __restrict__ part, int nb, int C, long long M,
                           const float* __restrict__ gamma, const float* __restrict__ beta, float eps,
                           float momentum, int training, float* __restrict__ run_mean,
                           float* __restrict__ run_var, float* __restrict__ stat) {
    const int c = blockIdx.x;
    __shared__ double r1[256], r2[256];
    double a = 0.0, b = 0.0;
    bn_part_sums(part, nb, C, c, a, b);
    r1[threadIdx.x] = a;
    r2[threadIdx.x] = b;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double mean, var;
    if (training) {
        mean = r1[0] / (double)M;
        var = r2[0] / (double)M - mean * mean;
        if (var < 0.0) var = 0.0;
        const double unb = M > 1 ? var * (double)M / (double)(M - 1) : var;
        run_mean[c] = (float)((1.0 - momentum) * run_mean[c] + momentum * mean);
        run_var[c] = (float)((1.0 - momentum) * run_var[c] + momentum * unb);
    } else {
        mean = run_mean[c];
        var = run_var[c];
    }
    const double inv = 1.0 / sqrt(var + (double)eps);
    const double sc = (double)gamma[c] * inv;
    stat[c] = (float)mean;
    stat[C + c] = (float)inv;
    stat[2 * C + c] = (float)sc;
    stat[3 * C + c] = (float)((double)beta[c] - mean * sc);
}

// Eight consecutive floats from a 32-byte-aligned address as two vector loads.
__device__ __forceinline__ void load8(const float* __restrict__ p, float (&v)[8]) {
    const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}

__global__ void k_bn_relu(const bf16* __restrict__ z, const float* __restrict__ stat,
                          bf16* __restrict__ a, long long items, int C) {
    const long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= items) return;
    const int c0 = (int)(it % (C / 8)) * 8;
    const bf16x8 v = __builtin_bit_cast(bf16x8, *(const u32x4*)(z + it * 8));
    float sc[8], sh[8];
    load8(stat + 2 * C + c0, sc);
    load8(stat + 3 * C + c0, sh);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (bf16)fmaxf(fmaf((float)v[j], sc[j], sh[j]), 0.f);
    *(u32x4*)(a + it * 8) = __builtin_bit_cast(u32x4, o);
}

// BN + ReLU of an encoder's second convolution and the 2 x 2 max pooling of
// its result in one pass: one thread per (pooled pixel, 8-channel group)
// writes the four activations and their maximum (the max of the window's
// BF16 values taken in FP32, exact), with k_bn_relu's arithmetic.
__global__ void k_bn_relu_pool(const bf16* __restrict__ z, const float* __restrict__ stat, bf16* __restrict__ a,
                               bf16* __restrict__ pool, int images, int S, int C) {
    const int H = S / 2, G8 = C / 8;
    const long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= (long long)images * H * H * G8) return;
    const int cg = (int)(it % G8);
    const long long q = it / G8;
    const int X = (int)(q % H), Y = (int)((q / H) % H), img = (int)(q / ((long long)H * H));
    const size_t p00 = (((size_t)img * S + 2 * Y) * S + 2 * X) * C + 8 * cg;
    const size_t off[4] = {0, (size_t)C, (size_t)S * C, (size_t)S * C + C};
    float sc[8], sh[8];
    load8(stat + 2 * C + 8 * cg, sc);
    load8(stat + 3 * C + 8 * cg, sh);
    bf16x8 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = __builtin_bit_cast(bf16x8, *(const u32x4*)(z + p00 + off[k]));
    bf16x8 h[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int j = 0; j < 8; ++j) h[k][j] = (bf16)fmaxf(fmaf((float)v[k][j], sc[j], sh[j]), 0.f);
        *(u32x4*)(a + p00 + off[k]) = __builtin_bit_cast(u32x4, h[k]);
    }
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        o[j] = (bf16)fmaxf(fmaxf((float)h[0][j], (float)h[1][j]), fmaxf((float)h[2][j], (float)h[3][j]));
    *(u32x4*)(pool + q * C + 8 * cg) = __builtin_bit_cast(u32x4, o);
}

__global__ void k_up_concat(const bf16* __restrict__ d, const bf16* __restrict__ e, bf16* __restrict__ cat,
                            int images, int S, int Cd, int Ce) {
    const int C = Cd + Ce, G8 = C / 8, H = S / 2;
    const long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= (long long)images * S * S * G8) return;
    const int cg = (int)(it % G8);
    const long long p = it / G8;
    const int x = (int)(p % S), y = (int)((p / S) % S), img = (int)(p / ((long long)S * S));
    u32x4 outv;
    if (8 * cg < Cd) {
        int y0, y1, x0, x1;
        float wy, wx;
        up_taps(y, H, y0, y1, wy);
        up_taps(x, H, x0, x1, wx);
        const bf16* db = d + (size_t)img * H * H * Cd + 8 * cg;
        const bf16x8 a = __builtin_bit_cast(bf16x8, *(const u32x4*)(db + ((size_t)y0 * H + x0) * Cd));
        const bf16x8 b = __builtin_bit_cast(bf16x8, *(const u32x4*)(db + ((size_t)y0 * H + x1) * Cd));
        const bf16x8 c = __builtin_bit_cast(bf16x8, *(const u32x4*)(db + ((size_t)y1 * H + x0) * Cd));
        const bf16x8 dd = __builtin_bit_cast(bf16x8, *(const u32x4*)(db + ((size_t)y1 * H + x1) * Cd));
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float top = (1.f - wx) * (float)a[j] + wx * (float)b[j];
            const float bot = (1.f - wx) * (float)c[j] + wx * (float)dd[j];
            o[j] = (bf16)((1.f - wy) * top + wy * bot);
        }
        outv = __builtin_bit_cast(u32x4, o);
    } else {
        outv = *(const u32x4*)(e + p * Ce + (8 * cg - Cd));
    }
    *(u32x4*)(cat + p * C + 8 * cg) = outv;
}

// Output channel o of the head is plane o of mask (mask + o images S^2); w is [ch][C][3][3].
// A block computes a 16 x 64-pixel tile of every output channel from its
// 18 x 66-pixel input patch staged in LDS with zeros outside the image (all
// loads issued before the stores); a thread owns four pixels of one column.
// Each pixel sums its nine taps in tap order; a tap outside the image adds
// products of zero, which leave every nonzero sum unchanged and change at
// most the sign of a zero one (the sigmoid maps both zeros to 1/2), so the
// masks are those of a sum over the taps inside the image.  The weights sit
// in LDS as [o][tap][channel], read as 16-byte broadcasts.
constexpr int kHeadRows = 16, kHeadCols = 64;
template <int C>
__global__ __launch_bounds__(256) void k_head_fwd(const bf16* __restrict__ a, const float* __restrict__ w,
                                                  const float* __restrict__ b, float* __restrict__ mask,
                                                  int images, int S, int ch) {
    constexpr int PR = kHeadRows + 2, PC = kHeadCols + 2, G = C / 8, NE = PR * PC * G;
    constexpr int NL = (NE + 255) / 256;
    __shared__ u32x4 tile[NE];
    __shared__ f32x4 wl[2 * 9 * C / 4];   // up to two output channels
    const int tx = S / kHeadCols, ty = S / kHeadRows;
    const int img = blockIdx.x / (tx * ty), k = blockIdx.x % (tx * ty);
    const int y0 = (k / tx) * kHeadRows, x0 = (k % tx) * kHeadCols;
    u32x4 v[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int it = threadIdx.x + 256 * l;
        const int q = it / G, cg = it % G;
        const int y = y0 - 1 + q / PC, x = x0 - 1 + q % PC;
        v[l] = u32x4{0u, 0u, 0u, 0u};
        if (it < NE && y >= 0 && y < S && x >= 0 && x < S)
            v[l] = *(const u32x4*)(a + (((size_t)img * S + y) * S + x) * C + 8 * cg);
    }
    for (int i = threadIdx.x; i < ch * 9 * C; i += 256) {
        const int o = i / (9 * C), t = (i / C) % 9, ci = i % C;
        reinterpret_cast<float*>(wl)[i] = w[((size_t)o * C + ci) * 9 + t];
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int it = threadIdx.x + 256 * l;
        if (it < NE) tile[it] = v[l];
    }
    __syncthreads();
    const long long npix = (long long)images * S * S;
    const int c = threadIdx.x % kHeadCols, r0 = (threadIdx.x / kHeadCols) * 4;
    for (int o = 0; o < ch; ++o) {
        const float bo = b[o];
        float acc[4] = {bo, bo, bo, bo};
#pragma unroll 1
        for (int t = 0; t < 9; ++t) {   // one tap at a time (fewer operands live at once)
#pragma unroll
            for (int cg = 0; cg < G; ++cg) {
                const f32x4 w0 = wl[((o * 9 + t) * C + 8 * cg) / 4], w1 = wl[((o * 9 + t) * C + 8 * cg) / 4 + 1];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const bf16x8 e = __builtin_bit_cast(bf16x8, tile[((r0 + rr + t / 3) * PC + c + t % 3) * G + cg]);
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[rr] = fmaf((float)e[j], w0[j], acc[rr]);
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[rr] = fmaf((float)e[j + 4], w1[j], acc[rr]);
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
            mask[o * npix + ((size_t)img * S + y0 + r0 + rr) * S + x0 + c] = 1.f / (1.f + expf(-acc[rr]));
    }
}

// The head's logit gradient dl = d_mask m (1 - m) (the sigmoid's derivative),
// formed where it is read from the mask gradient and the saved mask.
__device__ __forceinline__ float head_dl(float dm, float m) {
#pragma clang fp contract(off)
    return dm * m * (1.f - m);
}

// g[p][ci] = sum_o sum_taps w[o][ci][tap] dl[o][p - (ky - 1, kx - 1)], one pixel
// (8 channels) per thread, output channels o in order.
__global__ void k_head_g(const float* __restrict__ dm, const float* __restrict__ m, const float* __restrict__ w,
                         float* __restrict__ g, int images, int S, int ch) {
    const long long npix = (long long)images * S * S;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const int x = (int)(p % S), y = (int)((p / S) % S), img = (int)(p / ((long long)S * S));
    float acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.f;
    for (int o = 0; o < ch; ++o) {
        const float* wo = w + (size_t)o * 8 * 9;
        const float* dmo = dm + o * npix;
        const float* mo = m + o * npix;
        // the loads first (clamped addresses), then the taps inside the image in order
        float dv[9], mv[9], d[9];
        unsigned inb = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const int yy = y - (k / 3 - 1), xx = x - (k % 3 - 1);
            inb |= (yy >= 0 && yy < S && xx >= 0 && xx < S ? 1u : 0u) << k;
            const int yc = min(max(yy, 0), S - 1), xc = min(max(xx, 0), S - 1);
            dv[k] = dmo[((size_t)img * S + yc) * S + xc];
            mv[k] = mo[((size_t)img * S + yc) * S + xc];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) d[k] = head_dl(dv[k], mv[k]);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            if (!((inb >> k) & 1u)) continue;
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] = fmaf(wo[j * 9 + k], d[k], acc[j]);
        }
    }
    float4* o = reinterpret_cast<float4*>(g + p * 8);
    o[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    o[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
}

constexpr int kHeadPix = 4096;   // pixels per head weight-gradient block

// part[block][ci 9 + tap] = sum dl[p] a[p + tap][ci]; part[block][9 C] = sum dl.
__global__ __launch_bounds__(256) void k_head_wgrad(const float* __restrict__ dm, const float* __restrict__ m,
                                                    const bf16* __restrict__ a, float* __restrict__ part,
                                                    int images, int S) {
    constexpr int C = 8, NW = 9 * C + 1;
    // output channel o = blockIdx.y: its mask and mask-gradient planes, and its
    // NW columns of a partial row that holds every output channel's (row = blockIdx.x)
    const int o = blockIdx.y;
    dm += (size_t)o * images * S * S;
    m += (size_t)o * images * S * S;
    part += (size_t)blockIdx.x * gridDim.y * NW + (size_t)o * NW;
    float acc[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[j] = 0.f;
    const long long n = (long long)images * S * S;
    const long long p0 = (long long)blockIdx.x * kHeadPix;
    const long long pend = min(n, p0 + kHeadPix);
    // One pixel's nine taps: every load issued at a clamped address, the taps
    // outside the image then skipped by selects (the same sums as branching).
    struct Taps {
        float dm, m;
        u32x4 v[9];
        unsigned inb;
    };
    auto load = [&](long long p) {
        Taps t;
        const int x = (int)(p % S), y = (int)((p / S) % S), img = (int)(p / ((long long)S * S));
        t.dm = dm[p];
        t.m = m[p];
        t.inb = 0;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int yy = y + ky - 1, xx = x + kx - 1;
                const bool in = yy >= 0 && yy < S && xx >= 0 && xx < S;
                const int yc = min(max(yy, 0), S - 1), xc = min(max(xx, 0), S - 1);
                t.v[ky * 3 + kx] = *(const u32x4*)(a + (((size_t)img * S + yc) * S + xc) * C);
                t.inb |= (in ? 1u : 0u) << (ky * 3 + kx);
            }
        return t;
    };
    auto add = [&](const Taps& t) {
        const float d = head_dl(t.dm, t.m);
        {
#pragma clang fp contract(off)
            acc[NW - 1] += d;   // d rounded, then added: not fused into its product
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const bf16x8 v = __builtin_bit_cast(bf16x8, t.v[k]);
            const bool in = (t.inb >> k) & 1u;
#pragma unroll
            for (int j = 0; j < C; ++j) {
                const float r = fmaf(d, (float)v[j], acc[j * 9 + k]);
                acc[j * 9 + k] = in ? r : acc[j * 9 + k];
            }
        }
    };
    long long p = p0 + threadIdx.x;
    // two pixels' loads in flight, accumulated in pixel order
    for (; p + kConvThreads < pend; p += 2 * kConvThreads) {
        const Taps t0 = load(p), t1 = load(p + kConvThreads);
        add(t0);
        add(t1);
    }
    if (p < pend) add(load(p));
    __shared__ float red[4][NW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        float v = acc[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < NW; j += kConvThreads)
        part[j] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
}

// Per-block channel sums for the batch-norm adjoint: part[block][0][c] = sum dy,
// part[block][1][c] = sum dy xhat over the block's bn_pixels(C) pixels (8192
// channel values per block whatever C, so deep layers with few pixels still
// spread over many blocks).  Thread (pixel lane, 8-channel group) with
// blockDim = (C/8) (256 / (C/8)); the pixel lanes are summed in order
// through LDS.
constexpr int kBnValues = 8192;
__host__ __device__ constexpr int bn_pixels(int C) { return kBnValues / C; }

__global__ __launch_bounds__(256) void k_bn_bwd_part(const float* __restrict__ g, const bf16* __restrict__ z,
                                                     const float* __restrict__ stat, float* __restrict__ part,
                                                     long long M, int C) {
    const int G8 = C / 8, PL = blockDim.x / G8, cg = threadIdx.x % G8, pl = threadIdx.x / G8;
    const long long p0 = (long long)blockIdx.x * bn_pixels(C);
    const long long p1 = min(M, p0 + bn_pixels(C));
    float sd[8], sx[8], mean[8], inv[8], sc[8], sh[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int c = 8 * cg + j;
        sd[j] = sx[j] = 0.f;
        mean[j] = stat[c];
        inv[j] = stat[C + c];
        sc[j] = stat[2 * C + c];
        sh[j] = stat[3 * C + c];
    }
    auto add = [&](const u32x4 zr, const float4 g0, const float4 g1) {
        const bf16x8 zv = __builtin_bit_cast(bf16x8, zr);
        const float gv[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float zz = (float)zv[j];
            const float dy = fmaf(zz, sc[j], sh[j]) > 0.f ? gv[j] : 0.f;
            sd[j] += dy;
            sx[j] = fmaf(dy, (zz - mean[j]) * inv[j], sx[j]);
        }
    };
    long long p = p0 + pl;
    // four pixels' loads in flight, then accumulated in pixel order
    for (; p + 3 * PL < p1; p += 4 * PL) {
        u32x4 zr[4];
        float4 ga[4], gb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const long long q = p + u * PL;
            zr[u] = *(const u32x4*)(z + q * C + 8 * cg);
            ga[u] = *(const float4*)(g + q * C + 8 * cg);
            gb[u] = *(const float4*)(g + q * C + 8 * cg + 4);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) add(zr[u], ga[u], gb[u]);
    }
    for (; p < p1; p += PL)
        add(*(const u32x4*)(z + p * C + 8 * cg), *(const float4*)(g + p * C + 8 * cg),
            *(const float4*)(g + p * C + 8 * cg + 4));
    __shared__ float red[2][256 * 8];   // [sum][pixel lane][channel]
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        red[0][pl * C + 8 * cg + j] = sd[j];
        red[1][pl * C + 8 * cg + j] = sx[j];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < 2 * C; c += blockDim.x) {
        const int k = c / C, cc = c % C;
        float s = 0.f;
        for (int q = 0; q < PL; ++q) s += red[k][q * C + cc];
        part[(size_t)blockIdx.x * 2 * C + c] = s;
    }
}

// dbeta, dgamma (double sums of the partials in block order) and the apply coefficients.
__global__ void k_bn_bwd_fin(const float* __restrict__ part, int nb, int C, long long M,
                             const float* __restrict__ gamma, const float* __restrict__ stat,
                             float* __restrict__ coef, float* __restrict__ dgamma, float* __restrict__ dbeta) {
    const int c = blockIdx.x;
    __shared__ double r1[256], r2[256];
    double a = 0.0, b = 0.0;
    bn_part_sums(part, nb, C, c, a, b);
    r1[threadIdx.x] = a;
    r2[threadIdx.x] = b;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    dbeta[c] = (float)r1[0];
    dgamma[c] = (float)r2[0];
    coef[c] = gamma[c] * stat[C + c];                 // gamma invstd
    coef[C + c] = (float)(r1[0] / (double)M);         // mean dy
    coef[2 * C + c] = (float)(r2[0] / (double)M);     // mean dy xhat
}

__global__ void k_bn_bwd_apply(const float* __restrict__ g, const bf16* __restrict__ z,
                               const float* __restrict__ stat, const float* __restrict__ coef,
                               bf16* __restrict__ dz, long long items, int C) {
    const long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= items) return;
    const int c0 = (int)(it % (C / 8)) * 8;
    const bf16x8 zv = __builtin_bit_cast(bf16x8, *(const u32x4*)(z + it * 8));
    // eight channels of g and of each statistic as vector loads (C and c0 are
    // multiples of 8), all issued before the arithmetic
    float gv[8], mean[8], inv[8], sc[8], sh[8], k0[8], k1[8], k2[8];
    load8(g + it * 8, gv);
    load8(stat + c0, mean);
    load8(stat + C + c0, inv);
    load8(stat + 2 * C + c0, sc);
    load8(stat + 3 * C + c0, sh);
    load8(coef + c0, k0);
    load8(coef + C + c0, k1);
    load8(coef + 2 * C + c0, k2);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float zz = (float)zv[j];
        const float dy = fmaf(zz, sc[j], sh[j]) > 0.f ? gv[j] : 0.f;
        const float xh = (zz - mean[j]) * inv[j];
        o[j] = (bf16)(k0[j] * (dy - k1[j] - xh * k2[j]));
    }
    *(u32x4*)(dz + it * 8) = __builtin_bit_cast(u32x4, o);
}

__global__ void k_pool_bwd(const float* __restrict__ d_pool, const bf16* __restrict__ e,
                           const float* __restrict__ skip, int skip_stride, int skip_off,
                           float* __restrict__ g, int images, int S, int C) {
    const int G8 = C / 8;
    const long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= (long long)images * S * S * G8) return;
    const int cg = (int)(it % G8);
    const long long p = it / G8;
    const int x = (int)(p % S), y = (int)((p / S) % S), img = (int)(p / ((long long)S * S));
    const int H = S / 2, Y = y / 2, X = x / 2;
    const bf16* b = e + (((size_t)img * S + 2 * Y) * S + 2 * X) * C + 8 * cg;
    const bf16x8 w0 = __builtin_bit_cast(bf16x8, *(const u32x4*)b);
    const bf16x8 w1 = __builtin_bit_cast(bf16x8, *(const u32x4*)(b + C));
    const bf16x8 w2 = __builtin_bit_cast(bf16x8, *(const u32x4*)(b + (size_t)S * C));
    const bf16x8 w3 = __builtin_bit_cast(bf16x8, *(const u32x4*)(b + (size_t)S * C + C));
    const int mine = (y - 2 * Y) * 2 + (x - 2 * X);
    // the pooled gradient and the skip gradient as vector loads, always issued
    // (skip offsets and strides are multiples of 8 channels), then selects
    const float4* dp = reinterpret_cast<const float4*>(d_pool + (((size_t)img * H + Y) * H + X) * C + 8 * cg);
    const float4 d0 = dp[0], d1 = dp[1];
    const float* sk = skip ? skip + p * skip_stride + skip_off + 8 * cg : d_pool;
    const float4 s0 = reinterpret_cast<const float4*>(sk)[0], s1 = reinterpret_cast<const float4*>(sk)[1];
    const float dv[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    const float sv[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
    float r[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float v[4] = {(float)w0[j], (float)w1[j], (float)w2[j], (float)w3[j]};
        int arg = 0;
#pragma unroll
        for (int k = 1; k < 4; ++k)
            if (v[k] > v[arg]) arg = k;
        r[j] = (skip ? sv[j] : 0.f) + (arg == mine ? dv[j] : 0.f);
    }
    float4* o = reinterpret_cast<float4*>(g + p * C + 8 * cg);
    o[0] = make_float4(r[0], r[1], r[2], r[3]);
    o[1] = make_float4(r[4], r[5], r[6], r[7]);
}

// Adjoint 1-D taps of up2 (bilinear x2, half-pixel centres): the outputs that
// read input q, in four fixed slots 2q - 1 .. 2q + 2, with their weights; a slot
// outside the output gets weight 0 and a clamped index.
__device__ __forceinline__ void up_taps(int q, int n, int* o, float* w) {
    o[0] = q >= 1 ? 2 * q - 1 : 0;
    w[0] = q >= 1 ? 0.25f : 0.f;
    o[1] = 2 * q;
    w[1] = q == 0 ? 1.f : 0.75f;
    o[2] = 2 * q + 1;
    w[2] = q == n - 1 ? 1.f : 0.75f;
    o[3] = q <= n - 2 ? 2 * q + 2 : 2 * q + 1;
    w[3] = q <= n - 2 ? 0.25f : 0.f;
}

// A block takes a TH x TW tile of low-resolution pixels (TW = min(32, H),
// TH = 256 / TW) and gpb of its 8-channel groups (from blockIdx.y gpb) one
// after another, all of them when the tiles alone fill the GPU: for each, the
// full-resolution rows 2 Y0 - 1 .. 2 (Y0 + TH) and columns likewise, clamped
// to the image, are staged in LDS first (each value read once from memory
// instead of by up to four taps), then each thread sums its pixel's sixteen
// taps as below.
__global__ __launch_bounds__(256) void k_up_bwd(const float* __restrict__ d_cat, float* __restrict__ d_d,
                                                int images, int S, int Cd, int Ce, int gpb) {
    const int H = S / 2, C = Cd + Ce;
    const int TW = H < 32 ? H : 32, TH = 256 / TW, RW = 2 * TW + 2, RH = 2 * TH + 2;
    const int tiles_x = H / TW, tiles_y = H / TH;
    const int img = blockIdx.x / (tiles_x * tiles_y), k = blockIdx.x % (tiles_x * tiles_y);
    const int Y0 = (k / tiles_x) * TH, X0 = (k % tiles_x) * TW;
    const int ry0 = 2 * Y0 - 1, rx0 = 2 * X0 - 1;
    extern __shared__ float4 stg[];   // [RH][RW][2]
    const int Y = Y0 + threadIdx.x / TW, X = X0 + threadIdx.x % TW;
    // the four output rows and columns that can read input (Y, X), in order;
    // the ones outside get weight 0 and a clamped index (adding 0 w leaves the same sums)
    int oy[4], ox[4];
    float wy[4], wx[4];
    up_taps(Y, H, oy, wy);
    up_taps(X, H, ox, wx);
    for (int cg = blockIdx.y * gpb; cg < (blockIdx.y + 1) * gpb; ++cg) {
    if (cg != blockIdx.y * gpb) __syncthreads();   // the previous group's taps have been read
    // every staged value's loads first, then the LDS stores
    constexpr int NL = 10;   // ceil(2 * 34 * 34 / 256) and ceil(2 * 18 * 66 / 256)
    float4 v[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int it = threadIdx.x + 256 * l;
        v[l] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (it < RH * RW * 2) {
            const int e = it >> 1, h = it & 1;
            const int y = min(max(ry0 + e / RW, 0), S - 1), x = min(max(rx0 + e % RW, 0), S - 1);
            v[l] = reinterpret_cast<const float4*>(d_cat + (((size_t)img * S + y) * S + x) * C + 8 * cg)[h];
        }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const int it = threadIdx.x + 256 * l;
        if (it < RH * RW * 2) stg[it] = v[l];
    }
    __syncthreads();
    float acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        float row[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) row[j] = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int e = (oy[a] - ry0) * RW + ox[b] - rx0;
            const float4 u0 = stg[2 * e], u1 = stg[2 * e + 1];
            const float vals[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) row[j] = fmaf(wx[b], vals[j], row[j]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = fmaf(wy[a], row[j], acc[j]);
    }
    float4* o = reinterpret_cast<float4*>(d_d + (((size_t)img * H + Y) * H + X) * Cd + 8 * cg);
    o[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    o[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
    }   // channel groups
}

__global__ void k_pack(const PackLayers t, const float* __restrict__ params, bf16* __restrict__ packed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= t.start[t.n]) return;
    int l = 0;
    while (i >= t.start[l + 1]) ++l;
    const int cin = t.cin[l], cout = t.cout[l], cink = t.cink[l];
    const int e = i - t.start[l];
    const int co = e / (9 * cink), k = e % (9 * cink), tap = k / cink, ci = k % cink;
    const float* w = params + t.w[l];
    packed[t.pf[l] + e] = ci < cin ? (bf16)w[((size_t)co * cin + ci) * 9 + tap] : (bf16)0.f;
    if (t.pb[l] >= 0 && ci < cin) {
        // data gradient: [cin][9 cout], tap flipped
        packed[t.pb[l] + (size_t)ci * 9 * cout + (8 - tap) * cout + co] = (bf16)w[((size_t)co * cin + ci) * 9 + tap];
    }
}


__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_pose_loss(int batch, const float* __restrict__ pose, const float* __restrict__ target,
                            int kind, float* __restrict__ loss, float* __restrict__ d_pose) {
    float acc = 0.f;
    const float inv_b = 1.f / (float)batch;
    for (int i = threadIdx.x; i < 3 * batch; i += blockDim.x) {
        const float d = pose[i] - target[i];
        if (kind == 1) {
            acc += fabsf(d);
            d_pose[i] = (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) * inv_b;
        } else {
            acc += d * d;
            d_pose[i] = 2.f * d * inv_b;
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (threadIdx.x == 0) loss[0] = acc * inv_b;
}

inline unsigned grid_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

// Stage 1 of the column sums; returns the number of chunks written to tmp.
int colsum1(int id, const float* part, int nb, long long stride, int n, float* tmp, hipStream_t s) {
    const int nbc = nb < kColChunks ? nb : kColChunks;
    const int per = (nb + nbc - 1) / nbc;
    const int used = (nb + per - 1) / per;
    FMBYM_LAUNCH(id, k_colsum1, dim3(grid_for(n, 64), used), dim3(256), s, part, nb, stride, n, per, tmp);
    return used;
}

}  // namespace

size_t colsum_tmp_floats(int n) { return (size_t)kColChunks * n; }

// ------------------------------------------------------------------ launchers

// (c_in, c_out) of the supported convolutions: the forward pairs of the 4- and
// 6-level networks (base 8) and their data gradients (c_out -> c_in).
#define FMBYM_CONV_PAIRS(X)                                                                      \
    X(8, 8) X(8, 16) X(16, 16) X(16, 32) X(32, 32) X(32, 64) X(64, 64) X(96, 32) X(48, 16) X(24, 8) \
    X(16, 8) X(32, 16) X(64, 32) X(32, 96) X(16, 48) X(8, 24)                                       \
    X(64, 128) X(128, 128) X(128, 256) X(256, 256) X(384, 128) X(192, 64)                           \
    X(128, 64) X(256, 128) X(128, 384) X(64, 192)

template <int CI, int COUT, int CO>
void launch_conv_co(int mode, dim3 grid, size_t lds, hipStream_t s, const bf16* in, const bf16* w, void* out,
                    float* part, int S, const BnInfer& bn, int tpb, int tiles) {
    const ConvSrc src{in, nullptr, nullptr, nullptr, 0, 0};
    if (mode == kConvTrain)
        FMBYM_LAUNCH_LDS(kMConvFwd, (k_conv3x3<CI, COUT, kConvTrain, CO>), grid, dim3(256), lds, s, src, w, out,
                         part, nullptr, S, bn, tpb, tiles);
    else if (mode == kConvInfer)
        FMBYM_LAUNCH_LDS(kMConvFwd, (k_conv3x3<CI, COUT, kConvInfer, CO>), grid, dim3(256), lds, s, src, w, out,
                         part, nullptr, S, bn, tpb, tiles);
    else
        FMBYM_LAUNCH_LDS(kMConvDgrad, (k_conv3x3<CI, COUT, kConvDgrad, CO>), grid, dim3(256), lds, s, src, w, out,
                         part, nullptr, S, bn, tpb, tiles);
}

bool launch_conv3x3(int cin, int cout, int mode, const bf16* in, const bf16* w, void* out, float* part,
                    const BnInfer& bn, int images, int S, hipStream_t s) {
    const int tiles = conv_blocks(images, S), tpb = conv_tpb(tiles), nb = conv_part_blocks(images, S);
    const int co = conv_chunk(cout, nb);
    const dim3 grid(nb, cout / co);
    const int elem = mode == kConvDgrad ? 4 : 2;
    const size_t lds = conv_lds_region(cin, kSrcPlain, co, elem) + w_stage_bytes(cin, co);
    if (lds + 4 * 2 * 96 * sizeof(float) > kLdsLimit) return false;
#define FMBYM_CONV_CASE(CI, CO)                                                                   \
    if (cin == CI && cout == CO) {                                                                \
        constexpr int C0 = co_chunk(CO);                                                          \
        if (co == C0)                                                                             \
            launch_conv_co<CI, CO, C0>(mode, grid, lds, s, in, w, out, part, S, bn, tpb, tiles);  \
        else if constexpr (C0 % 32 == 0) {                                                        \
            if (co == C0 / 2)                                                                     \
                launch_conv_co<CI, CO, C0 / 2>(mode, grid, lds, s, in, w, out, part, S, bn, tpb, tiles); \
            else if constexpr (C0 % 64 == 0) {                                                    \
                if (co == C0 / 4)                                                                 \
                    launch_conv_co<CI, CO, C0 / 4>(mode, grid, lds, s, in, w, out, part, S, bn, tpb, tiles); \
                else                                                                              \
                    return false;                                                                 \
            } else {                                                                              \
                return false;                                                                     \
            }                                                                                     \
        } else {                                                                                  \
            return false;                                                                         \
        }                                                                                         \
        return true;                                                                              \
    }
    FMBYM_CONV_PAIRS(FMBYM_CONV_CASE)
#undef FMBYM_CONV_CASE
    return false;
}

template <int CI, int COUT, int SRC, bool POOL, int CO>
void launch_infer_co(dim3 grid, size_t lds, hipStream_t s, const ConvSrc& src, const bf16* w, bf16* out, bf16* pool,
                     int S, const BnInfer& bn, int tpb, int tiles) {
    FMBYM_LAUNCH_LDS(kMConvFwd, (k_conv3x3<CI, COUT, kConvInfer, CO, SRC, POOL>), grid, dim3(256), lds, s, src, w,
                     (void*)out, (float*)nullptr, pool, S, bn, tpb, tiles);
}

// The output-channel chunk co of conv_chunk: co_chunk(COUT), or a half or a quarter of it.
template <int CI, int COUT, int SRC, bool POOL>
bool launch_infer_ci(int co, dim3 grid, size_t lds, hipStream_t s, const ConvSrc& src, const bf16* w, bf16* out,
                     bf16* pool, int S, const BnInfer& bn, int tpb, int tiles) {
    constexpr int C0 = co_chunk(COUT);
    if (co == C0) {
        launch_infer_co<CI, COUT, SRC, POOL, C0>(grid, lds, s, src, w, out, pool, S, bn, tpb, tiles);
        return true;
    }
    if constexpr (C0 % 32 == 0) {
        if (co == C0 / 2) {
            launch_infer_co<CI, COUT, SRC, POOL, C0 / 2>(grid, lds, s, src, w, out, pool, S, bn, tpb, tiles);
            return true;
        }
        if constexpr (C0 % 64 == 0) {
            if (co == C0 / 4) {
                launch_infer_co<CI, COUT, SRC, POOL, C0 / 4>(grid, lds, s, src, w, out, pool, S, bn, tpb, tiles);
                return true;
            }
        }
    }
    return false;
}

bool launch_conv_infer(int cin, int cout, int kind, const ConvSrc& src, const bf16* w, bf16* out, bf16* pool,
                       const BnInfer& bn, int images, int S, hipStream_t s) {
    if (kind == kSrcPlain && !pool) return launch_conv3x3(cin, cout, kConvInfer, src.in, w, out, nullptr, bn, images, S, s);
    const int tiles = conv_blocks(images, S), tpb = conv_tpb(tiles), nb = conv_part_blocks(images, S);
    const int co = conv_chunk(cout, nb);
    const dim3 grid(nb, cout / co);
    const size_t lds = conv_lds_region(cin, kind, co, 2) + w_stage_bytes(cin, co);
    if (lds > kLdsLimit) return false;
#define FMBYM_INFER_CASE(KIND, POOL, CI, CO)                                                                \
    if (kind == KIND && (pool != nullptr) == POOL && cin == CI && cout == CO)                               \
        return launch_infer_ci<CI, CO, KIND, POOL>(co, grid, lds, s, src, w, out, pool, S, bn, tpb, tiles);
    FMBYM_INFER_CASE(kSrcScan, false, 8, 8)
    FMBYM_INFER_CASE(kSrcUpCat, false, 24, 8)
    FMBYM_INFER_CASE(kSrcUpCat, false, 48, 16)
    FMBYM_INFER_CASE(kSrcUpCat, false, 96, 32)
    FMBYM_INFER_CASE(kSrcUpCat, false, 192, 64)
    FMBYM_INFER_CASE(kSrcUpCat, false, 384, 128)
    FMBYM_INFER_CASE(kSrcPlain, true, 8, 8)
    FMBYM_INFER_CASE(kSrcPlain, true, 16, 16)
    FMBYM_INFER_CASE(kSrcPlain, true, 32, 32)
    FMBYM_INFER_CASE(kSrcPlain, true, 64, 64)
    FMBYM_INFER_CASE(kSrcPlain, true, 128, 128)
#undef FMBYM_INFER_CASE
    return false;
}

void wgrad_grid(int images, int S, int* blocks, int* tiles_per_block) {
    const int tiles = conv_blocks(images, S);
    int tpb = tiles / 2048;
    tpb = tpb < 1 ? 1 : (tpb > 16 ? 16 : tpb);
    *tiles_per_block = tpb;
    *blocks = (tiles + tpb - 1) / tpb;
}

template <int CI, int COUT, int CO>
bool launch_wgrad_co(const bf16* dz, const bf16* in, float* part, int S, int nb, int tpb, int tiles, hipStream_t s) {
    using Geo = WgradGeo<CI, COUT, CO>;
    const size_t lds = (size_t)Geo::CO * kDztPitch * 2 + (size_t)Geo::CC * wg_plane(S) * 2 + Geo::red_bytes;
    if (lds > kLdsLimit) return false;
    // input-channel chunks over blocks until the launch has kConvMinBlocks (a divisor of NCH)
    int kz = 1;
    while (kz * 2 <= Geo::NCH && Geo::NCH % (kz * 2) == 0 && nb * (COUT / CO) * kz < kConvMinBlocks) kz *= 2;
    FMBYM_LAUNCH_LDS(kMWgrad, (k_wgrad<CI, COUT, CO>), dim3(nb, COUT / CO, kz), dim3(256), lds, s, dz, in, part, S,
                     tpb, tiles);
    return true;
}

bool launch_wgrad(int cin, int cout, const bf16* dz, const bf16* in, float* part, float* tmp, float* dw,
                  int real_cin, int images, int S, hipStream_t s) {
    int nb, tpb;
    wgrad_grid(images, S, &nb, &tpb);
    const int tiles = conv_blocks(images, S);
    const int n = cout * 9 * cin;
    const int co = conv_chunk(cout, nb);
#define FMBYM_WGRAD_CASE(CI, COUT_)                                                                  \
    if (cin == CI && cout == COUT_) {                                                                \
        constexpr int C0 = co_chunk(COUT_);                                                          \
        bool ok = false;                                                                             \
        if (co == C0)                                                                                \
            ok = launch_wgrad_co<CI, COUT_, C0>(dz, in, part, S, nb, tpb, tiles, s);                 \
        else if constexpr (C0 % 32 == 0) {                                                           \
            if (co == C0 / 2)                                                                        \
                ok = launch_wgrad_co<CI, COUT_, C0 / 2>(dz, in, part, S, nb, tpb, tiles, s);         \
            else if constexpr (C0 % 64 == 0) {                                                       \
                if (co == C0 / 4) ok = launch_wgrad_co<CI, COUT_, C0 / 4>(dz, in, part, S, nb, tpb, tiles, s); \
            }                                                                                        \
        }                                                                                            \
        if (!ok) return false;                                                                       \
        /* up to kColChunks partial rows: the second stage reads them directly (the first would copy \
           them: one row per chunk), with the same sums */                                           \
        const float* rows = part;                                                                    \
        int nbc = nb;                                                                                \
        if (nb > kColChunks) {                                                                       \
            nbc = colsum1(kMWgrad, part, nb, (long long)n, n, tmp, s);                               \
            rows = tmp;                                                                              \
        }                                                                                            \
        FMBYM_LAUNCH(kMWgrad, k_colsum2, dim3(grid_for(n, 256)), dim3(256), s, rows, nbc, n, 0, n, dw,  \
                     real_cin, cin);                                                                 \
        return true;                                                                                 \
    }
    FMBYM_CONV_PAIRS(FMBYM_WGRAD_CASE)
#undef FMBYM_WGRAD_CASE
    return false;
}

int bn_part_blocks(long long M, int C) { return (int)((M + bn_pixels(C) - 1) / bn_pixels(C)); }

void launch_input8(const float* x, const float* const* x_tab, bf16* x8, int images, int S, int ch,
                   hipStream_t s) {
    const long long n = (long long)images * S * S;
    FMBYM_LAUNCH(kMInput, k_input8, dim3(grid_for(n, 256)), dim3(256), s, x, x_tab, x8, n, S * S, ch);
}

void launch_input_grad(const bf16* dz, const float* w, float* dx, int images, int S, int C, int ch,
                       hipStream_t s) {
    const long long n = (long long)images * S * S;
    FMBYM_LAUNCH(kMInputGrad, k_input_grad, dim3(grid_for(n * ch, 256)), dim3(256), s, dz, w, dx, n, S, C, ch);
}

void launch_bn_stats(const float* part, int nb, int C, long long M, const float* gamma,
                     const float* beta, float eps, float momentum, int training, float* run_mean,
                     float* run_var, float* stat, float* tmp, hipStream_t s) {
    (void)tmp;
    FMBYM_LAUNCH(kMBnStats, k_bn_stats, dim3(C), dim3(256), s, part, nb, C, M, gamma, beta, eps, momentum,
                 training, run_mean, run_var, stat);
}

void launch_bn_relu(const bf16* z, const float* stat, bf16* a, long long M, int C, hipStream_t s) {
    const long long items = M * (C / 8);
    FMBYM_LAUNCH(kMBnRelu, k_bn_relu, dim3(grid_for(items, 256)), dim3(256), s, z, stat, a, items, C);
}

void launch_bn_relu_pool(const bf16* z, const float* stat, bf16* a, bf16* pool, int images, int S, int C,
                         hipStream_t s) {
    const long long items = (long long)images * (S / 2) * (S / 2) * (C / 8);
    FMBYM_LAUNCH(kMBnRelu, k_bn_relu_pool, dim3(grid_for(items, 256)), dim3(256), s, z, stat, a, pool, images, S, C);
}

void launch_up_concat(const bf16* d, const bf16* e, bf16* cat, int images, int S, int Cd, int Ce,
                      hipStream_t s) {
    const long long items = (long long)images * S * S * ((Cd + Ce) / 8);
    FMBYM_LAUNCH(kMUpCat, k_up_concat, dim3(grid_for(items, 256)), dim3(256), s, d, e, cat, images, S,
                       Cd, Ce);
}

bool launch_head_fwd(const bf16* a, const float* w, const float* b, float* mask, int images, int S,
                     int C, int ch, hipStream_t s) {
    const long long n = (long long)images * S * S;
    if (C != 8 || ch < 1 || ch > 2 || S % kHeadCols != 0 || S % kHeadRows != 0) return false;
    FMBYM_LAUNCH(kMHeadFwd, k_head_fwd<8>, dim3(n / (kHeadRows * kHeadCols)), dim3(256), s, a, w, b, mask, images, S,
                 ch);
    return true;
}

void launch_head_bwd(const float* d_mask, const float* mask, const bf16* a, const float* w, float* g,
                     float* part, float* tmp, float* dw, float* db, int images, int S, int C, int ch,
                     hipStream_t s) {
    const long long n = (long long)images * S * S;
    FMBYM_LAUNCH(kMHeadBwd, k_head_g, dim3(grid_for(n, 256)), dim3(256), s, d_mask, mask, w, g, images, S, ch);
    // every output channel in one launch (blockIdx.y), its partials in its own
    // columns of each block's row; the column sums as one array of ch NW columns
    const int nb = (int)((n + kHeadPix - 1) / kHeadPix), NW = 9 * C + 1;
    FMBYM_LAUNCH(kMHeadBwd, k_head_wgrad, dim3(nb, ch), dim3(256), s, d_mask, mask, a, part, images, S);
    const int nbc = colsum1(kMHeadBwd, part, nb, (long long)ch * NW, ch * NW, tmp, s);
    FMBYM_LAUNCH(kMHeadBwd, k_head_colsum2, dim3(1), dim3(256), s, tmp, nbc, ch * NW, dw, db);
}

void launch_bn_relu_bwd(const float* g, const bf16* z, const float* stat, const float* gamma, float* part,
                        float* tmp, float* coef, float* dgamma, float* dbeta, bf16* dz, long long M, int C,
                        hipStream_t s) {
    const int nb = bn_part_blocks(M, C);
    FMBYM_LAUNCH(kMBnBwd, k_bn_bwd_part, dim3(nb), dim3((C / 8) * (256 / (C / 8))), s, g, z, stat, part, M, C);
    (void)tmp;
    FMBYM_LAUNCH(kMBnBwd, k_bn_bwd_fin, dim3(C), dim3(256), s, part, nb, C, M, gamma, stat, coef, dgamma,
                       dbeta);
    const long long items = M * (C / 8);
    FMBYM_LAUNCH(kMBnBwd, k_bn_bwd_apply, dim3(grid_for(items, 256)), dim3(256), s, g, z, stat, coef, dz,
                       items, C);
}

void launch_pool_bwd(const float* d_pool, const bf16* e, const float* skip, int skip_stride,
                     int skip_off, float* g, int images, int S, int C, hipStream_t s) {
    const long long n = (long long)images * S * S * (C / 8);
    FMBYM_LAUNCH(kMPoolBwd, k_pool_bwd, dim3(grid_for(n, 256)), dim3(256), s, d_pool, e, skip, skip_stride,
                       skip_off, g, images, S, C);
}

void launch_up_bwd(const float* d_cat, float* d_d, int images, int S, int Cd, int Ce, hipStream_t s) {
    const int H = S / 2, TW = H < 32 ? H : 32, TH = 256 / TW;
    const int tiles = images * (H / TW) * (H / TH), gpb = tiles >= 1024 ? Cd / 8 : 1;
    const dim3 grid(tiles, Cd / 8 / gpb);
    const size_t lds = (size_t)(2 * TH + 2) * (2 * TW + 2) * 32;
    FMBYM_LAUNCH_LDS(kMUpBwd, k_up_bwd, grid, dim3(256), lds, s, d_cat, d_d, images, S, Cd, Ce, gpb);
}

void launch_pack(const PackLayers& t, const float* params, bf16* packed, hipStream_t s) {
    FMBYM_LAUNCH(kMPack, k_pack, dim3(grid_for(t.start[t.n], 256)), dim3(256), s, t, params, packed);
}


void launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1, float b2,
                 float eps, float c1, float c2, hipStream_t s) {
    FMBYM_LAUNCH(kMAdam, k_adam, dim3(grid_for(n, 256)), dim3(256), s, p, g, m, v, n, lr, b1, b2, eps, c1,
                       c2);
}

void launch_pose_loss(int batch, const float* pose, const float* target, int kind, float* loss,
                      float* d_pose, hipStream_t s) {
    FMBYM_LAUNCH(kMLoss, k_pose_loss, dim3(1), dim3(64), s, batch, pose, target, kind, loss, d_pose);
}

}  // namespace fmbym
