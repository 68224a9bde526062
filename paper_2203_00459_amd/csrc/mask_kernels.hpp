// Kernels of the mask network (a U-Net of 3x3 convolutions, Section III-E /
// Table II pattern): BF16 matrix-core convolutions with FP32 accumulation and
// the FP32 element-wise layers around them.  Tensors are NHWC: element
// (image, y, x, c) of a [I][S][S][C] tensor sits at ((image S + y) S + x) C + c.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fmbym {

typedef __bf16 bf16;

// Output pixels per convolution block (16 matrix-core rows per M-tile, 16 tiles).
constexpr int kConvTile = 256;

__host__ __device__ constexpr int pad16(int c) { return (c + 15) / 16 * 16; }

// Tiles (16 x 16 pixels) of one conv launch over `images` images of side S.
inline int conv_blocks(int images, int S) { return images * (S * S / kConvTile); }
// Tiles each block of a conv launch computes in sequence (the next tile's
// input in flight during the current one), and the blocks: one partial-sum
// record each for the batch-norm statistics.
inline int conv_tpb(int tiles) {
    const int t = tiles / 2048;
    return t < 1 ? 1 : (t > 16 ? 16 : t);
}
inline int conv_part_blocks(int images, int S) {
    const int tiles = conv_blocks(images, S), tpb = conv_tpb(tiles);
    return (tiles + tpb - 1) / tpb;
}

// Partial-sum blocks of the channel reductions (batch-norm statistics) over
// M pixels of C channels; see bn_part_blocks in the kernels.
int bn_part_blocks(long long M, int C);
// Blocks of a weight-gradient launch and the tiles each one covers.
void wgrad_grid(int images, int S, int* blocks, int* tiles_per_block);

// --- launchers (all asynchronous on s; shapes checked by the caller) -------

// x [ch][I][S][S] float (ch = 1 or 2 planes; for ch = 1 image i may instead
// come from x_tab[i]) -> [I][S][S][8] bf16 with plane c in channel c, zeros
// elsewhere.
void launch_input8(const float* x, const float* const* x_tab, bf16* x8, int images, int S, int ch,
                   hipStream_t s);
// Gradient of the network input x [ch][I][S][S] from the first convolution's
// output gradient dz [images][S][S][C] (BF16, NHWC) and its FP32 weights
// w [C][ch][3][3]: dx[ci][p] = sum_{c, tap} w[c][ci][tap] dz[p - tap + 1][c].
void launch_input_grad(const bf16* dz, const float* w, float* dx, int images, int S, int C, int ch,
                       hipStream_t s);

// Batch norm on the running statistics, for the inference-mode convolution.
struct BnInfer {
    const float* gamma;
    const float* beta;
    const float* run_mean;
    const float* run_var;
    float eps;
};
enum ConvMode { kConvDgrad = 0, kConvTrain = 1, kConvInfer = 2 };

// Input of a convolution.  Plain: in [I][S][S][cin] BF16.  The inference pass
// also reads two fused inputs:
//   kSrcUpCat: concat[up2(in), skip] formed while staging (the upsampling
//              layer's arithmetic), in [I][S/2][S/2][2 cin / 3] the deeper
//              activation and skip [I][S][S][cin / 3];
//   kSrcScan:  the FP32 scans as the 8-channel first input (plane c in channel
//              c, zeros elsewhere): x [ch][I][S][S] with plane stride `plane`
//              (I S^2), or for ch = 1 image i at x_tab[i].
enum ConvSrcKind { kSrcPlain = 0, kSrcUpCat = 1, kSrcScan = 2 };
struct ConvSrc {
    const bf16* in;
    const bf16* skip;
    const float* x;
    const float* const* x_tab;
    long long plane;
    int ch;
};

// 3x3 convolution for (cin, cout) in the supported set; w packed [cout][9 cin]
// bf16 (k = tap cin + ci, tap = 3 ky + kx).
//   kConvDgrad: out = conv (float);
//   kConvTrain: out = z = bf16(conv), and part[block][2][cout] receives the
//               block's sums of z and z^2 (of the stored bf16 values; one record
//               per block of conv_part_blocks);
//   kConvInfer: out = bf16(relu(bf16(conv) scale + shift)) with bn's scale
//               gamma / sqrt(run_var + eps) and shift beta - run_mean scale
//               (computed in double as the statistics pass does); no partials.
// Returns false for an unsupported pair.
bool launch_conv3x3(int cin, int cout, int mode, const bf16* in, const bf16* w, void* out, float* part,
                    const BnInfer& bn, int images, int S, hipStream_t s);
// Inference convolution (kConvInfer arithmetic) from the input `kind` of src;
// with pool non-null it also writes the 2 x 2 max pooling of its output,
// pool [I][S/2][S/2][cout] (the next level's input).  Returns false for an
// unsupported (cin, cout, kind, pool) combination.
bool launch_conv_infer(int cin, int cout, int kind, const ConvSrc& src, const bf16* w, bf16* out, bf16* pool,
                       const BnInfer& bn, int images, int S, hipStream_t s);

// Weight gradient: sum over pixels of dz[p][co] in[p + tap][ci], through
// per-block partials part (wgrad_grid) and a fixed-order reduction (tmp:
// colsum_tmp_floats(cout 9 cin)); cin is the staged (padded) channel count and
// the result lands in the parameter layout dw[co][ci][tap] for ci < real_cin.
// Returns false for an unsupported pair.
bool launch_wgrad(int cin, int cout, const bf16* dz, const bf16* in, float* part, float* tmp, float* dw,
                  int real_cin, int images, int S, hipStream_t s);

// Floats of the scratch `tmp` that the two-stage column sums of n columns need.
size_t colsum_tmp_floats(int n);

// Batch-norm statistics: reduce part[nb][2][C] (sums of z, z^2) over nb in a
// fixed order; training: mean/var of the batch (and running-statistics
// update), else the running ones.  Writes stat[4][C] = mean, invstd, scale, shift.
void launch_bn_stats(const float* part, int nb, int C, long long M, const float* gamma,
                     const float* beta, float eps, float momentum, int training,
                     float* run_mean, float* run_var, float* stat, float* tmp, hipStream_t s);

// a = relu(z scale + shift) per channel, bf16 -> bf16.
void launch_bn_relu(const bf16* z, const float* stat, bf16* a, long long M, int C, hipStream_t s);

// a = BN + ReLU of z (as launch_bn_relu) and pool = its 2 x 2 max pooling in
// one pass; z, a [I][S][S][C], pool [I][S/2][S/2][C].
void launch_bn_relu_pool(const bf16* z, const float* stat, bf16* a, bf16* pool, int images, int S, int C,
                         hipStream_t s);

// cat = [up2(d), e] with d [I][S/2][S/2][Cd], e [I][S][S][Ce] -> [I][S][S][Cd + Ce].
void launch_up_concat(const bf16* d, const bf16* e, bf16* cat, int images, int S, int Cd, int Ce,
                      hipStream_t s);

// Head: mask = sigmoid(conv3x3(a, w) + b), a [I][S][S][C] bf16, w [ch][C][3][3]
// float, b [ch]; mask [ch][I][S][S] (plane o is output channel o).  Returns
// false unless C = 8 (the base width).
bool launch_head_fwd(const bf16* a, const float* w, const float* b, float* mask, int images, int S,
                     int C, int ch, hipStream_t s);
// Head adjoint: with dl = d_mask m (1 - m) ([ch][I][S][S], formed where read),
// g [I][S][S][C] float = conv3x3^T(dl, w); dw [ch][C][3][3] and db [ch] (float,
// written) through per-block partials in part.
void launch_head_bwd(const float* d_mask, const float* mask, const bf16* a, const float* w, float* g,
                     float* part, float* tmp, float* dw, float* db, int images, int S, int C, int ch,
                     hipStream_t s);

// Batch-norm + ReLU adjoint given g = dL/da (float): dy = g [a > 0];
// dgamma = sum dy xhat, dbeta = sum dy (written to dgamma/dbeta);
// dz = gamma invstd / M (M dy - dbeta - xhat dgamma), bf16.
void launch_bn_relu_bwd(const float* g, const bf16* z, const float* stat, const float* gamma,
                        float* part, float* tmp, float* coef, float* dgamma, float* dbeta, bf16* dz,
                        long long M, int C, hipStream_t s);

// Max-pool adjoint plus the skip gradient: g[p][c] = skip[p][c] (channel
// offset skip_off of a row of skip_stride floats, or 0 if skip is null) +
// d_pool[q][c] where p is the first maximum (row-major) of its window in e.
void launch_pool_bwd(const float* d_pool, const bf16* e, const float* skip, int skip_stride,
                     int skip_off, float* g, int images, int S, int C, hipStream_t s);

// up2 adjoint: d_d [I][S/2][S/2][Cd] = up2^T of channels [0, Cd) of d_cat
// (rows of Cd + Ce floats).
void launch_up_bwd(const float* d_cat, float* d_d, int images, int S, int Cd, int Ce, hipStream_t s);

// Pack conv weights (OIHW float) to the forward layout [cout][9 cink] (ci >=
// cin zero) and, where pb >= 0, the data-gradient layout [cin][9 cout] with
// the taps flipped: every layer of a network in one launch.  Offsets count
// floats of params (w) and bf16 elements of the packed buffer (pf, pb).
constexpr int kMaxPackLayers = 24;
struct PackLayers {
    int n;
    int cin[kMaxPackLayers], cout[kMaxPackLayers], cink[kMaxPackLayers];
    int start[kMaxPackLayers + 1];   // first element of each layer's forward layout
    long long w[kMaxPackLayers], pf[kMaxPackLayers], pb[kMaxPackLayers];
};
void launch_pack(const PackLayers& t, const float* params, bf16* packed, hipStream_t s);

void launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s);
void launch_pose_loss(int batch, const float* pose, const float* target, int kind, float* loss,
                      float* d_pose, hipStream_t s);

}  // namespace fmbym
