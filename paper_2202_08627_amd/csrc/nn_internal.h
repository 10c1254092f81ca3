// Internal declarations of the warm-start network kernels (nn_kernels.hip, nn_misc.hip) and
// their host orchestration (unet.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace eit {
namespace nn {

typedef __bf16 bf16;

// NHWC view: element (b, y, x, c) at p[((b*H + y)*W + x)*cs + coff + c]. C is the view's
// channel count (a power of two >= 8), cs the stride of the underlying buffer, coff the
// view's first channel (multiples of 8 keep 16-byte alignment).
struct Tensor {
    bf16* p;
    int B, H, W, C, cs, coff;
};

// GEMM-based layers (nn_kernels.hip)
hipError_t conv_fwd(const Tensor& x, const bf16* w, const float* bias, int relu, const Tensor& y,
                    int ksize, hipStream_t s);
// Data gradients; with relu_of (the post-ReLU activation at dx's positions) the stored
// gradient is zeroed where that activation is not positive.
hipError_t conv_dgrad(const Tensor& dz, const bf16* wt, const Tensor& dx, int ksize, hipStream_t s,
                      const Tensor* relu_of = nullptr);
// Weight gradients write part[z][co][tap][ci] for z < wgrad_splits_used(pixels, splits); the
// 3x3 conv's part[z] holds Co * 9 * Ci weight partials followed by Co bias partials
hipError_t conv_wgrad(const Tensor& x, const Tensor& dz, float* part, int splits, int ksize,
                      hipStream_t s);
hipError_t upconv_fwd(const Tensor& x, const bf16* w, const float* bias, const Tensor& y,
                      hipStream_t s);
hipError_t upconv_dgrad(const Tensor& g, const bf16* wt, const Tensor& dx, hipStream_t s,
                        const Tensor* relu_of = nullptr);
// Transposed-convolution weight gradients: part[z] holds the 4 Co Ci weight partials
// ([co][d][ci]) followed by 4 Co row sums sum_p G[(d, co)][p] (index d Co + co), whose sum over
// d is the bias gradient's partial
hipError_t upconv_wgrad(const Tensor& x, const Tensor& g, float* part, int splits, hipStream_t s);

// element-wise and reduction kernels (nn_misc.hip)
hipError_t pack_input(const float* x, int B, int H, int W, const Tensor& out, hipStream_t s);
hipError_t maxpool_fwd(const Tensor& x, const Tensor& y, hipStream_t s);
// dx += the pooled gradient dy routed to each window's maximum, then dx *= (x > 0) (x is the
// post-ReLU pooling input); the windows cover x (even sides)
hipError_t maxpool_bwd_add(const Tensor& x, const Tensor& y, const Tensor& dy, const Tensor& dx,
                           hipStream_t s);
// out[i] = sum_z part[z ld + i] for i < n (ld = 0: ld = n)
hipError_t splitk_reduce(const float* part, int splits, int n, float* out, hipStream_t s, size_t ld = 0);
// out[c] = sum_z sum_d part[z ld + d C + c], d < D
hipError_t fold_sums(const float* part, int splits, size_t ld, int C, int D, float* out, hipStream_t s);
hipError_t head_fwd(const Tensor& a, const float* w, const float* b, const float* x_in,
                    float* out, int B, int H, int W, hipStream_t s);
hipError_t mse_loss(const float* out, const float* target, size_t n, double* part, int nblk,
                    double* loss, float* dout, hipStream_t s);
hipError_t head_bwd(const Tensor& a, const float* w, const float* dout, int B, int H, int W,
                    float* dw, float* db, float* part, int nblk, const Tensor& da, hipStream_t s);
hipError_t to_bf16(const float* src, bf16* dst, size_t n, hipStream_t s);
// Weight transposes for the data gradients, all layers in one launch: layer j's weights
// src[src_j + (o T + t) I + i] (shape [O][T][I]) go to dst[dst_j + (i T + t) O + o] as BF16;
// begin[j] is the running element count (begin[0] = 0, begin[n] = the total).
constexpr int kOtiMax = 24;
struct OtiTable {
    int n;
    size_t begin[kOtiMax + 1], src[kOtiMax], dst[kOtiMax];
    int O[kOtiMax], T[kOtiMax], I[kOtiMax];
};
hipError_t transpose_oti(const OtiTable& tab, const float* src, bf16* dst, hipStream_t s);
hipError_t adam(float* p, float* m, float* v, const float* g, size_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t s);

constexpr int kSumBlocks = 256;   // partial-sum blocks of the deterministic reductions

// Pixel slab per split (a multiple of the 32-pixel step) and the number of slabs launched.
inline int wgrad_slab(int pixels, int splits) { return ((pixels + splits - 1) / splits + 31) / 32 * 32; }
inline int wgrad_splits_used(int pixels, int splits) {
    const int kps = wgrad_slab(pixels, splits);
    return (pixels + kps - 1) / kps;
}

// 3x3 weight gradients by 128-pixel halo tiles (k_wgrad3: 2 x 64 tiles, or 4 x 32 where the
// width is not a multiple of 64; 32 or 64 output channels per block) for input and output
// channel counts that are multiples of 32; the slabs are sized for about 512 blocks (at most
// one per tile: more blocks mean more partial sums to write and reduce, fewer leave CUs idle). wgrad3_parts is the number of partial slabs conv_wgrad then writes.
inline bool wgrad3_halo(int h, int w, int ci, int co) {
    return ci % 32 == 0 && co % 32 == 0 && w % 32 == 0 && (w % 64 == 0 ? h % 2 == 0 : h % 4 == 0);
}
inline int wgrad3_co(int co) { return co % 64 == 0 ? 64 : 32; }
inline int wgrad3_parts(int nb, int h, int w, int ci, int co) {
    const int T = nb * h * w / 128, bps = (co / wgrad3_co(co)) * (ci / 32);
    int sp = (512 + bps - 1) / bps;
    sp = sp < T ? sp : T;
    sp = sp > 1 ? sp : 1;
    const int tps = (T + sp - 1) / sp;
    return (T + tps - 1) / tps;
}
// Partial slabs written by conv_wgrad for an input of nb x h x w pixels, ci channels, and co
// output channels, given the split count of the general kernel.
inline int conv_wgrad_parts(int nb, int h, int w, int ci, int co, int splits) {
    return wgrad3_halo(h, w, ci, co) ? wgrad3_parts(nb, h, w, ci, co) : wgrad_splits_used(nb * h * w, splits);
}

}  // namespace nn
}  // namespace eit
