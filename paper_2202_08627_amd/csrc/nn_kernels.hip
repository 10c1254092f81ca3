// BF16 MFMA kernels of the warm-start network (4-level 2-D U-Net). Activations are NHWC
// BF16 with an explicit channel stride and offset (so concatenations are views); weights
// are BF16 copies of FP32 master weights; every product accumulates in FP32.
//
// All convolutions are one implicit GEMM, D[m][n] = sum_k A[m][k] B[n][k], with both operands
// staged in LDS as rows of k (8 consecutive k per 16-byte group) and multiplied with
// v_mfma_f32_16x16x32_bf16. A lane of that instruction supplies 8 consecutive k of one A row
// (row = lane % 16, group = lane / 16) and of one B row, and receives 4 rows of one D column.
// The loaders gather A/B groups straight from the activation tensors (im2col on the fly).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nn_internal.h"

namespace eit {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}
__device__ __forceinline__ bf16x8 ld8(const bf16* p) { return *(const bf16x8*)p; }

// --------------------------------------------------------------------------- loaders
// Each returns the 8 consecutive k (k0 .. k0+7, k0 % 8 == 0) of row r, zeros outside.

// 3x3 convolution input patches, k = tap * C + c (C % 8 == 0, power of two). flip = 1 gives
// the data-gradient form (input pixel p - (tap - 4) instead of p + (tap - 4)).
struct LoadConvA {
    const bf16* t; int B, H, W, C, cs, coff, cshift, K, flip, ksize;
    __device__ bf16x8 operator()(int m, int k0, int M) const {
        if (m >= M || k0 >= K) return zero8();
        const int tap = k0 >> cshift, c = k0 & (C - 1);
        const int x = m % W, yb = m / W, y = yb % H, b = yb / H;
        int dy, dx;
        if (ksize == 3) { dy = tap / 3 - 1; dx = tap % 3 - 1; } else { dy = 0; dx = 0; }
        if (flip) { dy = -dy; dx = -dx; }
        const int yy = y + dy, xx = x + dx;
        if ((unsigned)yy >= (unsigned)H || (unsigned)xx >= (unsigned)W) return zero8();
        return ld8(t + ((size_t)(b * H + yy) * W + xx) * cs + coff + c);
    }
};

// Dense row-major matrix [rows][K] (K contiguous, K % 8 == 0).
struct LoadRows {
    const bf16* t; int rows, K, ld;
    __device__ bf16x8 operator()(int r, int k0, int) const {
        if (r >= rows || k0 >= K) return zero8();
        return ld8(t + (size_t)r * ld + k0);
    }
};

// Transposed-convolution (2x2, stride 2) output gradient seen from an input pixel:
// row m = input pixel (b, y, x), k = d * C + c, value = g[b, 2y + d/2, 2x + d%2, c].
struct LoadUpGradA {
    const bf16* t; int B, H, W, C, cs, coff, cshift, K;   // H, W of the input (half size)
    __device__ bf16x8 operator()(int m, int k0, int M) const {
        if (m >= M || k0 >= K) return zero8();
        const int d = k0 >> cshift, c = k0 & (C - 1);
        const int x = m % W, yb = m / W, y = yb % H, b = yb / H;
        const int yy = 2 * y + (d >> 1), xx = 2 * x + (d & 1);
        return ld8(t + ((size_t)(b * 2 * H + yy) * (2 * W) + xx) * cs + coff + c);
    }
};

// Weight-gradient operands: the reduction index k runs over pixels, so a group gathers 8
// pixels of one channel (strided loads).
// Conv input channel c at pixel p shifted by a tap: row r = tap * C + c.
struct LoadWgInput {
    const bf16* t; int B, H, W, C, cs, coff, cshift, P, ksize;
    __device__ bf16x8 operator()(int r, int p0, int R) const {
        bf16x8 v = zero8();
        if (r >= R) return v;
        const int tap = r >> cshift, c = r & (C - 1);
        int dy = 0, dx = 0;
        if (ksize == 3) { dy = tap / 3 - 1; dx = tap % 3 - 1; }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int p = p0 + i;
            if (p >= P) break;
            const int x = p % W, yb = p / W, y = yb % H, b = yb / H;
            const int yy = y + dy, xx = x + dx;
            if ((unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W)
                v[i] = t[((size_t)(b * H + yy) * W + xx) * cs + coff + c];
        }
        return v;
    }
};
// Channel c of an NHWC tensor at 8 consecutive pixels (row r = c).
struct LoadWgChannel {
    const bf16* t; int C, cs, coff, P;
    __device__ bf16x8 operator()(int r, int p0, int R) const {
        bf16x8 v = zero8();
        if (r >= R) return v;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int p = p0 + i;
            if (p < P) v[i] = t[(size_t)p * cs + coff + r];
        }
        return v;
    }
};
// Transposed-conv output gradient for its weight gradient: row r = 4 * c + d, pixel p of
// the (half-size) input, value g[b, 2y + d/2, 2x + d%2, c].
struct LoadWgUpGrad {
    const bf16* t; int B, H, W, C, cs, coff, P;
    __device__ bf16x8 operator()(int r, int p0, int R) const {
        bf16x8 v = zero8();
        if (r >= R) return v;
        const int d = r & 3, c = r >> 2;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int p = p0 + i;
            if (p >= P) break;
            const int x = p % W, yb = p / W, y = yb % H, b = yb / H;
            v[i] = t[((size_t)(b * 2 * H + 2 * y + (d >> 1)) * (2 * W) + 2 * x + (d & 1)) * cs + coff + c];
        }
        return v;
    }
};

// --------------------------------------------------------------------------- epilogues
// NHWC store with optional bias and ReLU.
struct EpiAct {
    bf16* t; const float* bias; int cs, coff, relu, N;
    __device__ void operator()(int m, int n, float v, int) const {
        if (n >= N) return;
        if (bias) v += bias[n];
        if (relu) v = fmaxf(v, 0.f);
        t[(size_t)m * cs + coff + n] = (__bf16)v;
    }
};
// Transposed conv forward: n = 4 * c + d -> output pixel (2y + d/2, 2x + d%2), channel c.
struct EpiUp {
    bf16* t; const float* bias; int B, H, W, C, cs, coff, N;
    __device__ void operator()(int m, int n, float v, int) const {
        if (n >= N) return;
        const int d = n & 3, c = n >> 2;
        const int x = m % W, yb = m / W, y = yb % H, b = yb / H;
        v += bias[c];
        t[((size_t)(b * 2 * H + 2 * y + (d >> 1)) * (2 * W) + 2 * x + (d & 1)) * cs + coff + c] = (__bf16)v;
    }
};
// FP32 split-K partials [split][M][N].
struct EpiPart {
    float* t; int M, N;
    __device__ void operator()(int m, int n, float v, int z) const {
        if (n >= N) return;
        t[((size_t)z * M + m) * N + n] = v;
    }
};

// --------------------------------------------------------------------------- GEMM
// Block tile BM x BN with 4 wavefronts in a WM x WN grid; k advances 32 per step. Grid
// (ceil(M/BM), ceil(N/BN), splits); split z covers k in [z*kps, min(K, (z+1)*kps)).
template <int BM, int BN, int WM, int WN, class LA, class LB, class EP>
__global__ __launch_bounds__(256) void k_gemm(LA la, LB lb, EP ep, int M, int N, int K, int kps) {
    constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
    static_assert(WM * WN == 4 && TM >= 1 && TN >= 1, "tile shape");
    constexpr int GP = 5;                      // groups per LDS row: 4 + 1 pad (bank spread)
    __shared__ bf16x8 As[BM * GP], Bs[BN * GP];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv / WN, wn = wv % WN;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kb = blockIdx.z * kps, ke = min(K, kb + kps);
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += 32) {
        for (int e = tid; e < BM * 4; e += 256) {
            const int r = e >> 2, g = e & 3;
            const int k = k0 + 8 * g;
            As[r * GP + g] = k < ke ? la(m0 + r, k, M) : zero8();
        }
        for (int e = tid; e < BN * 4; e += 256) {
            const int r = e >> 2, g = e & 3;
            const int k = k0 + 8 * g;
            Bs[r * GP + g] = k < ke ? lb(n0 + r, k, N) : zero8();
        }
        __syncthreads();
        bf16x8 a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[(wm * TM * 16 + i * 16 + (lane & 15)) * GP + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[(wn * TN * 16 + j * 16 + (lane & 15)) * GP + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * TM * 16 + i * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wn * TN * 16 + j * 16 + (lane & 15);
                if (m < M) ep(m, n, acc[i][j][r], blockIdx.z);
            }
}

template <class LA, class LB, class EP>
hipError_t gemm(LA la, LB lb, EP ep, int M, int N, int K, int splits, hipStream_t s) {
    const int kps = ((K + splits - 1) / splits + 31) / 32 * 32;
    const int sp = (K + kps - 1) / kps;
    if (N <= 16) {
        dim3 g((M + 255) / 256, (N + 15) / 16, sp);
        k_gemm<256, 16, 4, 1><<<g, 256, 0, s>>>(la, lb, ep, M, N, K, kps);
    } else if (N <= 32) {
        dim3 g((M + 127) / 128, (N + 31) / 32, sp);
        k_gemm<128, 32, 4, 1><<<g, 256, 0, s>>>(la, lb, ep, M, N, K, kps);
    } else {
        dim3 g((M + 127) / 128, (N + 63) / 64, sp);
        k_gemm<128, 64, 2, 2><<<g, 256, 0, s>>>(la, lb, ep, M, N, K, kps);
    }
    return hipGetLastError();
}

int ilog2(int v) {
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

// --------------------------------------------------------------------------- layer ops
hipError_t conv_fwd(const Tensor& x, const bf16* w, const float* bias, int relu, const Tensor& y,
                    int ksize, hipStream_t s) {
    const int taps = ksize * ksize;
    LoadConvA la{x.p, x.B, x.H, x.W, x.C, x.cs, x.coff, ilog2(x.C), taps * x.C, 0, ksize};
    LoadRows lb{w, y.C, taps * x.C, taps * x.C};
    EpiAct ep{y.p, bias, y.cs, y.coff, relu, y.C};
    return gemm(la, lb, ep, x.B * x.H * x.W, y.C, taps * x.C, 1, s);
}

// dx[p][ci] = sum_{tap, co} dz[p - off(tap)][co] wt[ci][tap][co]
hipError_t conv_dgrad(const Tensor& dz, const bf16* wt, const Tensor& dx, int ksize, hipStream_t s) {
    const int taps = ksize * ksize;
    LoadConvA la{dz.p, dz.B, dz.H, dz.W, dz.C, dz.cs, dz.coff, ilog2(dz.C), taps * dz.C, 1, ksize};
    LoadRows lb{wt, dx.C, taps * dz.C, taps * dz.C};
    EpiAct ep{dx.p, nullptr, dx.cs, dx.coff, 0, dx.C};
    return gemm(la, lb, ep, dz.B * dz.H * dz.W, dx.C, taps * dz.C, 1, s);
}

// partial dW[z][co][tap * C + ci] over pixel slabs
hipError_t conv_wgrad(const Tensor& x, const Tensor& dz, float* part, int splits, int ksize,
                      hipStream_t s) {
    const int taps = ksize * ksize;
    const int P = x.B * x.H * x.W;
    LoadWgChannel la{dz.p, dz.C, dz.cs, dz.coff, P};
    LoadWgInput lb{x.p, x.B, x.H, x.W, x.C, x.cs, x.coff, ilog2(x.C), P, ksize};
    EpiPart ep{part, dz.C, taps * x.C};
    return gemm(la, lb, ep, dz.C, taps * x.C, P, splits, s);
}

// y[b, 2y+d/2, 2x+d%2, co] = sum_ci x[b,y,x,ci] w[co][d][ci] + bias[co]
hipError_t upconv_fwd(const Tensor& x, const bf16* w, const float* bias, const Tensor& y,
                      hipStream_t s) {
    LoadRows la{x.p + x.coff, x.B * x.H * x.W, x.C, x.cs};
    LoadRows lb{w, 4 * y.C, x.C, x.C};
    EpiUp ep{y.p, bias, x.B, x.H, x.W, y.C, y.cs, y.coff, 4 * y.C};
    return gemm(la, lb, ep, x.B * x.H * x.W, 4 * y.C, x.C, 1, s);
}

// dx[b,y,x,ci] = sum_{d,co} g[b,2y+d/2,2x+d%2,co] wt[ci][d][co]
hipError_t upconv_dgrad(const Tensor& g, const bf16* wt, const Tensor& dx, hipStream_t s) {
    LoadUpGradA la{g.p, dx.B, dx.H, dx.W, g.C, g.cs, g.coff, ilog2(g.C), 4 * g.C};
    LoadRows lb{wt, dx.C, 4 * g.C, 4 * g.C};
    EpiAct ep{dx.p, nullptr, dx.cs, dx.coff, 0, dx.C};
    return gemm(la, lb, ep, dx.B * dx.H * dx.W, dx.C, 4 * g.C, 1, s);
}

// partial dW[z][co][d][ci]
hipError_t upconv_wgrad(const Tensor& x, const Tensor& g, float* part, int splits, hipStream_t s) {
    const int P = x.B * x.H * x.W;
    LoadWgUpGrad la{g.p, x.B, x.H, x.W, g.C, g.cs, g.coff, P};
    LoadWgChannel lb{x.p, x.C, x.cs, x.coff, P};
    EpiPart ep{part, 4 * g.C, x.C};
    return gemm(la, lb, ep, 4 * g.C, x.C, P, splits, s);
}

}  // namespace nn
}  // namespace eit
