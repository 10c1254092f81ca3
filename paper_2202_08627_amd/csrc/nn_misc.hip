// Element-wise and reduction kernels of the warm-start network: input packing, 2x2 max
// pooling and its gradient (with the ReLU mask of its input), deterministic channel sums,
// split-K reduction, the 1x1 residual head, the MSE loss and Adam with FP32 master weights.
#include <algorithm>

#include "nn_internal.h"
#include "reduce.h"

namespace eit {
namespace nn {

__device__ __forceinline__ size_t at4(const Tensor& t, int b, int y, int x, int c) {
    return ((size_t)(b * t.H + y) * t.W + x) * t.cs + t.coff + c;
}

constexpr int kT = 256;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
inline int nblocks(size_t n) { return (int)std::min<size_t>((n + kT - 1) / kT, 65535 * 8); }

// FP32 [B][2][H][W] -> NHWC BF16 with 8 channels (channels 2..7 zero)
__global__ void k_pack(const float* x, int B, int H, int W, Tensor o) {
    const size_t n = (size_t)B * H * W;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int xx = p % W, yb = p / W, y = yb % H, b = yb / H;
        bf16* q = o.p + at4(o, b, y, xx, 0);
        bf16x8 v;
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = (bf16)0.f;
        v[0] = (bf16)x[((size_t)(b * 2 + 0) * H + y) * W + xx];
        v[1] = (bf16)x[((size_t)(b * 2 + 1) * H + y) * W + xx];
        *(bf16x8*)q = v;
        for (int c = 8; c < o.C; c += 8) *(bf16x8*)(q + c) = bf16x8{};
    }
}

__device__ __forceinline__ bf16x8 vld(const Tensor& t, int b, int y, int x, int c) {
    return *(const bf16x8*)(t.p + at4(t, b, y, x, c));
}
__device__ __forceinline__ void vst(const Tensor& t, int b, int y, int x, int c, bf16x8 v) {
    *(bf16x8*)(t.p + at4(t, b, y, x, c)) = v;
}

// 2x2 max pooling; thread = (output pixel, group of 8 channels), 16-byte accesses
__global__ void k_pool(Tensor x, Tensor y) {
    const int G = y.C / 8;
    const size_t n = (size_t)y.B * y.H * y.W * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int c = 8 * (int)(e % G);
        const size_t p = e / G;
        const int xx = p % y.W, yb = p / y.W, yy = yb % y.H, b = yb / y.H;
        const bf16x8 v0 = vld(x, b, 2 * yy, 2 * xx, c), v1 = vld(x, b, 2 * yy, 2 * xx + 1, c);
        const bf16x8 v2 = vld(x, b, 2 * yy + 1, 2 * xx, c), v3 = vld(x, b, 2 * yy + 1, 2 * xx + 1, c);
        bf16x8 m;
#pragma unroll
        for (int i = 0; i < 8; ++i)
            m[i] = (bf16)fmaxf(fmaxf(fmaxf((float)v0[i], (float)v1[i]), (float)v2[i]), (float)v3[i]);
        vst(y, b, yy, xx, c, m);
    }
}

// The gradient goes to the first input (row-major in the window) equal to the maximum; then
// every input of the window takes the ReLU derivative of x (the layer that produced x).
// Thread = (pooled pixel, group of 8 channels).
__global__ void k_pool_bwd(Tensor x, Tensor y, Tensor dy, Tensor dx) {
    const int G = y.C / 8;
    const size_t n = (size_t)y.B * y.H * y.W * G;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int c = 8 * (int)(e % G);
        const size_t p = e / G;
        const int xx = p % y.W, yb = p / y.W, yy = yb % y.H, b = yb / y.H;
        const bf16x8 m = vld(y, b, yy, xx, c), g = vld(dy, b, yy, xx, c);
        // every load of the window before the first store (the stores could alias them for
        // all the compiler knows, which would serialise four memory round trips)
        bf16x8 xv[4], d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int iy = 2 * yy + (q >> 1), ix = 2 * xx + (q & 1);
            xv[q] = vld(x, b, iy, ix, c);
            d[q] = vld(dx, b, iy, ix, c);
        }
        bool done[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) done[i] = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const bool arg = !done[i] && (float)xv[q][i] == (float)m[i];
                done[i] = done[i] || arg;
                if (!((float)xv[q][i] > 0.f)) d[q][i] = (bf16)0.f;
                else if (arg) d[q][i] = (bf16)((float)d[q][i] + (float)g[i]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) vst(dx, b, 2 * yy + (q >> 1), 2 * xx + (q & 1), c, d[q]);
    }
}

// out[c] = sum_k part[k][c] over per-block partials (the head backward's weight and bias sums),
// 32 columns per pass, eight row lanes each; the lanes' sums meet in LDS in a fixed order.
__global__ __launch_bounds__(kT) void k_chsum2(const float* part, int nblk, int C, float* out) {
    __shared__ float red[kT];
    const int cl = threadIdx.x & 31, rl = threadIdx.x >> 5;   // column lane, row lane (8)
    for (int c0 = blockIdx.x * 32; c0 < C; c0 += gridDim.x * 32) {
        const int c = c0 + cl;
        float v = 0.f;
        if (c < C)
            for (int k = rl; k < nblk; k += kT / 32) v += part[(size_t)k * C + c];
        red[threadIdx.x] = v;
        __syncthreads();
        if (rl == 0 && c < C) {
            float t = 0.f;
            for (int l = 0; l < kT / 32; ++l) t += red[l * 32 + cl];
            out[c] = t;
        }
        __syncthreads();
    }
}

// out[i] = sum_z part[z][i]. A block takes 32 consecutive i and its 8 wavefront halves split
// the slabs: half h sums z = h, h + 8, ... in order, then the 8 half sums are added in order
// of h (a fixed order: the result does not depend on scheduling). Every block reads 32
// consecutive floats (128 bytes) of each slab it visits.
constexpr int kSkCols = 32, kSkGroups = kT / kSkCols;
__global__ __launch_bounds__(kT) void k_splitk(const float* part, int splits, int n, size_t ld, float* out) {
    __shared__ float red[kSkGroups][kSkCols];
    const int col = threadIdx.x % kSkCols, grp = threadIdx.x / kSkCols;
    const int i = blockIdx.x * kSkCols + col;
    float s = 0.f;
    if (i < n) {
#pragma unroll 8
        for (int z = grp; z < splits; z += kSkGroups) s += part[(size_t)z * ld + i];
    }
    red[grp][col] = s;
    __syncthreads();
    if (grp == 0 && i < n) {
        float t = red[0][col];
#pragma unroll
        for (int h = 1; h < kSkGroups; ++h) t += red[h][col];
        out[i] = t;
    }
}

// out[b][o][y][x] = x_in[b][o][y][x] + b[o] + sum_c a[b,y,x,c] w[o][c]   (two outputs)
__global__ void k_head(Tensor a, const float* w, const float* bias, const float* x_in, float* out,
                       int B, int H, int W) {
    const size_t n = (size_t)B * H * W;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int xx = p % W, yb = p / W, y = yb % H, b = yb / H;
        const bf16* q = a.p + p * a.cs + a.coff;
        float s0 = bias[0], s1 = bias[1];
        for (int c0 = 0; c0 < a.C; c0 += 8) {          // 16-byte loads, channels in order
            const bf16x8 v8 = *(const bf16x8*)(q + c0);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float v = (float)v8[i];
                s0 = fmaf(v, w[c0 + i], s0);
                s1 = fmaf(v, w[a.C + c0 + i], s1);
            }
        }
        const size_t o0 = ((size_t)(b * 2 + 0) * H + y) * W + xx, o1 = ((size_t)(b * 2 + 1) * H + y) * W + xx;
        out[o0] = x_in[o0] + s0;
        out[o1] = x_in[o1] + s1;
    }
}

// MSE: part[k] = sum over the block's slice of (out - target)^2 (FP64); dout = 2 (out - t) / n
__global__ __launch_bounds__(kT) void k_mse1(const float* out, const float* t, size_t n, double* part,
                                             int nblk, float* dout) {
    __shared__ double red[kT / 64];
    const size_t i0 = n * blockIdx.x / nblk, i1 = n * (blockIdx.x + 1) / nblk;
    double s = 0.0;
    constexpr int U = 4;      // U elements' loads before their stores; the sum runs over i in order
    for (size_t iu = i0 + threadIdx.x; iu < i1; iu += (size_t)U * kT) {
        float r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = iu + (size_t)u * kT;
            r[u] = i < i1 ? out[i] - t[i] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = iu + (size_t)u * kT;
            if (i >= i1) break;
            s += (double)r[u] * r[u];
            if (dout) dout[i] = 2.f * r[u] / (float)n;
        }
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(kT) void k_mse2(const double* part, int nblk, size_t n, double* loss) {
    __shared__ double red[kT / 64];
    double s = 0.0;
    for (int k = threadIdx.x; k < nblk; k += kT) s += part[k];
    s = block_sum(s, red);                       // fixed order
    if (threadIdx.x == 0) *loss = s / (double)n;
}

// head backward: part[k][0..2C) = sum over the block's pixels of dout[o] * a[c] for o = 0, 1;
// part[k][2C..2C+2) = sum of dout[o]; da = (W^T dout) masked by a > 0 (a is post-ReLU).
// Thread (channel group g of 8 channels, pixel lane pl); sums meet in LDS in a fixed order.
__global__ __launch_bounds__(kT) void k_head_bwd1(Tensor a, const float* w, const float* dout,
                                                  int B, int H, int W, float* part, int nblk,
                                                  Tensor da) {
    __shared__ float red[kT * 18];
    const size_t P = (size_t)B * H * W;
    const size_t p0 = P * blockIdx.x / nblk, p1 = P * (blockIdx.x + 1) / nblk;
    const int C = a.C, G = C / 8;
    const int g = threadIdx.x % G, pl = threadIdx.x / G, NL = kT / G;
    float w0[8], w1[8], s0[8], s1[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        w0[i] = w[8 * g + i];
        w1[i] = w[C + 8 * g + i];
        s0[i] = 0.f;
        s1[i] = 0.f;
    }
    float b0 = 0.f, b1 = 0.f;
    // U pixels' loads are issued before their stores (which could alias them for all the
    // compiler knows); the sums still run over p in order
    constexpr int U = 4;
    for (size_t pu = p0 + pl; pu < p1; pu += (size_t)U * NL) {
        float g0[U], g1[U];
        bf16x8 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t p = pu + (size_t)u * NL;
            g0[u] = g1[u] = 0.f;
            if (p < p1) {
                const int xx = p % W, yb = p / W, y = yb % H, b = yb / H;
                g0[u] = dout[((size_t)(b * 2 + 0) * H + y) * W + xx];
                g1[u] = dout[((size_t)(b * 2 + 1) * H + y) * W + xx];
                v[u] = *(const bf16x8*)(a.p + p * a.cs + a.coff + 8 * g);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t p = pu + (size_t)u * NL;
            if (p >= p1) break;
            bf16x8 d;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float av = (float)v[u][i];
                s0[i] = fmaf(g0[u], av, s0[i]);
                s1[i] = fmaf(g1[u], av, s1[i]);
                d[i] = av > 0.f ? (bf16)fmaf(g0[u], w0[i], g1[u] * w1[i]) : (bf16)0.f;
            }
            *(bf16x8*)(da.p + p * da.cs + da.coff + 8 * g) = d;
            b0 += g0[u];
            b1 += g1[u];
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        red[threadIdx.x * 18 + i] = s0[i];
        red[threadIdx.x * 18 + 8 + i] = s1[i];
    }
    red[threadIdx.x * 18 + 16] = g == 0 ? b0 : 0.f;
    red[threadIdx.x * 18 + 17] = g == 0 ? b1 : 0.f;
    __syncthreads();
    const int E = 2 * C + 2;
    for (int e = threadIdx.x; e < E; e += kT) {
        float v = 0.f;
        if (e < 2 * C) {
            const int o = e / C, c = e % C;
            for (int l = 0; l < NL; ++l) v += red[(l * G + c / 8) * 18 + 8 * o + c % 8];
        } else {
            for (int l = 0; l < NL; ++l) v += red[(l * G) * 18 + 16 + (e - 2 * C)];
        }
        part[(size_t)blockIdx.x * E + e] = v;
    }
}

__global__ void k_tobf16(const float* s, bf16* d, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        d[i] = (bf16)s[i];
}

// Every layer's transposed BF16 weight copy in one launch: element e of the concatenated
// weight tensors belongs to the layer j with begin[j] <= e < begin[j + 1]; within it
// d[i][t][o] = s[o][t][i] for the layer's [O][T][I] weights.
__global__ void k_transpose_oti(OtiTable tab, const float* s, bf16* d) {
    const size_t n = tab.begin[tab.n];
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        int j = 0;
        while (e >= tab.begin[j + 1]) ++j;
        const size_t le = e - tab.begin[j];
        const int O = tab.O[j], T = tab.T[j], I = tab.I[j];
        const int i = le % I;
        const size_t r = le / I;
        const int t = r % T, o = r / T;
        d[tab.dst[j] + ((size_t)i * T + t) * O + o] = (bf16)s[tab.src[j] + le];
    }
}

__global__ void k_adam(float* p, float* m, float* v, const float* g, size_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// ---------------------------------------------------------------------------- launchers
hipError_t pack_input(const float* x, int B, int H, int W, const Tensor& o, hipStream_t s) {
    k_pack<<<nblocks((size_t)B * H * W), kT, 0, s>>>(x, B, H, W, o);
    return hipGetLastError();
}
hipError_t maxpool_fwd(const Tensor& x, const Tensor& y, hipStream_t s) {
    k_pool<<<nblocks((size_t)y.B * y.H * y.W * (y.C / 8)), kT, 0, s>>>(x, y);
    return hipGetLastError();
}
hipError_t maxpool_bwd_add(const Tensor& x, const Tensor& y, const Tensor& dy, const Tensor& dx,
                           hipStream_t s) {
    k_pool_bwd<<<nblocks((size_t)y.B * y.H * y.W * (y.C / 8)), kT, 0, s>>>(x, y, dy, dx);
    return hipGetLastError();
}
hipError_t splitk_reduce(const float* part, int splits, int n, float* out, hipStream_t s, size_t ld) {
    k_splitk<<<(n + kSkCols - 1) / kSkCols, kT, 0, s>>>(part, splits, n, ld ? ld : (size_t)n, out);
    return hipGetLastError();
}
// out[c] = sum_z sum_d part[z ld + d C + c] (d < D), z outer, in order (serial per output: for
// few slabs, e.g. the transposed convolution's bias from its slab-reduced per-sub-pixel sums).
__global__ __launch_bounds__(kT) void k_fold_sums(const float* part, int splits, size_t ld, int C, int D,
                                                  float* out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    float t = 0.f;
    for (int z = 0; z < splits; ++z)
        for (int d = 0; d < D; ++d) t += part[(size_t)z * ld + (size_t)d * C + c];
    out[c] = t;
}
hipError_t fold_sums(const float* part, int splits, size_t ld, int C, int D, float* out, hipStream_t s) {
    k_fold_sums<<<(C + kT - 1) / kT, kT, 0, s>>>(part, splits, ld, C, D, out);
    return hipGetLastError();
}
hipError_t head_fwd(const Tensor& a, const float* w, const float* b, const float* x_in, float* out,
                    int B, int H, int W, hipStream_t s) {
    k_head<<<nblocks((size_t)B * H * W), kT, 0, s>>>(a, w, b, x_in, out, B, H, W);
    return hipGetLastError();
}
hipError_t mse_loss(const float* out, const float* target, size_t n, double* part, int nblk,
                    double* loss, float* dout, hipStream_t s) {
    k_mse1<<<nblk, kT, 0, s>>>(out, target, n, part, nblk, dout);
    k_mse2<<<1, kT, 0, s>>>(part, nblk, n, loss);
    return hipGetLastError();
}
hipError_t head_bwd(const Tensor& a, const float* w, const float* dout, int B, int H, int W,
                    float* dw, float* db, float* part, int nblk, const Tensor& da, hipStream_t s) {
    // the head's bias gradient must directly follow its weight gradient (db == dw + 2C)
    if (db != dw + 2 * a.C) return hipErrorInvalidValue;
    const int E = 2 * a.C + 2;
    k_head_bwd1<<<nblk, kT, 0, s>>>(a, w, dout, B, H, W, part, nblk, da);
    k_chsum2<<<(E + 31) / 32, kT, 0, s>>>(part, nblk, E, dw);   // fixed-order reduction of [nblk][E]
    return hipGetLastError();
}
hipError_t to_bf16(const float* src, bf16* dst, size_t n, hipStream_t s) {
    k_tobf16<<<nblocks(n), kT, 0, s>>>(src, dst, n);
    return hipGetLastError();
}
hipError_t transpose_oti(const OtiTable& tab, const float* src, bf16* dst, hipStream_t s) {
    if (tab.n < 1 || tab.n > kOtiMax) return hipErrorInvalidValue;
    k_transpose_oti<<<nblocks(tab.begin[tab.n]), kT, 0, s>>>(tab, src, dst);
    return hipGetLastError();
}
hipError_t adam(float* p, float* m, float* v, const float* g, size_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t s) {
    k_adam<<<nblocks(n), kT, 0, s>>>(p, m, v, g, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace eit
