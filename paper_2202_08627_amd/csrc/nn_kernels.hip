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

// Buffer loads of 16 bytes: a load at a byte offset >= the resource's extent returns zeros
// without touching memory. The GEMM loaders turn every out-of-range or padding access into
// such an offset instead of a branch, so a step's loads are straight-line code (the
// compiler then tracks each register set's loads separately and can keep several steps'
// loads in flight). Extents stay below 2^31 bytes (tensor sizes are checked on the host).
constexpr int kOOB = 0x7ffffff0;
__device__ __forceinline__ bf16x8 bld8(const bf16* base, int bytes, int off) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, bytes, 0x00020000);
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

// --------------------------------------------------------------------------- loaders
// A loader is used in two stages: row(m, M) decodes row m once per output tile (pixel
// coordinates and validity), load(ctx, k0, ok) returns the 8 consecutive k (k0 .. k0+7,
// k0 % 8 == 0) of that row, zeros outside or when !ok.
struct PixRow { int b, y, x; bool ok; };

// 3x3 convolution input patches, k = tap * C + c (C % 8 == 0, power of two). flip = 1 gives
// the data-gradient form (input pixel p - (tap - 4) instead of p + (tap - 4)).
struct LoadConvA {
    const bf16* t; int B, H, W, C, cs, coff, cshift, K, flip, ksize, bytes;
    typedef PixRow Ctx;
    __device__ Ctx row(int m, int M) const {
        Ctx c;
        c.ok = m < M;
        const int mm = c.ok ? m : 0;
        const int yb = mm / W;
        c.x = mm - yb * W;
        c.b = yb / H;
        c.y = yb - c.b * H;
        return c;
    }
    __device__ bf16x8 load(const Ctx& r, int k0, bool ok) const {
        const int tap = k0 >> cshift, c = k0 & (C - 1);
        int dy = ksize == 3 ? tap / 3 - 1 : 0, dx = ksize == 3 ? tap - 3 * (tap / 3) - 1 : 0;
        if (flip) { dy = -dy; dx = -dx; }
        const int yy = r.y + dy, xx = r.x + dx;
        ok = ok && r.ok && k0 < K && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
        return bld8(t, bytes, ok ? 2 * (((r.b * H + yy) * W + xx) * cs + coff + c) : kOOB);
    }
};

// Dense row-major matrix [rows][K] (K contiguous, K % 8 == 0).
struct LoadRows {
    const bf16* t; int rows, K, ld, bytes;
    struct Ctx { int off; bool ok; };
    __device__ Ctx row(int r, int) const { return Ctx{r < rows ? 2 * r * ld : 0, r < rows}; }
    __device__ bf16x8 load(const Ctx& r, int k0, bool ok) const {
        return bld8(t, bytes, ok && r.ok && k0 < K ? r.off + 2 * k0 : kOOB);
    }
};

// Transposed-convolution (2x2, stride 2) output gradient seen from an input pixel:
// row m = input pixel (b, y, x), k = d * C + c, value = g[b, 2y + d/2, 2x + d%2, c].
struct LoadUpGradA {
    const bf16* t; int B, H, W, C, cs, coff, cshift, K, bytes;   // H, W of the input (half size)
    typedef PixRow Ctx;
    __device__ Ctx row(int m, int M) const {
        Ctx c;
        c.ok = m < M;
        const int mm = c.ok ? m : 0;
        const int yb = mm / W;
        c.x = mm - yb * W;
        c.b = yb / H;
        c.y = yb - c.b * H;
        return c;
    }
    __device__ bf16x8 load(const Ctx& r, int k0, bool ok) const {
        const int d = k0 >> cshift, c = k0 & (C - 1);
        const int yy = 2 * r.y + (d >> 1), xx = 2 * r.x + (d & 1);
        ok = ok && r.ok && k0 < K;
        return bld8(t, bytes, ok ? 2 * (((r.b * 2 * H + yy) * (2 * W) + xx) * cs + coff + c) : kOOB);
    }
};

// --------------------------------------------------------------------------- epilogues
// NHWC store with optional bias and ReLU; with `mask` (an NHWC view of a post-ReLU activation
// of the output's shape) the value is zeroed where the activation is not positive: the
// ReLU derivative of the layer that produced that activation, applied to its gradient.
// The GEMM stores it in two stages (kVector): pre() adds the bias and applies the ReLU to one
// value, the block stages the rounded tile in LDS, and store8() applies the mask to 8
// consecutive channels and writes them with one 16-byte store (N, cs, coff, mcs and mcoff
// are multiples of 8).
struct EpiAct {
    static constexpr bool kVector = true;
    bf16* t; const float* bias; int cs, coff, relu, N;
    const bf16* mask; int mcs, mcoff;
    __device__ float pre(int n, float v) const {
        if (bias && n < N) v += bias[n];
        if (relu) v = fmaxf(v, 0.f);
        return v;
    }
    __device__ void store8(int m, int n, bf16x8 v) const {
        if (mask) {
            const bf16x8 mk = *(const bf16x8*)(mask + (size_t)m * mcs + mcoff + n);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (!((float)mk[i] > 0.f)) v[i] = (__bf16)0.f;
        }
        *(bf16x8*)(t + (size_t)m * cs + coff + n) = v;
    }
};
// Transposed conv forward: n = 4 * c + d -> output pixel (2y + d/2, 2x + d%2), channel c.
struct EpiUp {
    static constexpr bool kVector = false;
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
    static constexpr bool kVector = false;
    float* t; int M, N;
    __device__ void operator()(int m, int n, float v, int z) const {
        if (n >= N) return;
        t[((size_t)z * M + m) * N + n] = v;
    }
};

// --------------------------------------------------------------------------- tile order
// The dispatcher hands workgroup L (linear id, x fastest) to XCD L % kXcds, and every XCD has
// an L2 of its own. tile_order(L, total) renumbers the workgroups so that XCD j takes the
// contiguous range of tile numbers [start_j, start_j + count_j) (a bijection on [0, total)):
// tiles that read the same activation rows then share one L2 instead of fetching them once
// per XCD.
constexpr int kXcds = 8;
__device__ __forceinline__ int tile_order(int L, int total) {
    const int xcd = L % kXcds, local = L / kXcds, q = total / kXcds, r = total % kXcds;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// --------------------------------------------------------------------------- GEMM
// Block tile BM x BN with 4 wavefronts in a WM x WN grid; k advances 32 per step. Grid
// (ceil(M/BM), ceil(N/BN), splits); split z covers k in [z*kps, min(K, (z+1)*kps)). Each
// thread stages fixed (row, 8-k group) slots of the tiles: rows are decoded once per tile,
// and the next step's groups are loaded into registers while the current step multiplies.
// (Two or three steps of loads in flight measured slower: the extra registers cost more
// resident blocks than the deeper prefetch hides. For the same reason the kernel is held to
// the registers of six wavefronts per SIMD.)
template <int BM, int BN, int WM, int WN, class LA, class LB, class EP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_gemm(LA la, LB lb, EP ep, int M, int N, int K, int kps) {
    constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
    static_assert(WM * WN == 4 && TM >= 1 && TN >= 1, "tile shape");
    // LDS rows of 4 groups (64 bytes, 16 banks), group g of row r stored in slot
    // g ^ ((r >> 2) & 3): the 16 lanes that read one group of 16 consecutive rows, and the 16
    // threads that write the 4 groups of 4 consecutive rows, each cover all 64 banks once.
    constexpr int SA = (BM * 4 + 255) / 256, SB = (BN * 4 + 255) / 256;
    // LDS: the operand tiles during the k loop; with a vector epilogue, afterwards, the
    // output tile as BF16 rows of BN + 8 elements (the padding spreads the four rows a
    // wavefront writes per instruction over distinct banks)
    constexpr int LDR = BN + 8;
    constexpr int OPS = BM * 4 + BN * 4, OUT = EP::kVector ? BM * LDR / 8 : 0;
    __shared__ bf16x8 smem[OPS > OUT ? OPS : OUT];
    bf16x8* const As = smem;
    bf16x8* const Bs = smem + BM * 4;
    auto slot = [](int r, int g) { return r * 4 + (g ^ ((r >> 2) & 3)); };
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv / WN, wn = wv % WN;
    // tile t: output-channel tiles of one pixel tile adjacent, then pixel tiles, split slowest
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = tile_order(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int bz = t / (gx * gy), bx = (t / gy) % gx, by = t % gy;
    const int m0 = bx * BM, n0 = by * BN;
    const int kb = bz * kps, ke = min(K, kb + kps);
    typename LA::Ctx ca[SA];
    typename LB::Ctx cb[SB];
#pragma unroll
    for (int q = 0; q < SA; ++q) ca[q] = la.row(m0 + ((tid + q * 256) >> 2), M);
#pragma unroll
    for (int q = 0; q < SB; ++q) cb[q] = lb.row(n0 + ((tid + q * 256) >> 2), N);
    bf16x8 ra[SA], rb[SB];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < SA; ++q) {
            const int e = tid + q * 256, k = k0 + 8 * (e & 3);
            ra[q] = la.load(ca[q], k, e < BM * 4 && k < ke);
        }
#pragma unroll
        for (int q = 0; q < SB; ++q) {
            const int e = tid + q * 256, k = k0 + 8 * (e & 3);
            rb[q] = lb.load(cb[q], k, e < BN * 4 && k < ke);
        }
    };
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    fetch(kb);
    for (int k0 = kb; k0 < ke; k0 += 32) {
        __syncthreads();                       // previous step's fragments consumed
#pragma unroll
        for (int q = 0; q < SA; ++q) {
            const int e = tid + q * 256;
            if (e < BM * 4) As[slot(e >> 2, e & 3)] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < SB; ++q) {
            const int e = tid + q * 256;
            if (e < BN * 4) Bs[slot(e >> 2, e & 3)] = rb[q];
        }
        __syncthreads();
        if (k0 + 32 < ke) fetch(k0 + 32);
        bf16x8 a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[slot(wm * TM * 16 + i * 16 + (lane & 15), lane >> 4)];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[slot(wn * TN * 16 + j * 16 + (lane & 15), lane >> 4)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if constexpr (EP::kVector) {
        bf16* const tile = (bf16*)smem;
        __syncthreads();                       // every wavefront done with the operand tiles
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm * TM * 16 + i * 16 + 4 * (lane >> 4) + r;
                    const int col = wn * TN * 16 + j * 16 + (lane & 15);
                    tile[row * LDR + col] = (__bf16)ep.pre(n0 + col, acc[i][j][r]);
                }
        __syncthreads();
        constexpr int GPR = BN / 8;            // 8-channel groups per row
        for (int e = tid; e < BM * GPR; e += 256) {
            const int row = e / GPR, g = e - row * GPR;
            const int m = m0 + row, n = n0 + 8 * g;
            if (m < M && n < ep.N) ep.store8(m, n, *(const bf16x8*)(tile + row * LDR + 8 * g));
        }
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = m0 + wm * TM * 16 + i * 16 + 4 * (lane >> 4) + r;
                    const int n = n0 + wn * TN * 16 + j * 16 + (lane & 15);
                    if (m < M) ep(m, n, acc[i][j][r], bz);
                }
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
// Byte extents of the loaders' buffers (below 2^31 by the host's size checks).
inline int tensor_bytes(const Tensor& t) { return (int)((size_t)t.B * t.H * t.W * t.cs * sizeof(bf16)); }
inline int matrix_bytes(int rows, int cols) { return (int)((size_t)rows * cols * sizeof(bf16)); }

hipError_t conv_fwd(const Tensor& x, const bf16* w, const float* bias, int relu, const Tensor& y,
                    int ksize, hipStream_t s) {
    const int taps = ksize * ksize;
    LoadConvA la{x.p, x.B, x.H, x.W, x.C, x.cs, x.coff, ilog2(x.C), taps * x.C, 0, ksize, tensor_bytes(x)};
    LoadRows lb{w, y.C, taps * x.C, taps * x.C, matrix_bytes(y.C, taps * x.C)};
    EpiAct ep{y.p, bias, y.cs, y.coff, relu, y.C};
    return gemm(la, lb, ep, x.B * x.H * x.W, y.C, taps * x.C, 1, s);
}

// dx[p][ci] = sum_{tap, co} dz[p - off(tap)][co] wt[ci][tap][co]
hipError_t conv_dgrad(const Tensor& dz, const bf16* wt, const Tensor& dx, int ksize, hipStream_t s,
                      const Tensor* relu_of) {
    const int taps = ksize * ksize;
    LoadConvA la{dz.p, dz.B, dz.H, dz.W, dz.C, dz.cs, dz.coff, ilog2(dz.C), taps * dz.C, 1, ksize, tensor_bytes(dz)};
    LoadRows lb{wt, dx.C, taps * dz.C, taps * dz.C, matrix_bytes(dx.C, taps * dz.C)};
    EpiAct ep{dx.p, nullptr, dx.cs, dx.coff, 0, dx.C, relu_of ? relu_of->p : nullptr,
              relu_of ? relu_of->cs : 0, relu_of ? relu_of->coff : 0};
    return gemm(la, lb, ep, dz.B * dz.H * dz.W, dx.C, taps * dz.C, 1, s);
}

// y[b, 2y+d/2, 2x+d%2, co] = sum_ci x[b,y,x,ci] w[co][d][ci] + bias[co]
hipError_t upconv_fwd(const Tensor& x, const bf16* w, const float* bias, const Tensor& y,
                      hipStream_t s) {
    LoadRows la{x.p + x.coff, x.B * x.H * x.W, x.C, x.cs, tensor_bytes(x) - 2 * x.coff};
    LoadRows lb{w, 4 * y.C, x.C, x.C, matrix_bytes(4 * y.C, x.C)};
    EpiUp ep{y.p, bias, x.B, x.H, x.W, y.C, y.cs, y.coff, 4 * y.C};
    return gemm(la, lb, ep, x.B * x.H * x.W, 4 * y.C, x.C, 1, s);
}

// dx[b,y,x,ci] = sum_{d,co} g[b,2y+d/2,2x+d%2,co] wt[ci][d][co]
hipError_t upconv_dgrad(const Tensor& g, const bf16* wt, const Tensor& dx, hipStream_t s,
                        const Tensor* relu_of) {
    LoadUpGradA la{g.p, dx.B, dx.H, dx.W, g.C, g.cs, g.coff, ilog2(g.C), 4 * g.C, tensor_bytes(g)};
    LoadRows lb{wt, dx.C, 4 * g.C, 4 * g.C, matrix_bytes(dx.C, 4 * g.C)};
    EpiAct ep{dx.p, nullptr, dx.cs, dx.coff, 0, dx.C, relu_of ? relu_of->p : nullptr,
              relu_of ? relu_of->cs : 0, relu_of ? relu_of->coff : 0};
    return gemm(la, lb, ep, dx.B * dx.H * dx.W, dx.C, 4 * g.C, 1, s);
}

// --------------------------------------------------------------------------- weight gradients
// Partial weight gradients over pixel slabs, as GEMMs whose reduction runs over pixels:
//   3x3 conv:    m = co, n = tap * Ci + ci:   sum_p dZ[p][co] X[p + off(tap)][ci]
//   2x2 up-conv: m = d * Co + co, n = ci:     sum_p G[b, 2y + d/2, 2x + d%2][co] X[p][ci]
//                (p = (b, y, x) over the up-conv's input)
// stored as part[z][co][tap][ci] (tap = d for the up-conv). For the 3x3 conv each split also
// stores the bias-gradient partials sum_p dZ[p][co] after its weight block, part[z] being
// Co * 9 * Ci + Co floats (the parameter layout's weights-then-bias order, so one split-K
// reduction yields both): the blocks of the first n tile add up the dZ rows they stage.
// Pixels are strided in NHWC, so
// each 64-pixel step stages both operands transposed into LDS ([row][pixel], rows padded to
// 72 elements): a thread loads 16 bytes (8 consecutive channels = 8 rows of one tap) for each
// of a few consecutive pixels and writes them as 8 short row segments, and an MFMA fragment
// (8 consecutive pixels of one row) is one 16-byte LDS read. Rows of a thread group and
// pixel groups interleave so that each LDS write instruction covers every bank once. The
// next step's operands are loaded into registers while the current step is multiplied.
// Block: TM x TN output tile (TM * TN = 64 * 64, 4 wavefronts of 32 x 32; TM = 32 when m
// has at most 32 rows); grid (m tiles, n tiles, splits), split z covering pixels
// [z kps, min(P, (z + 1) kps)), kps a multiple of 32. Channel counts are multiples of 8, so
// an 8-row group never straddles a tap or a sub-pixel. Registers are held to five wavefronts
// per SIMD (measured faster than four with the compiler's free choice).
constexpr int kWgStep = 64;
constexpr int kWgRow = kWgStep + 8;
template <int UP, int TM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_wgrad(Tensor dz, Tensor x, float* __restrict__ part,
                                               int P, int kps) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    constexpr int TN = 64 * 64 / TM;
    constexpr int WM = TM / 32, WN = 4 / WM;       // wavefront grid
    constexpr int NTAP = UP ? 4 : 9;
    // A staging: OA row groups x 16 pixel groups of AP = 4 pixels (threads past OA * 16 idle);
    // B staging: OB row groups x GB pixel groups of BP pixels (all 256 threads)
    constexpr int OA = TM / 8, GA = 16, AP = kWgStep / GA;
    constexpr int OB = TN / 8, GB = 256 / OB, BP = kWgStep / GB;
    static_assert(AP == 4 && (BP == 4 || BP == 2), "staging shapes");
    __shared__ __attribute__((aligned(16))) bf16 As[TM * kWgRow], Bs[TN * kWgRow];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv / WN, wn = wv % WN;
    // tile t: the (m, n) tiles of one pixel slab adjacent, slabs in order
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = tile_order(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int bz = t / (gx * gy), bx = t % gx, by = (t / gx) % gy;
    const int m0 = bx * TM, n0 = by * TN;
    const int pb = bz * kps, pe = min(P, pb + kps);
    const int Co = dz.C, Ci = x.C;
    const int M = UP ? 4 * Co : Co, N = UP ? Ci : 9 * Ci;
    const int H = x.H, W = x.W;                  // the pixel grid p runs over
    const int ga = tid % GA, oa = tid / GA;
    const bool a_act = oa < OA;
    const int gb = tid % GB, ob = tid / GB;
    const int m = m0 + 8 * oa;
    const bool m_ok = a_act && m < M;
    const int d = UP && m_ok ? m / Co : 0, co = m_ok ? m - d * Co : 0;
    const int n = n0 + 8 * ob;
    const bool n_ok = n < N;
    const int tap = !UP && n_ok ? n / Ci : 4, ci = n_ok ? n - (UP ? 0 : tap * Ci) : 0;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;  // zero shift for the up-conv (tap 4)
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 av[AP], bv[BP];
    const int a_bytes = (int)((size_t)dz.B * dz.H * dz.W * dz.cs * sizeof(bf16));
    const int b_bytes = (int)((size_t)x.B * x.H * x.W * x.cs * sizeof(bf16));
    auto load = [&](int k0) {
        if (a_act) {   // A: dZ at the pixel (conv), G at the row group's sub-pixel d (up-conv)
            int p = k0 + AP * ga;
            int yb = p / W, xx = p - yb * W;     // one division per step, then carries
            int b = yb / H, yy = yb - b * H;
#pragma unroll
            for (int q = 0; q < AP; ++q) {
                const int o = UP ? ((b * 2 * H + 2 * yy + (d >> 1)) * (2 * W) + 2 * xx + (d & 1)) * dz.cs
                                 : p * dz.cs;
                av[q] = bld8(dz.p, a_bytes, p < pe && m_ok ? 2 * (o + dz.coff + co) : kOOB);
                ++p;
                if (++xx == W) { xx = 0; if (++yy == H) { yy = 0; ++b; } }
            }
        }
        {   // B: X at the pixel shifted by the row group's tap (conv) or at the pixel (up-conv)
            int p = k0 + BP * gb;
            int yb = p / W, xx = p - yb * W;
            int b = yb / H, yy = yb - b * H;
#pragma unroll
            for (int q = 0; q < BP; ++q) {
                const int sy = yy + dy, sx = xx + dx;
                const bool ok = p < pe && n_ok && (unsigned)sy < (unsigned)H && (unsigned)sx < (unsigned)W;
                bv[q] = bld8(x.p, b_bytes, ok ? 2 * (((b * H + sy) * W + sx) * x.cs + x.coff + ci) : kOOB);
                ++p;
                if (++xx == W) { xx = 0; if (++yy == H) { yy = 0; ++b; } }
            }
        }
    };
    // bias partials (3x3 conv, first n tile): thread t adds 8 pixels of rows t / 8 + 32 r
    constexpr int BR = TM / 32;
    const bool bias_blk = !UP && by == 0;
    float bsum[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) bsum[r] = 0.f;
    load(pb);
    for (int k0 = pb; k0 < pe; k0 += kWgStep) {
        __syncthreads();                       // previous step's fragments consumed
        if (a_act) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                *(bf16x4*)(As + (8 * oa + c) * kWgRow + AP * ga) =
                    bf16x4{av[0][c], av[1][c], av[2][c], av[3][c]};
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if constexpr (BP == 4)
                *(bf16x4*)(Bs + (8 * ob + c) * kWgRow + BP * gb) =
                    bf16x4{bv[0][c], bv[1][c], bv[2][c], bv[3][c]};
            else
                *(bf16x2*)(Bs + (8 * ob + c) * kWgRow + BP * gb) = bf16x2{bv[0][c], bv[1][c]};
        }
        __syncthreads();
        if (k0 + kWgStep < pe) load(k0 + kWgStep);
        if (bias_blk) {
#pragma unroll
            for (int r = 0; r < BR; ++r) {
                const bf16x8 v = *(const bf16x8*)(As + ((tid >> 3) + 32 * r) * kWgRow + 8 * (tid & 7));
#pragma unroll
                for (int u = 0; u < 8; ++u) bsum[r] += (float)v[u];
            }
        }
#pragma unroll
        for (int kk = 0; kk < kWgStep; kk += 32) {
            bf16x8 a[2], bb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *(const bf16x8*)(As + (wm * 32 + i * 16 + (lane & 15)) * kWgRow + kk + 8 * (lane >> 4));
                bb[i] = *(const bf16x8*)(Bs + (wn * 32 + i * 16 + (lane & 15)) * kWgRow + kk + 8 * (lane >> 4));
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
    }
    float* dst = part + (size_t)bz * (Co * NTAP * Ci + (UP ? 0 : Co));
    if (bias_blk) {
#pragma unroll
        for (int r = 0; r < BR; ++r) {
            float v = bsum[r];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            const int o = m0 + (tid >> 3) + 32 * r;
            if ((tid & 7) == 0 && o < M) dst[(size_t)M * N + o] = v;
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int nn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (o < M && nn < N) {
                    if (UP) {
                        const int dd = o / Co, cc = o - dd * Co;
                        dst[((size_t)cc * 4 + dd) * Ci + nn] = acc[i][j][r];
                    } else {
                        dst[(size_t)o * N + nn] = acc[i][j][r];
                    }
                }
            }
}

template <int UP>
hipError_t wgrad(const Tensor& x, const Tensor& dz, float* part, int splits, hipStream_t s) {
    const int P = x.B * x.H * x.W;
    const int kps = wgrad_slab(P, splits);
    const int sp = wgrad_splits_used(P, splits);
    const int M = UP ? 4 * dz.C : dz.C, N = UP ? x.C : 9 * x.C;
    if (M <= 32) {
        dim3 g(1, (N + 127) / 128, sp);
        k_wgrad<UP, 32><<<g, 256, 0, s>>>(dz, x, part, P, kps);
    } else {
        dim3 g((M + 63) / 64, (N + 63) / 64, sp);
        k_wgrad<UP, 64><<<g, 256, 0, s>>>(dz, x, part, P, kps);
    }
    return hipGetLastError();
}

hipError_t conv_wgrad(const Tensor& x, const Tensor& dz, float* part, int splits, int ksize,
                      hipStream_t s) {
    if (ksize != 3) return hipErrorInvalidValue;
    return wgrad<0>(x, dz, part, splits, s);
}

hipError_t upconv_wgrad(const Tensor& x, const Tensor& g, float* part, int splits, hipStream_t s) {
    return wgrad<1>(x, g, part, splits, s);
}

}  // namespace nn
}  // namespace eit
