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
#include <type_traits>

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

// Direct buffer-to-LDS loads (the halo-tile convolution and the 3x3 weight gradients).
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
typedef __attribute__((address_space(3))) bf16 lds_bf16;

__device__ __forceinline__ i32x4 rsrc_words(const void* base, int bytes) {
    const unsigned long long a = (unsigned long long)base;
    return i32x4{(int)(unsigned)a, (int)((unsigned)(a >> 32) & 0xffffu), bytes, 0x00020000};
}
// 16 bytes per lane from byte offset voff of the resource (>= extent: zeros) into LDS at
// lds_base + 16 * lane; lds_base is uniform across the wavefront. The LDS base is an operand
// bound to M0 (the "{m0}" constraint), so the compiler sets M0 itself and knows it is read.
__device__ __forceinline__ void dma16(i32x4 rs, unsigned lds_base, int voff) {
    asm volatile("buffer_load_dwordx4 %0, %1, 0 offen lds"
                 :: "v"(voff), "s"(rs), "{m0}"(lds_base) : "memory");
}
// Wait until at most N vector-memory operations of this wavefront are outstanding (the
// expcnt and lgkmcnt fields of the s_waitcnt immediate left at their maximum).
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
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

// Transposed-convolution weights [Co][4][Ci] read with the rows in sub-pixel-major order:
// GEMM row n = d Co + co is parameter row 4 co + d, so 8 consecutive GEMM columns are 8
// consecutive channels of one output pixel (the epilogue stores them with one 16-byte store).
struct LoadRowsUp {
    const bf16* t; int co_n, K, ld, bytes;
    typedef LoadRows::Ctx Ctx;
    __device__ Ctx row(int r, int) const {
        const int d = r / co_n, co = r - d * co_n;
        return Ctx{r < 4 * co_n ? 2 * (4 * co + d) * ld : 0, r < 4 * co_n};
    }
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
// The same with the GEMM columns in sub-pixel-major order (n = d C + c, LoadRowsUp): staged
// through LDS and stored 8 channels (16 bytes) at a time.
struct EpiUpV {
    static constexpr bool kVector = true;
    bf16* t; const float* bias; int B, H, W, C, cs, coff, N;
    __device__ float pre(int n, float v) const { return n < N ? v + bias[n % C] : v; }
    __device__ void store8(int m, int n, bf16x8 v) const {
        const int d = n / C, c = n - d * C;
        const int x = m % W, yb = m / W, y = yb % H, b = yb / H;
        *(bf16x8*)(t + ((size_t)(b * 2 * H + 2 * y + (d >> 1)) * (2 * W) + 2 * x + (d & 1)) * cs + coff + c) = v;
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

// --------------------------------------------------------------------------- 3x3 convolution, halo tiles
// The implicit GEMM above fetches every input pixel once per tap (nine times per layer) and
// every weight row once per 32-k step of every 128-pixel tile; at the 32- and 64-channel
// layers that operand stream keeps the L2 channels 80-85 % busy and bounds the kernel. This
// kernel computes a TR x TW pixel tile (TR * TW = 64 TM, TM 16-pixel fragments per wavefront,
// 4 wavefronts) over BN (32) output channels and runs the reduction as C / 32 channel chunks, each
// staged once: the chunk's (TR + 2) x (TW + 2) input pixels (the tile and its one-pixel border,
// zeros outside the image) and its BN x 9 x 32 weights, both by direct buffer-to-LDS loads;
// the nine taps then read shifted A fragments from the staged tile. Per 32-channel chunk a
// block reads (TR + 2)(TW + 2) input pixels instead of 9 TR TW, and its weights once.
// LDS layouts (16-byte groups of 8 channels):
//   tile:    pixel h = hr (TW + 2) + hc, group g at slot 4 h + (g ^ ((h >> 2) & 3)): the 16 lanes
//            of one fragment read 16 consecutive h at one g and cover all 64 banks once;
//   weights: row n (37 slots: tap t, group g at slot 4 t + g, one pad slot), so 16 consecutive
//            rows at one slot fall on distinct banks (37 x 16 bytes = 148 words = 20 mod 64).
// A direct load writes lane i's 16 bytes at the wavefront's base + 16 i, so each lane loads
// the (pixel, group) or (row, tap, group) its slot holds; slots past the data read zeros.
// flip = 1 is the data-gradient form (input pixel p - off(tap)). Sums run chunk by chunk,
// taps in order inside a chunk, 32 k per MFMA.
template <int TR, int TW, int BN>
__global__ __launch_bounds__(256) void k_conv3(Tensor x, const bf16* __restrict__ w, int ldw, int N,
                                               int flip, EpiAct ep) {
    constexpr int BM = TR * TW, TM = BM / 64, TN = BN / 16;
    static_assert(BM % 64 == 0 && TM >= 1 && BN % 16 == 0, "tile shape");
    constexpr int HW = TW + 2, HP = (TR + 2) * HW;                 // staged pixels
    constexpr int HS = (4 * HP + 63) / 64 * 64;                    // tile slots, whole wavefront loads
    constexpr int WR = 37, WS = (BN * WR + 63) / 64 * 64;           // weight slots
    constexpr int DH = HS / 64, DW = WS / 64;                       // wavefront loads per chunk
    constexpr int LDR = BN + 8;
    constexpr int OUT = BM * LDR / 8;
    __shared__ bf16x8 smem[HS + WS > OUT ? HS + WS : OUT];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int H = x.H, W = x.W, C = x.C;
    const int tx = W / TW, ty = H / TR;
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = tile_order(blockIdx.x + gx * blockIdx.y, gx * gy);
    const int pt = t / gy, by = t % gy;                             // n tiles of a pixel tile adjacent
    const int b = pt / (tx * ty), y0 = (pt / tx) % ty * TR, x0 = pt % tx * TW;
    const int n0 = by * BN;
    const i32x4 rsX = rsrc_words(x.p, (int)((size_t)x.B * H * W * x.cs * sizeof(bf16)));
    const i32x4 rsW = rsrc_words(w, (int)((size_t)N * ldw * sizeof(bf16)));
    const unsigned lds0 = (unsigned)(size_t)(lds_bf16*)(bf16*)smem;
    const unsigned ldsW = lds0 + HS * 16u;
    // tile loads: slot s = 64 (DH-slot wavefront load index) + lane -> staged pixel, group
    // byte offsets of channel 0 of each load's group (-1: the slot reads zeros)
    int offX[(DH + 3) / 4];
#pragma unroll
    for (int j = 0; j < (DH + 3) / 4; ++j) {
        const int q = wv + 4 * j, sl = 64 * q + lane, h = sl >> 2;
        const int g = (sl & 3) ^ ((h >> 2) & 3);
        const int hr = h / HW, hc = h - hr * HW;
        const int yy = y0 - 1 + hr, xx = x0 - 1 + hc;
        const bool ok = q < DH && h < HP && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
        offX[j] = ok ? 2 * (((b * H + yy) * W + xx) * x.cs + x.coff + 8 * g) : -1;
    }
    int offW[(DW + 3) / 4];
#pragma unroll
    for (int j = 0; j < (DW + 3) / 4; ++j) {
        const int q = wv + 4 * j, sl = 64 * q + lane, n = sl / WR, e = sl - n * WR;
        const int tap = e >> 2, g = e & 3;
        const bool ok = q < DW && n < BN && e < 36 && n0 + n < N;
        offW[j] = ok ? 2 * ((n0 + n) * ldw + tap * C + 8 * g) : -1;
    }
    // A fragment slots of this lane for tap offset (0, 0): tile pixel of fragment i, group
    const int g = lane >> 4;
    int hA[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int p = wv * TM * 16 + i * 16 + (lane & 15), r = p / TW, c = p - r * TW;
        hA[i] = (r + 1) * HW + c + 1;
    }
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int sgn = flip ? -1 : 1;
    for (int c0 = 0; c0 < C; c0 += 32) {
        if (c0) __syncthreads();               // every wavefront done with the previous chunk
#pragma unroll
        for (int j = 0; j < (DH + 3) / 4; ++j)
            if (wv + 4 * j < DH) dma16(rsX, lds0 + (unsigned)(wv + 4 * j) * 1024u, offX[j] >= 0 ? offX[j] + 2 * c0 : kOOB);
#pragma unroll
        for (int j = 0; j < (DW + 3) / 4; ++j)
            if (wv + 4 * j < DW) dma16(rsW, ldsW + (unsigned)(wv + 4 * j) * 1024u, offW[j] >= 0 ? offW[j] + 2 * c0 : kOOB);
        wait_vm<0>();
        __syncthreads();                       // the chunk is staged
        const bf16x8* Ws = smem + HS;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dh = sgn * ((tap / 3 - 1) * HW + (tap % 3 - 1));
            bf16x8 a[TM], bb[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int h = hA[i] + dh;
                a[i] = smem[4 * h + (g ^ ((h >> 2) & 3))];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) bb[j] = Ws[(j * 16 + (lane & 15)) * WR + 4 * tap + g];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
    }
    bf16* const tile = (bf16*)smem;
    __syncthreads();                           // every wavefront done with the staged chunk
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wv * TM * 16 + i * 16 + 4 * (lane >> 4) + r;
                const int col = j * 16 + (lane & 15);
                tile[row * LDR + col] = (__bf16)ep.pre(n0 + col, acc[i][j][r]);
            }
    __syncthreads();
    constexpr int GPR = BN / 8;
    for (int e = tid; e < BM * GPR; e += 256) {
        const int row = e / GPR, gg = e - row * GPR;
        const int r = row / TW, c = row - r * TW;
        const int m = (b * H + y0 + r) * W + x0 + c, n = n0 + 8 * gg;
        if (n < ep.N) ep.store8(m, n, *(const bf16x8*)(tile + row * LDR + 8 * gg));
    }
}

// Halo-tile launch for a 3x3 convolution whose input has C % 32 == 0 channels and whose image
// sides are multiples of the tile (returns false otherwise: the implicit GEMM runs instead).
// 256-pixel tiles, or 128-pixel tiles where 256 would leave fewer than 1024 blocks.
template <int TR, int TW, int BN>
hipError_t conv3_launch(const Tensor& x, const bf16* w, int ldw, int N, int flip, const EpiAct& ep,
                        hipStream_t s) {
    dim3 g(x.B * (x.H / TR) * (x.W / TW), (N + BN - 1) / BN);
    k_conv3<TR, TW, BN><<<g, 256, 0, s>>>(x, w, ldw, N, flip, ep);
    return hipGetLastError();
}
template <int BN>
bool conv3_halo(const Tensor& x, const bf16* w, int N, int flip, const EpiAct& ep, hipStream_t s,
                hipError_t* err) {
    if (x.C % 32 || x.W % 32) return false;
    const int ldw = 9 * x.C, nt = (N + BN - 1) / BN;
    const long px = (long)x.B * x.H * x.W;
    const bool big = px / 256 * nt >= 1024;
    if (x.W % 64 == 0) {
        if (big && x.H % 4 == 0) { *err = conv3_launch<4, 64, BN>(x, w, ldw, N, flip, ep, s); return true; }
        if (x.H % 2 == 0) { *err = conv3_launch<2, 64, BN>(x, w, ldw, N, flip, ep, s); return true; }
        return false;
    }
    if (big && x.H % 8 == 0) { *err = conv3_launch<8, 32, BN>(x, w, ldw, N, flip, ep, s); return true; }
    if (x.H % 4 == 0) { *err = conv3_launch<4, 32, BN>(x, w, ldw, N, flip, ep, s); return true; }
    return false;
}
bool conv3_halo_any(const Tensor& x, const bf16* w, int N, int flip, const EpiAct& ep, hipStream_t s,
                    hipError_t* err) {
    // 32 output channels per block at every width: 45 KB of LDS and 128 VGPRs leave three
    // blocks per CU (64-channel blocks: 64 KB, two), which outweighs staging each pixel tile
    // once per 32 output channels (training step 2.38 -> 2.31 ms)
    return conv3_halo<32>(x, w, N, flip, ep, s, err);
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
    EpiAct ep{y.p, bias, y.cs, y.coff, relu, y.C};
    hipError_t err;
    if (ksize == 3 && conv3_halo_any(x, w, y.C, 0, ep, s, &err)) return err;
    LoadConvA la{x.p, x.B, x.H, x.W, x.C, x.cs, x.coff, ilog2(x.C), taps * x.C, 0, ksize, tensor_bytes(x)};
    LoadRows lb{w, y.C, taps * x.C, taps * x.C, matrix_bytes(y.C, taps * x.C)};
    return gemm(la, lb, ep, x.B * x.H * x.W, y.C, taps * x.C, 1, s);
}

// dx[p][ci] = sum_{tap, co} dz[p - off(tap)][co] wt[ci][tap][co]
hipError_t conv_dgrad(const Tensor& dz, const bf16* wt, const Tensor& dx, int ksize, hipStream_t s,
                      const Tensor* relu_of) {
    const int taps = ksize * ksize;
    EpiAct ep{dx.p, nullptr, dx.cs, dx.coff, 0, dx.C, relu_of ? relu_of->p : nullptr,
              relu_of ? relu_of->cs : 0, relu_of ? relu_of->coff : 0};
    hipError_t err;
    if (ksize == 3 && conv3_halo_any(dz, wt, dx.C, 1, ep, s, &err)) return err;
    LoadConvA la{dz.p, dz.B, dz.H, dz.W, dz.C, dz.cs, dz.coff, ilog2(dz.C), taps * dz.C, 1, ksize, tensor_bytes(dz)};
    LoadRows lb{wt, dx.C, taps * dz.C, taps * dz.C, matrix_bytes(dx.C, taps * dz.C)};
    return gemm(la, lb, ep, dz.B * dz.H * dz.W, dx.C, taps * dz.C, 1, s);
}

// y[b, 2y+d/2, 2x+d%2, co] = sum_ci x[b,y,x,ci] w[co][d][ci] + bias[co]
hipError_t upconv_fwd(const Tensor& x, const bf16* w, const float* bias, const Tensor& y,
                      hipStream_t s) {
    LoadRows la{x.p + x.coff, x.B * x.H * x.W, x.C, x.cs, tensor_bytes(x) - 2 * x.coff};
    if (y.C % 8 == 0 && y.cs % 8 == 0 && y.coff % 8 == 0) {
        LoadRowsUp lb{w, y.C, x.C, x.C, matrix_bytes(4 * y.C, x.C)};
        EpiUpV ep{y.p, bias, x.B, x.H, x.W, y.C, y.cs, y.coff, 4 * y.C};
        return gemm(la, lb, ep, x.B * x.H * x.W, 4 * y.C, x.C, 1, s);
    }
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
// Partial weight gradients over pixel slabs, as GEMMs whose reduction runs over pixels, stored
// as part[z][co][tap][ci] for split z:
//   3x3 conv:    m = co, n = tap * Ci + ci:   sum_p dZ[p][co] X[p + off(tap)][ci]
//                (k_wgrad_tr below; part[z] also holds the Co bias partials sum_p dZ[p][co]
//                after its Co * 9 * Ci weights, the parameter layout's order, so one split-K
//                reduction yields both)
//   2x2 up-conv: m = d * Co + co, n = ci:     sum_p G[b, 2y + d/2, 2x + d%2][co] X[p][ci]
//                (p = (b, y, x) over the up-conv's input; tap = d; k_wgrad_up)
// k_wgrad_up: pixels are strided in NHWC, so each 64-pixel step stages both operands
// transposed into LDS ([row][pixel], rows padded to 72 elements): a thread loads 16 bytes
// (8 consecutive channels = 8 rows of one sub-pixel) for each of a few consecutive pixels and
// writes them as 8 short row segments, and an MFMA fragment (8 consecutive pixels of one row)
// is one 16-byte LDS read. Rows of a thread group and pixel groups interleave so that each
// LDS write instruction covers every bank once. The next step's operands are loaded into
// registers while the current step is multiplied.
// Block: TM x TN output tile (TM * TN = 64 * 64, 4 wavefronts of 32 x 32; TM = 32 when m
// has at most 32 rows); grid (m tiles, n tiles, splits), split z covering pixels
// [z kps, min(P, (z + 1) kps)), kps a multiple of 32. Channel counts are multiples of 8, so
// an 8-row group never straddles a sub-pixel. Registers are held to five wavefronts per SIMD
// (measured faster than four with the compiler's free choice).
constexpr int kWgStep = 64;
constexpr int kWgRow = kWgStep + 8;
template <int TM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_wgrad_up(Tensor dz, Tensor x, float* __restrict__ part,
                                                  int P, int kps) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    constexpr int TN = 64 * 64 / TM;
    constexpr int WM = TM / 32, WN = 4 / WM;       // wavefront grid
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
    const int M = 4 * Co, N = Ci;
    const int H = x.H, W = x.W;                  // the pixel grid p runs over
    const int ga = tid % GA, oa = tid / GA;
    const bool a_act = oa < OA;
    const int gb = tid % GB, ob = tid / GB;
    const int m = m0 + 8 * oa;
    const bool m_ok = a_act && m < M;
    const int d = m_ok ? m / Co : 0, co = m_ok ? m - d * Co : 0;
    const int n = n0 + 8 * ob;
    const bool n_ok = n < N;
    const int ci = n_ok ? n : 0;
    f32x4 acc[2][2], accb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        accb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // bias sums (first n tile, first wavefront column): products with a fragment of ones give
    // sum_p G[(d, co)][p] per row, the up-conv bias gradient before its sum over d
    const bool bias_w = by == 0 && wn == 0;
    bf16x8 ones;
#pragma unroll
    for (int u = 0; u < 8; ++u) ones[u] = (__bf16)1.0f;
    bf16x8 av[AP], bv[BP];
    const int a_bytes = (int)((size_t)dz.B * dz.H * dz.W * dz.cs * sizeof(bf16));
    const int b_bytes = (int)((size_t)x.B * x.H * x.W * x.cs * sizeof(bf16));
    auto load = [&](int k0) {
        if (a_act) {   // A: G at the row group's sub-pixel d
            int p = k0 + AP * ga;
            int yb = p / W, xx = p - yb * W;     // one division per step, then carries
            int b = yb / H, yy = yb - b * H;
#pragma unroll
            for (int q = 0; q < AP; ++q) {
                const int o = ((b * 2 * H + 2 * yy + (d >> 1)) * (2 * W) + 2 * xx + (d & 1)) * dz.cs;
                av[q] = bld8(dz.p, a_bytes, p < pe && m_ok ? 2 * (o + dz.coff + co) : kOOB);
                ++p;
                if (++xx == W) { xx = 0; if (++yy == H) { yy = 0; ++b; } }
            }
        }
#pragma unroll
        for (int q = 0; q < BP; ++q) {           // B: X at the pixel
            const int p = k0 + BP * gb + q;
            bv[q] = bld8(x.p, b_bytes, p < pe && n_ok ? 2 * (p * x.cs + x.coff + ci) : kOOB);
        }
    };
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
            if (bias_w) {
#pragma unroll
                for (int i = 0; i < 2; ++i) accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], ones, accb[i], 0, 0, 0);
            }
        }
    }
    float* dst = part + (size_t)bz * (Co * 4 * Ci + 4 * Co);     // weights, then the 4 Co row sums
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                if (bias_w && (lane & 15) == 0 && o < M) dst[(size_t)Co * 4 * Ci + o] = accb[i][r];
                const int nn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (o < M && nn < N) {
                    const int dd = o / Co, cc = o - dd * Co;
                    dst[((size_t)cc * 4 + dd) * Ci + nn] = acc[i][j][r];
                }
            }
}

// --------------------------------------------------------------------------- weight gradients, 3x3
// The 3x3 convolution's weight gradient without register staging: both operands go from
// memory to LDS by direct buffer loads (buffer_load ... lds: lane i of a wavefront writes
// its 16 bytes at the wavefront's LDS base + 16 i), kept in their memory layout (rows of
// pixels, 8 channels per 16-byte slot), and the MFMA fragments, which need 8 consecutive
// pixels of one channel per lane, are read with the transposing LDS load ds_read_b64_tr_b16:
// in each 16-lane group, lane 4r + c supplies the address of 4 consecutive channels
// (4c .. 4c + 3) of pixel row r, and lane 4c + e receives channel 4c + e of the 4 rows. Two
// such reads (pixel rows 8g .. 8g + 3 and 8g + 4 .. 8g + 7 for lane group g) give a lane the
// same 8 pixels of one channel that the MFMA's k layout asks for, so the products are those
// of the register-staged kernel. No VALU work transposes data and no registers hold the next
// step's operands, so NS stages of 64 pixels are in flight: the loads of stage s + NS - 1
// are issued while stage s is multiplied. The stage ring is counted with explicit vmcnt
// waits (the loads are written in inline asm, which the compiler does not track): every
// wavefront issues the same number of loads per stage (past the slab's end they read zeros),
// so "stage s landed" is "at most (NS - 2) stages' loads outstanding", and a barrier then
// makes every wavefront's part visible.
// Slot layout of an operand with C chunks (16-byte groups) per pixel row: pixel p, chunk q
// at slot C p + (q ^ swz(p)); the XOR spreads the 8 rows that one 32-lane half of a
// transposing read touches (rows 8g + 4h + r, r < 4, two values of g) over distinct 32-byte
// bank windows. Bias gradients (first n tile) are products with a fragment of ones in the
// wavefronts of the first n column: sum_p dZ[p][co] in the MFMA's FP32 accumulation.
template <int C>
__device__ __forceinline__ int wg_swz(int p) {
    static_assert(C == 4 || C == 8 || C == 16, "chunks per pixel row");
    if constexpr (C == 4) return ((p >> 3) & 1) << 1;
    else if constexpr (C == 8) return (((p >> 1) & 1) << 1) | (((p >> 3) & 1) << 2);
    else return ((p & 3) << 1) | (((p >> 3) & 1) << 3);
}

constexpr int kWtStep = 64;   // pixels per stage
template <int TM, int NS>
__global__ __launch_bounds__(256) void k_wgrad_tr(Tensor dz, Tensor x, float* __restrict__ part,
                                                  int P, int kps) {
    constexpr int TN = 64 * 64 / TM;
    constexpr int WM = TM / 32, WN = 4 / WM;
    constexpr int CA = TM / 8, CB = TN / 8;           // 16-byte chunks per pixel row
    constexpr int SA = kWtStep * CA, SB = kWtStep * CB;   // slots per stage
    constexpr int DA = SA / 256, DB = SB / 256;       // loads per wavefront per stage
    constexpr int D = DA + DB;
    static_assert(NS >= 2 && DA >= 1 && DB >= 1, "stage shape");
    __shared__ __attribute__((aligned(16))) bf16 lds[NS * (SA + SB) * 8];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: LDS bases go to m0
    const int wm = wv / WN, wn = wv % WN;
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = tile_order(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int bz = t / (gx * gy), bx = t % gx, by = (t / gx) % gy;
    const int m0 = bx * TM, n0 = by * TN;
    const int pb = bz * kps, pe = min(P, pb + kps);
    const int Co = dz.C, Ci = x.C, M = Co, N = 9 * Ci;
    const int H = x.H, W = x.W;
    const i32x4 rsA = rsrc_words(dz.p, (int)((size_t)dz.B * dz.H * dz.W * dz.cs * sizeof(bf16)));
    const i32x4 rsB = rsrc_words(x.p, (int)((size_t)x.B * x.H * x.W * x.cs * sizeof(bf16)));
    const unsigned lds0 = (unsigned)(size_t)(lds_bf16*)lds;

    // this lane's slots: pixel row and chunk of A load j and of B load j (fixed per stage)
    int pA[DA];
    unsigned offA[DA];      // byte offsets, modulo 2^32 (used only where the access is valid)
    bool okA[DA];
#pragma unroll
    for (int j = 0; j < DA; ++j) {
        const int sl = 64 * (wv * DA + j) + lane, p = sl / CA, q = (sl % CA) ^ wg_swz<CA>(p);
        pA[j] = p;
        okA[j] = m0 + 8 * q < M;
        offA[j] = 2u * (unsigned)((pb + p) * dz.cs + dz.coff + m0 + 8 * q);
    }
    int pB[DB], dyB[DB], dxB[DB], yyB[DB], xxB[DB];
    unsigned offB[DB];
    bool okB[DB];
#pragma unroll
    for (int j = 0; j < DB; ++j) {
        const int sl = 64 * (wv * DB + j) + lane, p = sl / CB, q = (sl % CB) ^ wg_swz<CB>(p);
        const int n = n0 + 8 * q;
        okB[j] = n < N;
        const int tap = okB[j] ? n / Ci : 4, ci = okB[j] ? n - tap * Ci : 0;
        dyB[j] = tap / 3 - 1;
        dxB[j] = tap % 3 - 1;
        pB[j] = p;
        const int P0 = pb + p;
        xxB[j] = P0 % W;
        yyB[j] = (P0 / W) % H;
        offB[j] = 2u * (unsigned)((P0 + dyB[j] * W + dxB[j]) * x.cs + x.coff + ci);
    }
    const unsigned stepA = 2u * kWtStep * dz.cs, stepB = 2u * kWtStep * x.cs;
    // loads of stage index st (pixels pb + 64 st ..) into ring buffer st % NS
    auto issue = [&](int st, int buf) {
        const int k0 = pb + kWtStep * st;
        const unsigned baseA = lds0 + (unsigned)(buf * (SA + SB)) * 16u;
        const unsigned baseB = baseA + SA * 16u;
#pragma unroll
        for (int j = 0; j < DA; ++j) {
            const bool ok = okA[j] && k0 + pA[j] < pe;
            dma16(rsA, baseA + (unsigned)(wv * DA + j) * 1024u, ok ? (int)offA[j] : kOOB);
            offA[j] += stepA;
        }
#pragma unroll
        for (int j = 0; j < DB; ++j) {
            const bool ok = okB[j] && k0 + pB[j] < pe && (unsigned)(yyB[j] + dyB[j]) < (unsigned)H &&
                            (unsigned)(xxB[j] + dxB[j]) < (unsigned)W;
            dma16(rsB, baseB + (unsigned)(wv * DB + j) * 1024u, ok ? (int)offB[j] : kOOB);
            offB[j] += stepB;
            xxB[j] += kWtStep;
            while (xxB[j] >= W) {
                xxB[j] -= W;
                if (++yyB[j] == H) yyB[j] = 0;
            }
        }
    };

    // fragment addresses (bytes from the operand's stage base): lane group g, row r, column
    // group c of a transposing read at pixel rows 8g + 4h + r (+ kk)
    const int g = lane >> 4, r = (lane >> 2) & 3, c = lane & 3;
    const int prow = 8 * g + r;
    unsigned fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int qa = (wm * 32 + i * 16) / 8, qb = (wn * 32 + i * 16) / 8;
        fa[i] = (unsigned)((CA * prow + ((qa ^ wg_swz<CA>(prow)) + (c >> 1))) * 16 + 8 * (c & 1));
        fb[i] = (unsigned)(SA * 16 + (CB * prow + ((qb ^ wg_swz<CB>(prow)) + (c >> 1))) * 16 + 8 * (c & 1));
    }
    const bool bias_w = by == 0 && wn == 0;
    f32x4 acc[2][2], accb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        accb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const int nsteps = (pe - pb + kWtStep - 1) / kWtStep;
#pragma unroll
    for (int st = 0; st < NS - 1; ++st) issue(st, st);
    // the step loop, instantiated with and without the bias products (a wavefront-uniform
    // choice; one loop with a branch inside costs accumulator copies every step)
    auto run = [&](auto bias_tag) {
        constexpr bool BIAS = decltype(bias_tag)::value;
        bf16x8 ones;
#pragma unroll
        for (int u = 0; u < 8; ++u) ones[u] = (__bf16)1.0f;
        int cur = 0, nxt = NS - 1;
        for (int s = 0; s < nsteps; ++s) {
            wait_vm<(NS - 2) * D>();               // this wavefront's loads of stage s landed
            __syncthreads();                       // everyone's landed; stage s - 1 consumed
            issue(s + NS - 1, nxt);
            const char __attribute__((address_space(3)))* st0 =
                (const char __attribute__((address_space(3)))*)(lds_bf16*)lds + cur * (SA + SB) * 16;
            auto tr = [&](unsigned off) {
                return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(st0 + off));
            };
#pragma unroll
            for (int kk = 0; kk < kWtStep; kk += 32) {
                bf16x8 a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const s16x4 a0 = tr(fa[i] + CA * 16 * kk), a1 = tr(fa[i] + CA * 16 * (kk + 4));
                    const s16x4 b0 = tr(fb[i] + CB * 16 * kk), b1 = tr(fb[i] + CB * 16 * (kk + 4));
                    a[i] = __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7));
                    b[i] = __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7));
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
                if constexpr (BIAS) {
#pragma unroll
                    for (int i = 0; i < 2; ++i)
                        accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], ones, accb[i], 0, 0, 0);
                }
            }
            cur = cur + 1 == NS ? 0 : cur + 1;
            nxt = nxt + 1 == NS ? 0 : nxt + 1;
        }
    };
    if (bias_w) run(std::true_type{});
    else run(std::false_type{});
    wait_vm<0>();                              // no load may still write this block's LDS
    float* dst = part + (size_t)bz * (Co * 9 * Ci + Co);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
            const int o = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r4;
            if (bias_w && (lane & 15) == 0 && o < M) dst[(size_t)M * N + o] = accb[i][r4];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int nn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (o < M && nn < N) dst[(size_t)o * N + nn] = acc[i][j][r4];
            }
        }
}

// --------------------------------------------------------------------------- weight gradients, 3x3 halo tiles
// dW[co][tap][ci] = sum_p dZ[p][co] X[p + off(tap)][ci] and db[co] = sum_p dZ[p][co] over
// TR x TW pixel tiles: per tile a block stages the tile's dZ (CO output channels) and the tile's
// X with its one-pixel border (32 input channels, zeros outside the image) once, by direct
// buffer-to-LDS loads, and all nine taps read from the staged X; k_wgrad_tr instead loads X
// once per tap column of every n tile. Three wavefronts, one per stencil row dy: wavefront w
// takes the taps (w, dx = -1, 0, 1) for CO output x 32 input channels and reads the dZ
// fragments once per 32-pixel k step for its three taps. Layouts: groups of 8 channels per
// pixel (CO / 8 for dZ, 4 for X), group g of pixel h at slot G h + (g ^ ((h >> 2) & 3)); MFMA
// fragments (8 consecutive pixels of one channel per lane) come from pairs of transposing
// reads (ds_read_b64_tr_b16), as in k_wgrad_tr. A block's split z covers tiles
// [z tps, (z + 1) tps) in order, with the next tile's loads in flight during the current one
// (two stage buffers); it writes its partial sums as part[z][co][tap][ci] followed by the Co
// bias partials (first input-channel chunk).
template <int TR, int TW, int CO>
__global__ __launch_bounds__(192) void k_wgrad3(Tensor dz, Tensor x, float* __restrict__ part, int tps, int ntiles) {
    constexpr int BM = TR * TW, HW = TW + 2, HP = (TR + 2) * HW, GA = CO / 8, TMo = CO / 16;
    constexpr int SA = BM * GA, SH = (4 * HP + 63) / 64 * 64, STG = SA + SH;
    constexpr int DA = SA / 64, DH = SH / 64, NW = 3;
    static_assert(BM % 32 == 0 && (GA == 4 || GA == 8), "tile");
    __shared__ __attribute__((aligned(16))) bf16 lds[2 * STG * 8];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int H = x.H, W = x.W, Co = dz.C, Ci = x.C;
    const int tx = W / TW, ty = H / TR;
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = tile_order(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int bz = t / (gx * gy), cot = t % gx, cic = (t / gx) % gy;   // channel tiles of a slab adjacent
    const int t0 = bz * tps, t1 = min(ntiles, t0 + tps);
    const i32x4 rsA = rsrc_words(dz.p, (int)((size_t)dz.B * H * W * dz.cs * sizeof(bf16)));
    const i32x4 rsX = rsrc_words(x.p, (int)((size_t)x.B * H * W * x.cs * sizeof(bf16)));
    const unsigned lds0 = (unsigned)(size_t)(lds_bf16*)lds;
    auto swz = [](int h) { return (h >> 2) & 3; };
    // loads of tile tt into stage buffer buf: wavefront w issues wavefront loads w, w + 3, ...
    auto issue = [&](int tt, int buf) {
        const int b = tt / (tx * ty), y0 = (tt / tx) % ty * TR, x0 = tt % tx * TW;
        const unsigned base = lds0 + (unsigned)(buf * STG) * 16u;
        for (int q = wv; q < DA + DH; q += NW) {
            int off = kOOB;
            if (q < DA) {
                const int sl = 64 * q + lane, P = sl / GA, g = (sl % GA) ^ swz(P);
                const int r = P / TW, c = P - r * TW;
                off = 2 * (((b * H + y0 + r) * W + x0 + c) * dz.cs + dz.coff + CO * cot + 8 * g);
                dma16(rsA, base + (unsigned)q * 1024u, off);
            } else {
                const int sl = 64 * (q - DA) + lane, h = sl >> 2, g = (sl & 3) ^ swz(h);
                const int hr = h / HW, hc = h - hr * HW, yy = y0 - 1 + hr, xx = x0 - 1 + hc;
                if (h < HP && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W)
                    off = 2 * (((b * H + yy) * W + xx) * x.cs + x.coff + 32 * cic + 8 * g);
                dma16(rsX, base + (unsigned)q * 1024u, off);
            }
        }
    };
    // transposing-read addresses: lane group g, row r, column piece c reads pixel row
    // 8 g + 4 hh + r of a 32-pixel k step, channels 16 i + 4 c .. + 3
    const int g = lane >> 4, r = (lane >> 2) & 3, c = lane & 3;
    auto slot_addr = [&](int G, int h, int i) {   // byte address of channels 16 i + 4 c .. of pixel h
        const int q = 2 * i + (c >> 1);
        return (G * h + (q ^ swz(h))) * 16 + 8 * (c & 1);
    };
    f32x4 acc[3][TMo][2], accb[TMo];
#pragma unroll
    for (int i = 0; i < TMo; ++i) {
        accb[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[d][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const bool bias_w = cic == 0 && wv == 0;
    bf16x8 ones;
#pragma unroll
    for (int u = 0; u < 8; ++u) ones[u] = (__bf16)1.0f;
    const int dyw = wv - 1;
    if (t0 < t1) issue(t0, 0);
    for (int tt = t0, it = 0; tt < t1; ++tt, ++it) {
        wait_vm<0>();                          // this wavefront's loads of tile tt landed
        __syncthreads();                       // every part landed; the other buffer consumed
        if (tt + 1 < t1) issue(tt + 1, (it + 1) & 1);
        const char __attribute__((address_space(3)))* st0 =
            (const char __attribute__((address_space(3)))*)(lds_bf16*)lds + (it & 1) * STG * 16;
        auto tr = [&](int off) { return __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(st0 + off)); };
        auto frag = [&](int o0, int o1) {
            const s16x4 v0 = tr(o0), v1 = tr(o1);
            return __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(v0, v1, 0, 1, 2, 3, 4, 5, 6, 7));
        };
#pragma unroll 1
        for (int k0 = 0; k0 < BM; k0 += 32) {
            const int P0 = k0 + 8 * g + r, P1 = P0 + 4;
            bf16x8 a[TMo];
#pragma unroll
            for (int i = 0; i < TMo; ++i) a[i] = frag(slot_addr(GA, P0, i), slot_addr(GA, P1, i));
            // halo pixel of tile pixel P shifted by (dyw, dx)
            const int h0 = (P0 / TW + 1 + dyw) * HW + P0 % TW + 1, h1 = (P1 / TW + 1 + dyw) * HW + P1 % TW + 1;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                bf16x8 bb[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) bb[j] = frag(SA * 16 + slot_addr(4, h0 + d - 1, j), SA * 16 + slot_addr(4, h1 + d - 1, j));
#pragma unroll
                for (int i = 0; i < TMo; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[d][i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[d][i][j], 0, 0, 0);
            }
            if (bias_w) {
#pragma unroll
                for (int i = 0; i < TMo; ++i) accb[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], ones, accb[i], 0, 0, 0);
            }
        }
    }
    wait_vm<0>();
    const size_t mn = (size_t)Co * 9 * Ci;
    float* dst = part + (size_t)bz * (mn + Co);
#pragma unroll
    for (int i = 0; i < TMo; ++i)
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
            const int co = CO * cot + 16 * i + 4 * (lane >> 4) + r4;
            if (bias_w && (lane & 15) == 0) dst[mn + co] = accb[i][r4];
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int tap = 3 * wv + d, ci = 32 * cic + 16 * j + (lane & 15);
                    dst[((size_t)co * 9 + tap) * Ci + ci] = acc[d][i][j][r4];
                }
        }
}

constexpr int kWtStages = 2;
hipError_t conv_wgrad(const Tensor& x, const Tensor& dz, float* part, int splits, int ksize,
                      hipStream_t s) {
    if (ksize != 3) return hipErrorInvalidValue;
    if (wgrad3_halo(x.H, x.W, x.C, dz.C)) {
        const int co = wgrad3_co(dz.C);
        const int tr = x.W % 64 == 0 ? 2 : 4, tw = x.W % 64 == 0 ? 64 : 32;
        const int T = x.B * (x.H / tr) * (x.W / tw);
        const int sp = wgrad3_parts(x.B, x.H, x.W, x.C, dz.C), tps = (T + sp - 1) / sp;
        dim3 g(dz.C / co, x.C / 32, sp);
        if (co == 32) {
            if (tw == 64) k_wgrad3<2, 64, 32><<<g, 192, 0, s>>>(dz, x, part, tps, T);
            else k_wgrad3<4, 32, 32><<<g, 192, 0, s>>>(dz, x, part, tps, T);
        } else {
            if (tw == 64) k_wgrad3<2, 64, 64><<<g, 192, 0, s>>>(dz, x, part, tps, T);
            else k_wgrad3<4, 32, 64><<<g, 192, 0, s>>>(dz, x, part, tps, T);
        }
        return hipGetLastError();
    }
    const int P = x.B * x.H * x.W;
    const int kps = wgrad_slab(P, splits);
    const int sp = wgrad_splits_used(P, splits);
    const int M = dz.C, N = 9 * x.C;
    if (M <= 32) {
        dim3 g(1, (N + 127) / 128, sp);
        k_wgrad_tr<32, kWtStages><<<g, 256, 0, s>>>(dz, x, part, P, kps);
    } else {
        dim3 g((M + 63) / 64, (N + 63) / 64, sp);
        k_wgrad_tr<64, kWtStages><<<g, 256, 0, s>>>(dz, x, part, P, kps);
    }
    return hipGetLastError();
}

hipError_t upconv_wgrad(const Tensor& x, const Tensor& g, float* part, int splits, hipStream_t s) {
    const int P = x.B * x.H * x.W;
    const int kps = wgrad_slab(P, splits);
    const int sp = wgrad_splits_used(P, splits);
    const int M = 4 * g.C, N = x.C;
    if (M <= 32) {
        dim3 gr(1, (N + 127) / 128, sp);
        k_wgrad_up<32><<<gr, 256, 0, s>>>(g, x, part, P, kps);
    } else {
        dim3 gr((M + 63) / 64, (N + 63) / 64, sp);
        k_wgrad_up<64><<<gr, 256, 0, s>>>(g, x, part, P, kps);
    }
    return hipGetLastError();
}

}  // namespace nn
}  // namespace eit
