// HIP kernels of one cost/gradient evaluation for gfx950:
//   transpose  -- x -> x^T (projector source for column-stepping angles) + ||x||^2 partials
//   project    -- Joseph ray-driven R for mu and delta in one pass (eq. 1), LDS-staged windows
//   ic         -- EI model, residual, FP64 cost partials and adjoint seeds (eq. 2/4, eq. 5)
//   cost       -- deterministic FP64 reduction of the partials (eq. 5)
//   backproject-- gather-form R^T (+ regulariser term of the gradient), LDS-staged windows
// Every kernel walks a list of work items (slice, a, b, c) with a grid-stride loop, so one
// launch can cover one slice or a batch of slices of different sizes.
#include "eit_internal.h"
#include "reduce.h"

namespace eit {

__device__ __forceinline__ bool skipped(const SliceDesc& d) {
    return d.skip != nullptr && *d.skip != 0;
}
__device__ __forceinline__ bool skipped_adj(const SliceDesc& d) {
    return (d.skip != nullptr && *d.skip != 0) || (d.skip_adj != nullptr && *d.skip_adj != 0);
}

// ------------------------------------------------------------------------ transpose
// Item (slice, tile_x, tile_y, -): 32x32 tile of both maps through LDS. Also writes the
// tile's sums of mu^2 and delta^2 (FP64) to part_reg[tile] for the regulariser.
__global__ __launch_bounds__(kTrThreads) void k_transpose(const SliceDesc* __restrict__ D,
                                                         const Item* __restrict__ items,
                                                         int n_items) {
    __shared__ float tile[2][kTrTile][kTrTile + 1];
    __shared__ double red[kTrThreads / 64];
    const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // 32 x 8
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped(d)) continue;
        const int n = d.n, tx = w.y, ty = w.z;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float* src = d.x + (size_t)c * n * n;
            for (int r = ly; r < kTrTile; r += 8) {
                const int j = ty * kTrTile + r, i = tx * kTrTile + lx;
                float v = 0.f;
                if (j < n && i < n) v = src[(size_t)j * n + i];
                tile[c][r][lx] = v;
                if (c == 0) s0 = fma((double)v, (double)v, s0);
                else s1 = fma((double)v, (double)v, s1);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            float* dst = d.xT + (size_t)c * n * n;
            for (int r = ly; r < kTrTile; r += 8) {
                const int i = tx * kTrTile + r, j = ty * kTrTile + lx;
                if (i < n && j < n) dst[(size_t)i * n + j] = tile[c][lx][r];
            }
        }
        s0 = block_sum(s0, red);
        s1 = block_sum(s1, red);
        if (threadIdx.x == 0) {
            const int ntx = (n + kTrTile - 1) / kTrTile;
            double* p = d.part_reg + 2 * (size_t)(ty * ntx + tx);
            p[0] = s0;
            p[1] = s1;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ projector
// Item (slice, group, detector block, -). Thread (angle slot al, detector kl) follows one
// ray. The block walks the stepped axis in strips of R rows; for each strip it stages the
// window [lo, lo + win_w) of the interpolation axis (host-computed lo, conservative in FP64)
// as interleaved (mu, delta) pairs in LDS; each sample is then one 16-byte LDS read of the
// two neighbouring pairs and four FMAs.
template <int A, int W, int R>
__global__ __launch_bounds__(A* W) void k_project(const SliceDesc* __restrict__ D,
                                                  const Item* __restrict__ items, int n_items) {
    extern __shared__ float2 win[];   // [R][pitch]
    constexpr int NT = A * W;
    const int tid = threadIdx.x;
    const int al = tid / W, kl = tid % W;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped(d)) continue;
        const int n = d.n, grp = w.y, dblk = w.z;
        const int a = d.groups[grp * A + al];
        const int a0 = d.groups[grp * A];
        const ProjAngle pa = d.pang[a >= 0 ? a : a0];
        const int src = d.pang[a0].src;
        const int k = dblk * W + kl;
        const int k_eff = k < d.n_det ? k : d.n_det - 1;
        const double t = (double)k_eff - 0.5 * (double)(d.n_det - 1);
        const double ut0 = fma(t, pa.inv, pa.base);
        const float* sm = src ? d.xT : d.x;
        const float* sd = sm + (size_t)n * n;
        const int32_t* lo_tab = d.win_lo + ((size_t)grp * d.n_dblk + dblk) * d.n_strips;
        const int pshift = d.win_shift, pitch = 1 << pshift, win_w = d.win_w;
        double acc_m = 0.0, acc_d = 0.0;
        for (int s = 0; s < d.n_strips; ++s) {
            const int p0 = s * R;
            const int lo = lo_tab[s];
            __syncthreads();
            for (int e = tid; e < R * pitch; e += NT) {
                const int r = e >> pshift, c = e & (pitch - 1);
                if (c < win_w) {
                    const int row = p0 + r, col = lo + c;
                    float2 v = make_float2(0.f, 0.f);
                    if (row < n && col >= 0 && col < n) {
                        const size_t o = (size_t)row * n + col;
                        v.x = sm[o];
                        v.y = sd[o];
                    }
                    win[e] = v;
                }
            }
            __syncthreads();
            // Ray origin for this strip split into an integer window column and a fraction
            // in [0, 1) (FP64), so the FP32 interpolation coordinate stays below ~R in
            // magnitude and keeps ~1e-6 absolute precision.
            const double up0 = fma((double)p0, pa.slope, ut0);
            const double fl0 = floor(up0);
            const float uf = (float)(up0 - fl0);
            const int ioff = (int)fl0 - lo;                 // >= 1 by construction of lo
            const int imin = -ioff, imax = win_w - 2 - ioff;
            const float2* rowp = win + ioff;
            float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float u = fmaf((float)r, pa.slope_f, uf);
                const float fl = floorf(u);
                const float ph = u - fl;
                const int i = min(max((int)fl, imin), imax);
                const float2* q = rowp + i;
                rowp += pitch;
                const float2 v0 = q[0], v1 = q[1];
                const float om = 1.f - ph;
                c0 = fmaf(om, v0.x, c0);
                c1 = fmaf(om, v0.y, c1);
                c2 = fmaf(ph, v1.x, c2);
                c3 = fmaf(ph, v1.y, c3);
            }
            acc_m += (double)c0 + (double)c2;     // strip sums combined in FP64
            acc_d += (double)c1 + (double)c3;
        }
        if (a >= 0 && k < d.n_det) {
            d.P[(size_t)a * d.n_det + k] = (float)(pa.w * acc_m);
            d.P[((size_t)d.n_theta + a) * d.n_det + k] = (float)(pa.w * acc_d);
        }
    }
}

// ------------------------------------------------------------------------ IC model
// Item (slice, angle, -, -). For every detector pixel of the angle:
//   T = exp(-P_mu), Delta = kappa (P_de[k+1] - P_de[k-1]) / 2,
//   s_mod_j = T f_k(m_j - Delta), r_j = s_mod_j - s_exp_j,
//   cost partial sum r^2 (FP64), G_Pmu = -2 T sum r f, G_Delta = -2 T sum r f',
//   G_Pde = kappa D^T G_Delta = -kappa (G_Delta[k+1] - G_Delta[k-1]) / 2.
// P holds scale * R x on input (scale folded in here) and the seeds times scale on output
// (chain rule for scaled unknowns), overwritten in place.
constexpr int kMaxDetLds = 4096;
__global__ __launch_bounds__(kIcThreads) void k_ic(const SliceDesc* __restrict__ D,
                                                  const Item* __restrict__ items, int n_items,
                                                  int want_seeds) {
    __shared__ float gdl[kMaxDetLds];
    __shared__ double red[kIcThreads / 64];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped(d)) continue;
        const int a = w.y, nd = d.n_det, M = d.n_mask;
        float* Pm = d.P + (size_t)a * nd;
        float* Pd = d.P + ((size_t)d.n_theta + a) * nd;
        const float* se = d.s_exp + (size_t)a * M * nd;
        const double sm = d.scale_mu, sdl = d.scale_de;
        const float kap = d.kappa;
        double r2 = 0.0;
        for (int k = threadIdx.x; k < nd; k += kIcThreads) {
            // The residual is a small difference of O(1) numbers, so the model is evaluated
            // in FP64 from the FP32 projections.
            const double pm = sm * (double)Pm[k];
            const double pp = k + 1 < nd ? sdl * (double)Pd[k + 1] : 0.0;
            const double pn = k > 0 ? sdl * (double)Pd[k - 1] : 0.0;
            const double T = exp(-pm);
            const double dl = (double)kap * 0.5 * (pp - pn);
            const float4 fl = d.flat[k];       // A, c, 1/(2 s^2), 1/s^2
            double sf = 0.0, sfp = 0.0;
            for (int j = 0; j < M; ++j) {
                const double uu = (double)d.mask[j] - dl - (double)fl.y;
                const double f = (double)fl.x * exp(-uu * uu * (double)fl.z);
                const double r = fma(T, f, -(double)se[(size_t)j * nd + k]);
                r2 = fma(r, r, r2);
                sf = fma(r, f, sf);
                sfp = fma(r, -uu * (double)fl.w * f, sfp);
            }
            if (want_seeds) {
                Pm[k] = (float)(sm * (-2.0 * T * sf));   // G_Pmu, scaled
                gdl[k] = (float)(-2.0 * T * sfp);               // G_Delta
            }
        }
        __syncthreads();   // all reads of Pd done, gdl complete
        if (want_seeds) {
            for (int k = threadIdx.x; k < nd; k += kIcThreads) {
                const float gp = k + 1 < nd ? gdl[k + 1] : 0.f;
                const float gn = k > 0 ? gdl[k - 1] : 0.f;
                Pd[k] = (float)(sdl * (-(double)kap * 0.5 * ((double)gp - (double)gn)));
            }
        }
        r2 = block_sum(r2, red);
        if (threadIdx.x == 0) d.part_ic[a] = r2;
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ cost reduce
// One block per slice: S = sum_a part_ic[a] + lam_mu sum mu^2 + lam_de sum delta^2.
__global__ __launch_bounds__(256) void k_cost_reduce(const SliceDesc* __restrict__ D) {
    __shared__ double red[4];
    const SliceDesc& d = D[blockIdx.x];
    if (skipped(d)) return;
    double s = 0.0, r0 = 0.0, r1 = 0.0;
    for (int a = threadIdx.x; a < d.n_theta; a += 256) s += d.part_ic[a];
    for (int b = threadIdx.x; b < d.n_reg_blocks; b += 256) {
        r0 += d.part_reg[2 * b];
        r1 += d.part_reg[2 * b + 1];
    }
    s = block_sum(s, red);
    r0 = block_sum(r0, red);
    r1 = block_sum(r1, red);
    if (threadIdx.x == 0) d.cost[0] = s + d.lam_mu * r0 + d.lam_de * r1;
}

// ------------------------------------------------------------------------ adjoint
// Item (slice, tile_x, tile_y, -). Thread = voxel (il, jl) of a TX x TY tile. For each
// chunk of AC angles the block stages, per angle, the kwin detector bins the tile can
// reach (starting at lo = floor(min over the tile of u) - 1, computed in FP64) as
// interleaved (G_mu, G_delta) pairs in LDS; a voxel then reads its two bins with one
// 16-byte LDS read and applies the Joseph triangle weights. No atomics: each voxel's sum
// is accumulated in a fixed angle order by one thread.
constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }
// Upper bound of the window width for a TX x TY tile: the span (TX-1)|cos| + (TY-1)|sin|
// is at most TX + TY - 2, plus 4 bins of margin.
template <int TX, int TY>
constexpr int adj_pitch_max() { return pow2_at_least(TX + TY + 2); }

template <int TX, int TY, int AC>
__global__ __launch_bounds__(TX* TY) void k_backproject(const SliceDesc* __restrict__ D,
                                                        const Item* __restrict__ items,
                                                        int n_items, int add_reg) {
    __shared__ float2 gw[AC * adj_pitch_max<TX, TY>()];      // [AC][pitch]
    __shared__ float offs[AC];
    __shared__ int los[AC];
    constexpr int NT = TX * TY;
    const int tid = threadIdx.x;
    const int il = tid % TX, jl = tid / TX;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped_adj(d)) continue;
        const int n = d.n, nd = d.n_det, nth = d.n_theta;
        const int kwin = d.kwin;
        int pshift = 0;
        while ((1 << pshift) < kwin) ++pshift;
        const int pitch = 1 << pshift;
        const int i0 = w.y * TX, j0 = w.z * TY;
        const float* Gm = d.P;
        const float* Gd = d.P + (size_t)nth * nd;
        double acc_m = 0.0, acc_d = 0.0;
        const float fil = (float)il, fjl = (float)jl;
        for (int ab = 0; ab < nth; ab += AC) {
            const int na = min(AC, nth - ab);
            __syncthreads();
            if (tid < na) {
                const AdjAngle q = d.aang[ab + tid];
                const double uc = fma((double)j0, q.sn, fma((double)i0, q.cs, q.cd));
                const double umin = uc + fmin(0.0, (TX - 1) * q.cs) + fmin(0.0, (TY - 1) * q.sn);
                const int lo = (int)floor(umin) - 1;
                los[tid] = lo;
                offs[tid] = (float)(uc - (double)lo);
            }
            __syncthreads();
            for (int e = tid; e < AC * pitch; e += NT) {
                const int aa = e >> pshift, b = e & (pitch - 1);
                if (aa < na && b < kwin) {
                    const int k = los[aa] + b;
                    float2 v = make_float2(0.f, 0.f);
                    if (k >= 0 && k < nd) {
                        const size_t o = (size_t)(ab + aa) * nd + k;
                        v.x = Gm[o];
                        v.y = Gd[o];
                    }
                    gw[e] = v;
                }
            }
            __syncthreads();
            float am = 0.f, ad = 0.f;
            for (int aa = 0; aa < na; ++aa) {
                const AdjAngle q = d.aang[ab + aa];
                const float u = fmaf(fil, q.cs_f, fmaf(fjl, q.sn_f, offs[aa]));
                int b = (int)u;
                const float f = u - (float)b;
                b = min(max(b, 0), kwin - 2);
                const float w0 = fmaxf(0.f, fmaf(-f, q.iw2, q.iw));
                const float w1 = fmaxf(0.f, fmaf(f, q.iw2, q.iwm));
                const float2* p = gw + (aa << pshift) + b;
                const float2 g0 = p[0], g1 = p[1];
                am = fmaf(w0, g0.x, fmaf(w1, g1.x, am));
                ad = fmaf(w0, g0.y, fmaf(w1, g1.y, ad));
            }
            acc_m += (double)am;          // chunk sums combined in FP64
            acc_d += (double)ad;
        }
        const int i = i0 + il, j = j0 + jl;
        if (i < n && j < n) {
            const size_t o = (size_t)j * n + i;
            const size_t o2 = o + (size_t)n * n;
            if (add_reg) {
                acc_m = fma(d.reg_mu, (double)d.x[o], acc_m);
                acc_d = fma(d.reg_de, (double)d.x[o2], acc_d);
            }
            d.g[o] = (float)acc_m;
            d.g[o2] = (float)acc_d;
        }
    }
}

// ------------------------------------------------------------------------ registry
// Projector variants (A angles x W detectors threads, R rows per strip).
#define EIT_PROJ_VARIANTS(X) \
    X(0, 8, 64, 16)          \
    X(1, 4, 64, 16)          \
    X(2, 16, 64, 8)          \
    X(3, 8, 64, 8)           \
    X(4, 4, 128, 16)         \
    X(5, 2, 128, 32)

#define EIT_ADJ_VARIANTS(X) \
    X(0, 16, 16, 32)        \
    X(1, 32, 8, 32)         \
    X(2, 16, 16, 64)        \
    X(3, 32, 16, 32)        \
    X(4, 16, 32, 32)

int proj_variant_count() {
    int c = 0;
#define X(id, A, W, R) ++c;
    EIT_PROJ_VARIANTS(X)
#undef X
    return c;
}
ProjTile proj_variant(int v) {
#define X(id, A, W, R) \
    if (v == id) return ProjTile{A, W, R};
    EIT_PROJ_VARIANTS(X)
#undef X
    return ProjTile{0, 0, 0};
}
int adj_pitch_limit(int v) {
#define X(id, TX, TY, AC) \
    if (v == id) return adj_pitch_max<TX, TY>();
    EIT_ADJ_VARIANTS(X)
#undef X
    return 0;
}
int adj_variant_count() {
    int c = 0;
#define X(id, TX, TY, AC) ++c;
    EIT_ADJ_VARIANTS(X)
#undef X
    return c;
}
AdjTile adj_variant(int v) {
#define X(id, TX, TY, AC) \
    if (v == id) return AdjTile{TX, TY, AC};
    EIT_ADJ_VARIANTS(X)
#undef X
    return AdjTile{0, 0, 0};
}

hipError_t launch_transpose(const SliceDesc* D, const Item* items, int n_items, int grid,
                            hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_transpose<<<grid, kTrThreads, 0, s>>>(D, items, n_items);
    return hipGetLastError();
}

hipError_t launch_project(int variant, const SliceDesc* D, const Item* items, int n_items,
                          int grid, size_t lds, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
#define X(id, A, W, R)                                                           \
    if (variant == id) {                                                         \
        k_project<A, W, R><<<grid, A * W, lds, s>>>(D, items, n_items);          \
        return hipGetLastError();                                                \
    }
    EIT_PROJ_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_ic(const SliceDesc* D, const Item* items, int n_items, int grid, int want_seeds,
                     hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_ic<<<grid, kIcThreads, 0, s>>>(D, items, n_items, want_seeds);
    return hipGetLastError();
}

hipError_t launch_cost_reduce(const SliceDesc* D, int n_slices, hipStream_t s) {
    k_cost_reduce<<<n_slices, 256, 0, s>>>(D);
    return hipGetLastError();
}

hipError_t launch_backproject(int variant, const SliceDesc* D, const Item* items, int n_items,
                              int grid, int add_reg, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
#define X(id, TX, TY, AC)                                                              \
    if (variant == id) {                                                               \
        k_backproject<TX, TY, AC><<<grid, TX * TY, 0, s>>>(D, items, n_items, add_reg); \
        return hipGetLastError();                                                      \
    }
    EIT_ADJ_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace eit
