// HIP kernels of one cost/gradient evaluation for gfx950:
//   transpose  -- x -> x^T (projector source for column-stepping angles) + ||x||^2 partials
//   project    -- Joseph ray-driven R for mu and delta in one pass (eq. 1), LDS-staged windows
//   ic         -- EI model, residual, FP64 cost partials and adjoint seeds (eq. 2/4, eq. 5)
//   cost       -- deterministic FP64 reduction of the partials (eq. 5)
//   backproject-- gather-form R^T (+ regulariser term of the gradient), LDS-staged windows
// Every kernel walks a list of work items (slice, a, b, c) with a grid-stride loop, so one
// launch can cover one slice or a batch of slices of different sizes.
#include <type_traits>

#include "device_common.h"

namespace eit {

// ------------------------------------------------------------------------ transpose
// Item (slice, tile_x, tile_y, -): 32x32 tile of both maps (map 0 alone when d.maps == 1)
// through LDS. Also writes the tile's sums of mu^2 and delta^2 (FP64) to part_reg[tile] for
// the regulariser.
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
        const int nm = d.maps == 1 ? 1 : 2;
        double s0 = 0.0, s1 = 0.0;
        for (int c = 0; c < nm; ++c) {
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
        for (int c = 0; c < nm; ++c) {
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
// in LDS, LP entries per row, and a sample interpolates between the neighbouring columns.
// Two LDS layouts (a tile-shape option):
//   DUP = 0: interleaved (mu, delta) pairs; a sample is two 8-byte LDS reads and applies the
//            weights 1 - ph and ph with four FMAs;
//   DUP = 1: 16-byte entries (mu, delta of column c, then the differences to column c + 1),
//            each column loaded twice; a sample is one aligned 16-byte read, an add and an
//            FMA per map (x_c + ph (x_{c+1} - x_c)), staging loads twice as much.
// The next strip's window is loaded into registers (buffer loads: rows past the map read as
// zero) while the current one is consumed.
//
// Index safety: every LDS index is ioff + (int)u (+1) with u in [1 - 1e-5, win_w - ioff - 1)
// for all rays of the block; the host builds lo and win_w from FP64 extremes with a 1e-3
// margin, and the host tests replay this exact FP32/FP64 arithmetic for every work item of
// the benchmark and test geometries.
// Interleaved 16-row variants are held to 80 VGPRs (six wavefronts per SIMD, three 512-thread
// blocks per CU); unconstrained they take 84 and only two blocks fit.
// MP = 1 projects map 0 alone (h-mode): entries hold one map (x_c, or x_c and x_{c+1} - x_c),
// a sample is one FMA pair fewer, and only plane 0 of P is written.
template <int A, int W, int R, int PW, int DUP, int LP, int IL, int MP>
__global__ __launch_bounds__(A* W) __attribute__((amdgpu_waves_per_eu(IL && R >= 16 ? 6 : 1)))
void k_project(const SliceDesc* __restrict__ D,
                                                  const Item* __restrict__ items, int n_items) {
    constexpr int NT = A * W;
    static_assert(W % 64 == 0, "one angle per whole wavefront");
    static_assert(NT % PW == 0 || PW % NT == 0, "staging must tile the block");
    // staging map: slot q of thread tid holds (row, column) of the strip window
    constexpr bool WIDE = NT >= PW;          // whole rows per slot step, else columns per slot
    constexpr int RS = WIDE ? NT / PW : 1;   // rows staged per slot step
    constexpr int CS = WIDE ? 1 : PW / NT;   // columns per thread and row
    static_assert(R % RS == 0, "strip must tile the block");
    static_assert(LP <= PW, "LDS rows hold at most the staged width");
    constexpr int SLOTS = R / RS * CS;
    static_assert(MP == 1 || MP == 2, "one or two maps");
    typedef typename std::conditional<MP == 2, typename std::conditional<DUP != 0, float4, float2>::type,
                                      typename std::conditional<DUP != 0, float2, float>::type>::type Entry;
    // LDS rows of LP entries (LP <= PW; window columns past LP are never staged or read)
    __shared__ Entry win[R * LP];
    const int tid = threadIdx.x;
    // ray of this thread: angle slot al, detector kl of the block
    //   IL = 0: a wavefront follows 64 consecutive detectors of one angle;
    //   IL = 1: a wavefront follows 8 consecutive detectors of 8 angles, each 16-lane group
    //           two angles x 8 detectors. LDS serves a 16-byte read 16 lanes at a time; 16
    //           rays of one angle reach over 16 / |cos| > 16 entries, so their entries meet
    //           in a bank, while two neighbouring angles over 8 detectors stay within ~15.
    static_assert(!IL || (A % 8 == 0 && W % 8 == 0), "interleaved rays need 8-angle groups");
    int al, kl;
    if constexpr (IL != 0) {
        constexpr int DO = W / 8;                // detector octets per angle
        const int wv = tid >> 6, lane = tid & 63;
        al = 8 * (wv / DO) + (lane >> 3);
        kl = 8 * (wv % DO) + (lane & 7);
    } else {
        al = __builtin_amdgcn_readfirstlane(tid / W);   // uniform per wavefront
        kl = tid % W;
    }
    const int sc = tid % PW, sr = tid / PW;  // staging column and first row of this thread
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped(d)) continue;
        const int n = d.n, grp = w.y, dblk = w.z;
        const int a0 = cld(d.groups + grp * A);
        int a;
        double inv, base, slope;
        float slope_f, wstep;
        if constexpr (IL != 0) {                 // angle differs across the wavefront
            a = d.groups[grp * A + al];
            const ProjAngle* pp = d.pang + (a >= 0 ? a : a0);
            inv = pp->inv; base = pp->base; slope = pp->slope;
            slope_f = pp->slope_f; wstep = pp->w;
        } else {
            a = cld(d.groups + grp * A + al);
            const ProjAngle* pp = d.pang + (a >= 0 ? a : a0);
            inv = cld(&pp->inv); base = cld(&pp->base); slope = cld(&pp->slope);
            slope_f = cld(&pp->slope_f); wstep = cld(&pp->w);
        }
        const int src = cld(&d.pang[a0].src);
        const int k = dblk * W + kl;
        const int k_eff = k < d.n_det ? k : d.n_det - 1;
        const double t = (double)k_eff - 0.5 * (double)(d.n_det - 1);
        const double ut0 = fma(t, inv, base);
        const float* map = src ? d.xT : d.x;
        const int nn4 = n * n * 4;
        const __amdgpu_buffer_rsrc_t bm = make_rsrc(map, nn4);
        const __amdgpu_buffer_rsrc_t bd = make_rsrc(map + (size_t)n * n, nn4);
        const int32_t* lo_tab = d.win_lo + ((size_t)grp * d.n_dblk + dblk) * d.n_strips;
        const int win_w = d.win_w, ns = d.n_strips;
        const int rstep4 = RS * n * 4;

        // DUP: entry c needs columns c and c + 1, both loaded (a window column past win_w - 1
        // or outside the map reads as zero; entry win_w - 1's second half is never used)
        Entry buf[SLOTS];
        auto load_pair = [&](int q, int vo, int vo1) {
            if constexpr (MP == 1) {
                if constexpr (DUP != 0) buf[q] = make_float2(buf_ld(bm, vo), buf_ld(bm, vo1));
                else buf[q] = buf_ld(bm, vo);
            } else if constexpr (DUP != 0) {
                buf[q] = make_float4(buf_ld(bm, vo), buf_ld(bd, vo), buf_ld(bm, vo1), buf_ld(bd, vo1));
            } else {
                buf[q] = make_float2(buf_ld(bm, vo), buf_ld(bd, vo));
            }
        };
        // (WIDE staging) a wavefront whose first staged column lies past the window skips its
        // loads and LDS writes: entries at or past win_w are never read
        const int c0w = __builtin_amdgcn_readfirstlane(sc);
        auto load_strip = [&](int s) {
            const int lo = cld(lo_tab + s);
            if constexpr (WIDE) {
                if (c0w >= win_w) return;
                const int col = lo + sc;
                const bool ok = sc < win_w && (unsigned)col < (unsigned)n;
                const bool ok1 = DUP != 0 && sc + 1 < win_w && (unsigned)(col + 1) < (unsigned)n;
                int vo = ok ? ((s * R + sr) * n + col) * 4 : kBufOOB;
                int vo1 = ok1 ? ((s * R + sr) * n + col + 1) * 4 : kBufOOB;   // col may be -1
#pragma unroll
                for (int q = 0; q < SLOTS; ++q) {
                    load_pair(q, vo, vo1);
                    vo += ok ? rstep4 : 0;
                    vo1 += ok1 ? rstep4 : 0;
                }
            } else {
#pragma unroll
                for (int q = 0; q < SLOTS; ++q) {
                    const int c = tid + (q % CS) * NT, col = lo + c;
                    const bool ok = c < win_w && (unsigned)col < (unsigned)n;
                    const bool ok1 = DUP != 0 && c + 1 < win_w && (unsigned)(col + 1) < (unsigned)n;
                    const int vo = ok ? ((s * R + q / CS) * n + col) * 4 : kBufOOB;
                    load_pair(q, vo, ok1 ? ((s * R + q / CS) * n + col + 1) * 4 : kBufOOB);
                }
            }
        };
        load_strip(0);
        double acc_m = 0.0, acc_d = 0.0;
        for (int s = 0; s < ns; ++s) {
            const int lo = cld(lo_tab + s);
            __syncthreads();                           // previous strip fully consumed
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) {
                Entry e = buf[q];
                if constexpr (DUP != 0 && MP == 2) {   // stored as (x_c, x_{c+1} - x_c) per map
                    e.z -= e.x;
                    e.w -= e.y;
                } else if constexpr (DUP != 0) {
                    e.y -= e.x;
                }
                if constexpr (WIDE) {
                    if (c0w < win_w && (LP == PW || sc < LP)) win[(sr + q * RS) * LP + sc] = e;
                } else {
                    const int c = tid + (q % CS) * NT;
                    if (LP == PW || c < LP) win[(q / CS) * LP + c] = e;
                }
            }
            __syncthreads();
            if (s + 1 < ns) load_strip(s + 1);         // in flight during this strip
            // Ray origin of the strip, split in FP64 into an integer window column (one
            // below the strip's lowest crossing) and a fraction, so the FP32 coordinate
            // u = uf + r*slope lies in [1, R + 1): truncation is the floor, and the
            // interpolation weight keeps ~2e-6 absolute precision.
            const double up0 = fma((double)(s * R), slope, ut0);
            const double fl0 = floor(up0 + fmin(0.0, (double)(R - 1) * slope)) - 1.0;
            const float uf = (float)(up0 - fl0);
            const Entry* rowp = win + ((int)fl0 - lo);
            float c0 = 0.f, c1 = 0.f;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float u = r == 0 ? uf : fmaf((float)r, slope_f, uf);
                const float ph = __builtin_amdgcn_fractf(u);
                const Entry* q = rowp + r * LP + (int)u;
                if constexpr (MP == 1 && DUP != 0) {
                    const float2 v = *(const float2*)q;
                    c0 = fmaf(ph, v.y, c0 + v.x);
                } else if constexpr (MP == 1) {
                    const float v0 = ((const float*)q)[0], v1 = ((const float*)q)[1];
                    c0 = fmaf(ph, v1, fmaf(1.f - ph, v0, c0));
                } else if constexpr (DUP != 0) {
                    // x_c + ph (x_{c+1} - x_c): the interpolation without a 1 - ph weight
                    const float4 v = *(const float4*)q;
                    c0 = fmaf(ph, v.z, c0 + v.x);
                    c1 = fmaf(ph, v.w, c1 + v.y);
                } else {
                    const float2 v0 = ((const float2*)q)[0], v1 = ((const float2*)q)[1];
                    const float om = 1.f - ph;
                    c0 = fmaf(ph, v1.x, fmaf(om, v0.x, c0));
                    c1 = fmaf(ph, v1.y, fmaf(om, v0.y, c1));
                }
            }
            acc_m += (double)c0;                  // strip sums combined in FP64
            acc_d += (double)c1;
        }
        if (a >= 0 && k < d.n_det) {
            d.P[(size_t)a * d.n_det + k] = (float)(wstep * acc_m);
            if constexpr (MP == 2) d.P[((size_t)d.n_theta + a) * d.n_det + k] = (float)(wstep * acc_d);
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
        // global-address-space views of the descriptor's (generic) pointers: global loads
        // and stores instead of flat ones
        typedef __attribute__((address_space(1))) float gf;
        typedef float f4v __attribute__((ext_vector_type(4)));
        typedef const __attribute__((address_space(1))) f4v gf4;
        gf* Pm = (gf*)(d.P + (size_t)a * nd);
        gf* Pd = (gf*)(d.P + ((size_t)d.n_theta + a) * nd);
        const gf* se = (const gf*)(d.s_exp + (size_t)a * M * nd);
        gf4* flat = (gf4*)d.flat;
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
            const f4v fl = flat[k];            // A, c, 1/(2 s^2), 1/s^2
            const double z = (double)fl.z, fw = (double)fl.w;
            double sf = 0.0, sfp = 0.0;
            float s_nx = se[k];                // the next mask position's signal is loaded
            for (int j = 0; j < M; ++j) {      // while the current one is evaluated
                const float s_j = s_nx;
                if (j + 1 < M) s_nx = se[(size_t)(j + 1) * nd + k];
                const double uu = d.mask[j] - dl - (double)fl.y;
                const double f = (double)fl.x * exp(-uu * uu * z);
                const double r = fma(T, f, -(double)s_j);
                r2 = fma(r, r, r2);
                sf = fma(r, f, sf);
                sfp = fma(r, -uu * fw * f, sfp);
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
// Item (slice, tile_x, tile_y, -). A TX x TY voxel tile; thread (il, jl) owns VPT voxels of
// column il (rows jl + q TY/VPT). For each chunk of AC angles the block stages, per angle, the
// kwin detector bins the tile can reach (starting at lo = floor(min over the tile of u) - 1,
// FP64) in LDS, premultiplied by the angle's 1/w, as 16-byte entries (G_mu, G_delta of bin
// c, G_mu, G_delta of bin c + 1) -- each bin stored twice so that a voxel's two bins are one
// aligned 16-byte LDS read -- plus the angle's FP32 constants; a voxel then applies the
// Joseph triangle weights. With the 1/w factor staged, each weight
// (1/w) max(0, 1 - d/w) is one FMA whose result the hardware clamps to [0, 1]:
//   bin floor(u):     max(0, 1 - f/w),   bin floor(u)+1:   max(0, (1 - 1/w) + f/w)
// (f = frac(u); neither exceeds 1 since f in [0, 1) and 1/w >= 1).
// Each voxel's sum is accumulated in a fixed angle order by one thread, chunk sums in FP64.
// The next chunk's bins are loaded into registers during the current chunk.
// Angle split (item .w = part g of d.adj_splits = G): with G > 1 the chunks of a tile are
// divided into G contiguous ranges, one block each, so that small maps still launch enough
// blocks. Each block then stores its FP64 partial sums as plane g of d.bp_part, and a later
// pass (k_bp_combine, or the optimiser's update) adds the G planes in the order g = 0 .. G-1
// before the regulariser term and the FP32 rounding -- the same arithmetic as the unsplit
// epilogue, with no inter-block synchronisation inside the launch.
constexpr int isqrt_ceil(int v) {
    int s = 0;
    while (s * s < v) ++s;
    return s;
}
constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }
// Window bound for a TX x TY tile: (TX-1)|cos| + (TY-1)|sin| <= sqrt((TX-1)^2 + (TY-1)^2),
// plus 4 bins of margin.
template <int TX, int TY>
constexpr int adj_pitch_max() {
    return pow2_at_least(isqrt_ceil((TX - 1) * (TX - 1) + (TY - 1) * (TY - 1)) + 4);
}

// Voxel (il, jl) of thread tid in a TX-wide tile. With TX = 32 a wavefront covers a 16 x 4
// patch (two wavefronts side by side) rather than two 32-voxel rows: the tile keeps its
// staging cost per voxel, and the bin reads of a wavefront stay as spread out as those of a
// 16-wide tile, which causes no LDS bank conflicts (the 32-wide rows did).
template <int TX>
__device__ __forceinline__ void adj_voxel(int tid, int& il, int& jl) {
    if constexpr (TX == 32) {   // the block has an even number of wavefronts (TY / VPT % 4 == 0)
        const int w = tid >> 6, l = tid & 63;
        il = (l & 15) + 16 * (w & 1);
        jl = (l >> 4) + 4 * (w >> 1);
    } else {
        il = tid % TX;
        jl = tid / TX;
    }
}

struct TileWin { int lo; float off; };
__device__ __forceinline__ TileWin tile_window_cs(double cs, double sn, double cd, int i0, int j0,
                                                  int TX, int TY) {
    const double uc = fma((double)j0, sn, fma((double)i0, cs, cd));
    const double umin = uc + fmin(0.0, (TX - 1) * cs) + fmin(0.0, (TY - 1) * sn);
    const int lo = (int)floor(umin) - 1;
    return TileWin{lo, (float)(uc - (double)lo)};
}
__device__ __forceinline__ TileWin tile_window(const AdjAngle* q, int i0, int j0, int TX, int TY) {
    return tile_window_cs(cld(&q->cs), cld(&q->sn), cld(&q->cd), i0, j0, TX, TY);
}

// Index safety: a voxel's coordinate relative to the window is u >= 1 - 1e-5 (lo is one bin
// below the tile's lowest crossing) and floor(u) + 1 <= kwin - 1 (kwin bounds the tile's
// span plus margin); the host tests replay this arithmetic for every tile and angle.
// MP = 1 backprojects seed plane 0 alone into gradient plane 0 (h-mode: the summed seeds);
// the staged entries are then (G of bin c, G of bin c + 1).
template <int TX, int TY, int AC, int VPT, int MP>
__global__ __launch_bounds__(TX* TY / VPT) void k_backproject(const SliceDesc* __restrict__ D,
                                                              const Item* __restrict__ items,
                                                              int n_items, int add_reg) {
    constexpr int NT = TX * TY / VPT;
    constexpr int PK = adj_pitch_max<TX, TY>();
    static_assert(NT % PK == 0, "staging must tile the block");
    static_assert(64 % PK == 0, "a staged angle row must not straddle wavefronts");
    constexpr int AS = NT / PK;              // angles staged per slot step
    static_assert(AC % AS == 0, "chunk must tile the block");
    constexpr int SLOTS = AC / AS;
    constexpr int JS = TY / VPT;
    static_assert(TX != 32 || JS % 4 == 0, "16 x 4 wavefront patches");
    static_assert(MP == 1 || MP == 2, "one or two maps");
    typedef typename std::conditional<MP == 2, float4, float2>::type GEntry;
    typedef typename std::conditional<MP == 2, float2, float>::type GLoad;
    __shared__ GEntry gw[AC * PK];
    __shared__ float4 rec[2][AC];            // cs, sn, offset, 1/w   (double-buffered by chunk)
    __shared__ float rec2[2][AC];            // 1 - 1/w
    __shared__ int los[2][AC];
    const int tid = threadIdx.x;
    int il, jl;
    adj_voxel<TX>(tid, il, jl);
    const int sb = tid % PK, sa = tid / PK;  // staging bin and first angle of this thread
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped_adj(d)) continue;
        const int n = d.n, nd = d.n_det, nth = d.n_theta;
        const int kwin = d.kwin;
        const int i0 = w.y * TX, j0 = w.z * TY;
        const int sz4 = nth * nd * 4;
        const __amdgpu_buffer_rsrc_t bGm = make_rsrc(d.P, sz4);
        const __amdgpu_buffer_rsrc_t bGd = make_rsrc(d.P + (size_t)nth * nd, sz4);
        const AdjAngle* aang = d.aang;
        const int nchunks = (nth + AC - 1) / AC;
        const int G = d.adj_splits, gs = w.w;
        const int ch0 = gs * nchunks / G, ch1 = (gs + 1) * nchunks / G;

        // per-angle constants and window origin of chunk ch into buffer slot ch & 1
        auto angle_setup = [&](int ch) {
            if (tid < AC) {
                const int a = ch * AC + tid;
                // padding angle: 1/w = 0 zeroes its staged bins
                float4 r1 = make_float4(0.f, 0.f, 1.f, 0.f);
                float r2 = 0.f;
                int lo = -(1 << 20);
                if (a < nth) {
                    const AdjAngle* q = aang + a;
                    const TileWin tw = tile_window(q, i0, j0, TX, TY);
                    r1 = make_float4(cld(&q->cs_f), cld(&q->sn_f), tw.off, cld(&q->iw));
                    r2 = cld(&q->omw);
                    lo = tw.lo;
                }
                rec[ch & 1][tid] = r1;
                rec2[ch & 1][tid] = r2;
                los[ch & 1][tid] = lo;
            }
        };
        GLoad buf[SLOTS];
        auto load_chunk = [&](int ch) {
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) {
                const int aa = sa + q * AS;
                const int a = ch * AC + aa;
                const int k = los[ch & 1][aa] + sb;
                const bool ok = a < nth && sb < kwin && (unsigned)k < (unsigned)nd;
                const int vo = ok ? (a * nd + k) * 4 : kBufOOB;
                if constexpr (MP == 2) buf[q] = make_float2(buf_ld(bGm, vo), buf_ld(bGd, vo));
                else buf[q] = buf_ld(bGm, vo);
            }
        };
        __syncthreads();                  // LDS of the previous work item fully consumed
        angle_setup(ch0);
        __syncthreads();
        load_chunk(ch0);
        double acc_m[VPT], acc_d[VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q) { acc_m[q] = 0.0; acc_d[q] = 0.0; }
        const float fil = (float)il, fjl = (float)jl;
        for (int ch = ch0; ch < ch1; ++ch) {
            __syncthreads();                           // previous chunk fully consumed
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) {
                // bin sb + 1 of the same angle is held by the next lane (PK divides 64)
                const float iw = rec[ch & 1][sa + q * AS].w;
                if constexpr (MP == 2) {
                    const float gm = iw * buf[q].x, gd = iw * buf[q].y;
                    float nm = __shfl_down(gm, 1), nd1 = __shfl_down(gd, 1);
                    if (sb == PK - 1) { nm = 0.f; nd1 = 0.f; }   // bin PK is never read
                    gw[(sa + q * AS) * PK + sb] = make_float4(gm, gd, nm, nd1);
                } else {
                    const float gm = iw * buf[q];
                    float nm = __shfl_down(gm, 1);
                    if (sb == PK - 1) nm = 0.f;
                    gw[(sa + q * AS) * PK + sb] = make_float2(gm, nm);
                }
            }
            if (ch + 1 < ch1) angle_setup(ch + 1);
            __syncthreads();
            if (ch + 1 < ch1) load_chunk(ch + 1);      // in flight during this chunk
            const int cb = ch & 1;
            float am[VPT], ad[VPT];
#pragma unroll
            for (int q = 0; q < VPT; ++q) { am[q] = 0.f; ad[q] = 0.f; }
#pragma unroll 4
            for (int aa = 0; aa < AC; ++aa) {
                const float4 r1 = rec[cb][aa];
                const float omw = rec2[cb][aa];
                const float u0 = fmaf(fil, r1.x, fmaf(fjl, r1.y, r1.z));
                const GEntry* row = gw + aa * PK;
                // all of the thread's bin reads for this angle are issued before any is used
                GEntry g[VPT];
                float f[VPT];
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    const float u = q == 0 ? u0 : fmaf((float)(q * JS), r1.y, u0);
                    f[q] = __builtin_amdgcn_fractf(u);
                    g[q] = row[(int)u];
                }
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    const float w0 = __builtin_amdgcn_fmed3f(fmaf(-f[q], r1.w, 1.f), 0.f, 1.f);
                    const float w1 = __builtin_amdgcn_fmed3f(fmaf(f[q], r1.w, omw), 0.f, 1.f);
                    if constexpr (MP == 2) {
                        am[q] = fmaf(w0, g[q].x, fmaf(w1, g[q].z, am[q]));
                        ad[q] = fmaf(w0, g[q].y, fmaf(w1, g[q].w, ad[q]));
                    } else {
                        am[q] = fmaf(w0, g[q].x, fmaf(w1, g[q].y, am[q]));
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < VPT; ++q) {        // chunk sums combined in FP64
                acc_m[q] += (double)am[q];
                acc_d[q] += (double)ad[q];
            }
        }
        const int i = i0 + il;
        if (G > 1) {
            const size_t nn = (size_t)n * n;
            double* part = d.bp_part + (size_t)gs * MP * nn;
#pragma unroll
            for (int q = 0; q < VPT; ++q) {
                const int j = j0 + jl + q * JS;
                if (i < n && j < n) {
                    part[(size_t)j * n + i] = acc_m[q];
                    if constexpr (MP == 2) part[nn + (size_t)j * n + i] = acc_d[q];
                }
            }
            continue;
        }
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int j = j0 + jl + q * JS;
            if (i < n && j < n) {
                const size_t o = (size_t)j * n + i;
                const size_t o2 = o + (size_t)n * n;
                double vm = acc_m[q], vd = acc_d[q];
                if (add_reg) {
                    vm = fma(d.reg_mu, (double)d.x[o], vm);
                    if constexpr (MP == 2) vd = fma(d.reg_de, (double)d.x[o2], vd);
                }
                d.g[o] = (float)vm;
                if constexpr (MP == 2) d.g[o2] = (float)vd;
            }
        }
    }
}

// ------------------------------------------------------------------------ mirror-pair adjoint
// Same operator as k_backproject, with each voxel paired with its row mirror and each angle
// with its mirror angle. With u = i cs + j sn + cd the detector coordinate of voxel v = (i, j)
// at angle theta, and u_s = -i cs + j sn + cd_s that of v at pi - theta (cos -> -cos), the
// voxel v' = (i, n-1-j) projects to n_det-1-u at pi - theta and to n_det-1-u_s at theta: four
// voxel-angle pairs from two coordinates. A reflected coordinate n_det-1-u has its two bins at
// fractional distances f and 1 - f from bins n_det-1-floor(u) and n_det-2-floor(u), so staging
// those bins in descending order gives the same entry index and weights as the direct read.
// Per pair slot (angle a, mirror b or -1) the block stages four windows, each kwin bins:
//   W0: bins of a around u (ascending)    -> v at a      W1: bins of b, reflected at u -> v' at b
//   W2: bins of b around u_s (ascending)  -> v at b      W3: bins of a, reflected at u_s -> v' at a
// An angle without a mirror in the set (b = -1) stages zeros in W1 and W2: it still reaches v
// and v' through W0 and W3. Item (slice, tile_x, tile_y, part): the tile's rows j lie in the
// top half; a thread writes v when 2j <= n-1 and v' = (i, n-1-j) when 2j < n-1, so every voxel
// (the middle row of an odd map included) is written once. Summation order: per voxel, the
// pairs in order, a before b, FP32 within a chunk of AC pairs, chunk sums in FP64. MP = 1:
// seed plane 0 alone into gradient plane 0, as in k_backproject.
template <int TX, int TY, int AC, int VPT, int MP>
__global__ __launch_bounds__(TX* TY / VPT) void k_backproject_pair(const SliceDesc* __restrict__ D,
                                                                   const Item* __restrict__ items,
                                                                   int n_items, int add_reg) {
    constexpr int NT = TX * TY / VPT;
    constexpr int PK = adj_pitch_max<TX, TY>();
    static_assert(NT % PK == 0, "staging must tile the block");
    static_assert(64 % PK == 0, "a staged window row must not straddle wavefronts");
    constexpr int NR = 4 * AC;               // window rows per chunk
    constexpr int AS = NT / PK;              // window rows staged per slot step
    static_assert(NR % AS == 0, "chunk must tile the block");
    constexpr int SLOTS = NR / AS;
    constexpr int JS = TY / VPT;
    static_assert(TX != 32 || JS % 4 == 0, "16 x 4 wavefront patches");
    static_assert(MP == 1 || MP == 2, "one or two maps");
    typedef typename std::conditional<MP == 2, float4, float2>::type GEntry;
    typedef typename std::conditional<MP == 2, float2, float>::type GLoad;
    __shared__ GEntry gw[NR * PK];
    __shared__ float4 rec[2][AC];            // cs, sn, offset of u, 1/w   (double-buffered)
    __shared__ float2 rec2[2][AC];           // offset of u_s, 1 - 1/w
    __shared__ int4 wins[2][AC];             // a, b, window origin for u, for u_s
    const int tid = threadIdx.x;
    int il, jl;
    adj_voxel<TX>(tid, il, jl);
    const int sb = tid % PK, sr = tid / PK;  // staging bin and first window row of this thread
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped_adj(d)) continue;
        const int n = d.n, nd = d.n_det, nth = d.n_theta, npair = d.n_pairs;
        const int kwin = d.kwin;
        const int i0 = w.y * TX, j0 = w.z * TY;
        const int sz4 = nth * nd * 4;
        const __amdgpu_buffer_rsrc_t bGm = make_rsrc(d.P, sz4);
        const __amdgpu_buffer_rsrc_t bGd = make_rsrc(d.P + (size_t)nth * nd, sz4);
        const int nchunks = (npair + AC - 1) / AC;
        const int G = d.adj_splits, gs = w.w;
        const int ch0 = gs * nchunks / G, ch1 = (gs + 1) * nchunks / G;

        auto pair_setup = [&](int ch) {
            if (tid < AC) {
                const int pi = ch * AC + tid;
                // padding slot: no angle, every window stages zeros
                float4 r1 = make_float4(0.f, 0.f, 1.f, 0.f);
                float2 r2 = make_float2(1.f, 0.f);
                int4 wv = make_int4(-1, -1, 0, 0);
                if (pi < npair) {
                    const int2 pr = d.apairs[pi];
                    const AdjAngle* q = d.aang + pr.x;
                    const double cs = cld(&q->cs), sn = cld(&q->sn);
                    const TileWin tu = tile_window_cs(cs, sn, cld(&q->cd), i0, j0, TX, TY);
                    const TileWin ts = tile_window_cs(-cs, sn, cld(&q->cd_s), i0, j0, TX, TY);
                    r1 = make_float4(cld(&q->cs_f), cld(&q->sn_f), tu.off, cld(&q->iw));
                    r2 = make_float2(ts.off, cld(&q->omw));
                    wv = make_int4(pr.x, pr.y, tu.lo, ts.lo);
                }
                rec[ch & 1][tid] = r1;
                rec2[ch & 1][tid] = r2;
                wins[ch & 1][tid] = wv;
            }
        };
        GLoad buf[SLOTS];
        auto load_chunk = [&](int ch) {
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) {
                const int rr = sr + q * AS, wk = rr & 3;
                const int4 wv = wins[ch & 1][rr >> 2];
                const int ang = (wk == 0 || wk == 3) ? wv.x : wv.y;
                const int lo = wk < 2 ? wv.z : wv.w;
                const int k = (wk == 1 || wk == 3) ? nd - 1 - lo - sb : lo + sb;
                const bool ok = ang >= 0 && sb < kwin && (unsigned)k < (unsigned)nd;
                const int vo = ok ? (ang * nd + k) * 4 : kBufOOB;
                if constexpr (MP == 2) buf[q] = make_float2(buf_ld(bGm, vo), buf_ld(bGd, vo));
                else buf[q] = buf_ld(bGm, vo);
            }
        };
        __syncthreads();                  // LDS of the previous work item fully consumed
        pair_setup(ch0);
        __syncthreads();
        load_chunk(ch0);
        double acc_m[VPT], acc_d[VPT], mir_m[VPT], mir_d[VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q) { acc_m[q] = 0.0; acc_d[q] = 0.0; mir_m[q] = 0.0; mir_d[q] = 0.0; }
        const float fil = (float)il, fjl = (float)jl;
        for (int ch = ch0; ch < ch1; ++ch) {
            __syncthreads();                           // previous chunk fully consumed
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) {
                // the next bin of the same window row is held by the next lane (PK divides 64)
                const int rr = sr + q * AS;
                const float iw = rec[ch & 1][rr >> 2].w;
                if constexpr (MP == 2) {
                    const float gm = iw * buf[q].x, gd = iw * buf[q].y;
                    float nm = __shfl_down(gm, 1), nd1 = __shfl_down(gd, 1);
                    if (sb == PK - 1) { nm = 0.f; nd1 = 0.f; }   // bin PK is never read
                    gw[rr * PK + sb] = make_float4(gm, gd, nm, nd1);
                } else {
                    const float gm = iw * buf[q];
                    float nm = __shfl_down(gm, 1);
                    if (sb == PK - 1) nm = 0.f;
                    gw[rr * PK + sb] = make_float2(gm, nm);
                }
            }
            if (ch + 1 < ch1) pair_setup(ch + 1);
            __syncthreads();
            if (ch + 1 < ch1) load_chunk(ch + 1);      // in flight during this chunk
            const int cb = ch & 1;
            float am[VPT], ad[VPT], bm[VPT], bd[VPT];
#pragma unroll
            for (int q = 0; q < VPT; ++q) { am[q] = 0.f; ad[q] = 0.f; bm[q] = 0.f; bd[q] = 0.f; }
#pragma unroll 2
            for (int pp = 0; pp < AC; ++pp) {
                const float4 r1 = rec[cb][pp];
                const float2 r2 = rec2[cb][pp];
                const float uu0 = fmaf(fil, r1.x, fmaf(fjl, r1.y, r1.z));
                const float us0 = fmaf(fil, -r1.x, fmaf(fjl, r1.y, r2.x));
                const GEntry* row = gw + pp * 4 * PK;
                GEntry g0[VPT], g1[VPT], g2[VPT], g3[VPT];
                float fu[VPT], fs[VPT];
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    const float uu = q == 0 ? uu0 : fmaf((float)(q * JS), r1.y, uu0);
                    const float us = q == 0 ? us0 : fmaf((float)(q * JS), r1.y, us0);
                    fu[q] = __builtin_amdgcn_fractf(uu);
                    fs[q] = __builtin_amdgcn_fractf(us);
                    const int ku = (int)uu, ks = (int)us;
                    g0[q] = row[ku];
                    g1[q] = row[PK + ku];
                    g2[q] = row[2 * PK + ks];
                    g3[q] = row[3 * PK + ks];
                }
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    const float u0 = __builtin_amdgcn_fmed3f(fmaf(-fu[q], r1.w, 1.f), 0.f, 1.f);
                    const float u1 = __builtin_amdgcn_fmed3f(fmaf(fu[q], r1.w, r2.y), 0.f, 1.f);
                    const float s0 = __builtin_amdgcn_fmed3f(fmaf(-fs[q], r1.w, 1.f), 0.f, 1.f);
                    const float s1 = __builtin_amdgcn_fmed3f(fmaf(fs[q], r1.w, r2.y), 0.f, 1.f);
                    if constexpr (MP == 2) {
                        am[q] = fmaf(u0, g0[q].x, fmaf(u1, g0[q].z, am[q]));
                        ad[q] = fmaf(u0, g0[q].y, fmaf(u1, g0[q].w, ad[q]));
                        bm[q] = fmaf(u0, g1[q].x, fmaf(u1, g1[q].z, bm[q]));
                        bd[q] = fmaf(u0, g1[q].y, fmaf(u1, g1[q].w, bd[q]));
                        am[q] = fmaf(s0, g2[q].x, fmaf(s1, g2[q].z, am[q]));
                        ad[q] = fmaf(s0, g2[q].y, fmaf(s1, g2[q].w, ad[q]));
                        bm[q] = fmaf(s0, g3[q].x, fmaf(s1, g3[q].z, bm[q]));
                        bd[q] = fmaf(s0, g3[q].y, fmaf(s1, g3[q].w, bd[q]));
                    } else {
                        am[q] = fmaf(u0, g0[q].x, fmaf(u1, g0[q].y, am[q]));
                        bm[q] = fmaf(u0, g1[q].x, fmaf(u1, g1[q].y, bm[q]));
                        am[q] = fmaf(s0, g2[q].x, fmaf(s1, g2[q].y, am[q]));
                        bm[q] = fmaf(s0, g3[q].x, fmaf(s1, g3[q].y, bm[q]));
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < VPT; ++q) {        // chunk sums combined in FP64
                acc_m[q] += (double)am[q];
                acc_d[q] += (double)ad[q];
                mir_m[q] += (double)bm[q];
                mir_d[q] += (double)bd[q];
            }
        }
        const int i = i0 + il;
        const size_t nn = (size_t)n * n;
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int j = j0 + jl + q * JS, jm = n - 1 - j;
            const bool wr = i < n && 2 * j <= n - 1;
            const bool wrm = i < n && 2 * j < n - 1;
            const size_t o = (size_t)j * n + i, om = (size_t)jm * n + i;
            if (G > 1) {
                double* part = d.bp_part + (size_t)gs * MP * nn;
                if (wr) {
                    part[o] = acc_m[q];
                    if constexpr (MP == 2) part[nn + o] = acc_d[q];
                }
                if (wrm) {
                    part[om] = mir_m[q];
                    if constexpr (MP == 2) part[nn + om] = mir_d[q];
                }
                continue;
            }
            if (wr) {
                double vm = acc_m[q], vd = acc_d[q];
                if (add_reg) {
                    vm = fma(d.reg_mu, (double)d.x[o], vm);
                    if constexpr (MP == 2) vd = fma(d.reg_de, (double)d.x[nn + o], vd);
                }
                d.g[o] = (float)vm;
                if constexpr (MP == 2) d.g[nn + o] = (float)vd;
            }
            if (wrm) {
                double vm = mir_m[q], vd = mir_d[q];
                if (add_reg) {
                    vm = fma(d.reg_mu, (double)d.x[om], vm);
                    if constexpr (MP == 2) vd = fma(d.reg_de, (double)d.x[nn + om], vd);
                }
                d.g[om] = (float)vm;
                if constexpr (MP == 2) d.g[nn + om] = (float)vd;
            }
        }
    }
}

// ------------------------------------------------------------------------ registry
// Projector variants (A angles x W detectors threads, R rows per strip, PW staged entries per
// row, DUP = duplicated 16-byte entries).
#define EIT_PROJ_VARIANTS(X)        \
    X(0, 8, 64, 16, 256, 0, 256, 0)    \
    X(1, 4, 64, 16, 128, 0, 128, 0)    \
    X(2, 16, 64, 8, 256, 0, 256, 0)    \
    X(3, 8, 64, 8, 256, 0, 256, 0)     \
    X(4, 4, 128, 16, 256, 0, 256, 0)   \
    X(5, 8, 64, 32, 256, 0, 256, 0)    \
    X(6, 16, 64, 16, 256, 0, 256, 0)   \
    X(7, 2, 64, 16, 128, 0, 128, 0)    \
    X(8, 1, 64, 16, 128, 0, 128, 0)    \
    X(9, 16, 64, 16, 256, 1, 256, 0)   \
    X(10, 16, 64, 8, 256, 1, 256, 0)   \
    X(11, 8, 64, 8, 256, 1, 256, 0)    \
    X(12, 8, 64, 8, 128, 1, 128, 0)    \
    X(13, 8, 64, 16, 128, 1, 128, 0)   \
    X(14, 4, 64, 16, 128, 1, 128, 0)   \
    X(15, 4, 64, 8, 128, 1, 128, 0)    \
    X(16, 8, 64, 16, 256, 1, 136, 0)   \
    X(17, 8, 64, 8, 256, 1, 128, 0)     \
    X(18, 8, 64, 8, 256, 1, 128, 1)     \
    X(19, 8, 64, 16, 256, 1, 136, 1)    \
    X(20, 16, 64, 8, 256, 1, 256, 1)    \
    X(21, 8, 64, 8, 256, 1, 256, 1)     \
    X(22, 8, 64, 12, 256, 1, 128, 1)    \
    X(23, 8, 64, 12, 256, 1, 136, 1)    \
    X(24, 8, 64, 12, 128, 1, 128, 1)    \
    X(25, 8, 64, 16, 128, 1, 128, 1)

// Adjoint variants (TX x TY voxel tile, AC angles per chunk -- angle pairs with MIR = 1 --,
// VPT voxels per thread, MIR = 1: mirror-pair kernel).
#define EIT_ADJ_VARIANTS(X)    \
    X(0, 16, 16, 32, 1, 0)     \
    X(1, 16, 16, 32, 2, 0)     \
    X(2, 32, 16, 32, 2, 0)     \
    X(3, 32, 32, 32, 4, 0)     \
    X(4, 16, 32, 32, 2, 0)     \
    X(5, 16, 16, 64, 1, 0)     \
    X(6, 32, 32, 16, 4, 0)     \
    X(7, 32, 16, 32, 4, 0)     \
    X(8, 32, 32, 8, 2, 1)      \
    X(9, 16, 16, 8, 1, 1)      \
    X(10, 32, 16, 8, 2, 1)     \
    X(11, 16, 32, 8, 2, 1)     \
    X(12, 32, 32, 16, 2, 1)

int proj_variant_count() {
    int c = 0;
#define X(id, A, W, R, PW, DUP, LP, IL) ++c;
    EIT_PROJ_VARIANTS(X)
#undef X
    return c;
}
ProjTile proj_variant(int v) {
#define X(id, A, W, R, PW, DUP, LP, IL) \
    if (v == id) return ProjTile{A, W, R, PW, DUP, LP, IL};
    EIT_PROJ_VARIANTS(X)
#undef X
    return ProjTile{0, 0, 0, 0, 0, 0, 0};
}
int adj_pitch_limit(int v) {
#define X(id, TX, TY, AC, VPT, MIR) \
    if (v == id) return adj_pitch_max<TX, TY>();
    EIT_ADJ_VARIANTS(X)
#undef X
    return 0;
}
int adj_variant_count() {
    int c = 0;
#define X(id, TX, TY, AC, VPT, MIR) ++c;
    EIT_ADJ_VARIANTS(X)
#undef X
    return c;
}
AdjTile adj_variant(int v) {
#define X(id, TX, TY, AC, VPT, MIR) \
    if (v == id) return AdjTile{TX, TY, AC, VPT, MIR};
    EIT_ADJ_VARIANTS(X)
#undef X
    return AdjTile{0, 0, 0, 0, 0};
}

hipError_t launch_transpose(const SliceDesc* D, const Item* items, int n_items, int grid,
                            hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_transpose<<<grid, kTrThreads, 0, s>>>(D, items, n_items);
    return hipGetLastError();
}

hipError_t launch_project(int variant, int maps, const SliceDesc* D, const Item* items,
                          int n_items, int grid, size_t lds, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (maps != 1 && maps != 2) return hipErrorInvalidValue;
#define X(id, A, W, R, PW, DUP, LP, IL)                                                     \
    if (variant == id) {                                                                    \
        (void)lds;                                                                          \
        if (maps == 1)                                                                      \
            k_project<A, W, R, PW, DUP, LP, IL, 1><<<grid, A * W, 0, s>>>(D, items, n_items); \
        else                                                                                \
            k_project<A, W, R, PW, DUP, LP, IL, 2><<<grid, A * W, 0, s>>>(D, items, n_items); \
        return hipGetLastError();                                                           \
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

template <int TX, int TY, int AC, int VPT, int MIR, int MP>
void launch_adjoint_kernel(const SliceDesc* D, const Item* items, int n_items, int grid,
                           int add_reg, hipStream_t s) {
    if constexpr (MIR != 0)
        k_backproject_pair<TX, TY, AC, VPT, MP><<<grid, TX * TY / VPT, 0, s>>>(D, items, n_items, add_reg);
    else
        k_backproject<TX, TY, AC, VPT, MP><<<grid, TX * TY / VPT, 0, s>>>(D, items, n_items, add_reg);
}

hipError_t launch_backproject(int variant, int maps, const SliceDesc* D, const Item* items,
                              int n_items, int grid, int add_reg, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (maps != 1 && maps != 2) return hipErrorInvalidValue;
#define X(id, TX, TY, AC, VPT, MIR)                                                        \
    if (variant == id) {                                                                   \
        if (maps == 1) launch_adjoint_kernel<TX, TY, AC, VPT, MIR, 1>(D, items, n_items, grid, add_reg, s); \
        else launch_adjoint_kernel<TX, TY, AC, VPT, MIR, 2>(D, items, n_items, grid, add_reg, s);           \
        return hipGetLastError();                                                          \
    }
    EIT_ADJ_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

// Split adjoint epilogue. Item (slice, chunk): kVecChunk consecutive elements e of the
// [2][n][n] output; g[e] = FP32(sum over parts of bp_part[part][e] (+ reg * x[e])).
__global__ __launch_bounds__(kVecThreads) void k_bp_combine(const SliceDesc* __restrict__ D,
                                                           const Item* __restrict__ items,
                                                           int n_items, int add_reg) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped_adj(d) || d.adj_splits <= 1) continue;
        const int G = d.adj_splits;
        const size_t nn = (size_t)d.n * d.n, nv = 2 * nn;
        const size_t e0 = (size_t)w.y * kVecChunk;
        const size_t e1 = min(e0 + kVecChunk, nv);
        for (size_t e = e0 + threadIdx.x; e < e1; e += kVecThreads) {
            double v = 0.0;
            for (int g = 0; g < G; ++g) v += d.bp_part[g * nv + e];
            if (add_reg) v = fma(e < nn ? d.reg_mu : d.reg_de, (double)d.x[e], v);
            d.g[e] = (float)v;
        }
    }
}

hipError_t launch_bp_combine(const SliceDesc* D, const Item* items, int n_items, int grid,
                             int add_reg, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_bp_combine<<<grid, kVecThreads, 0, s>>>(D, items, n_items, add_reg);
    return hipGetLastError();
}

}  // namespace eit
