// Device-resident L-BFGS for the EI cost (the paper minimises eq. 5 with an L-BFGS
// method). Compact representation (Byrd, Nocedal & Schnabel): with H_0 = gamma I,
//   H g = gamma g + S e - gamma Y c,  c = R^{-1} (S^T g),
//   e = R^{-T} ((D + gamma Y^T Y) c - gamma Y^T g),
// R the upper triangle of S^T Y and D its diagonal -- algebraically the two-loop recursion,
// but every inner product of an iteration is gathered in one vector pass and the small
// m x m algebra runs in one thread. Inner products accumulate in FP64. The line search
// (Armijo backtracking) is a device-side state machine: each replay of the evaluation
// sequence either starts a new direction or halves the step, with no host round trip.
#include "solver_dev.h"

namespace eit {

// ------------------------------------------------------------------------ init / scale
__global__ void k_lb_init(const LbDesc* __restrict__ L, int m, int max_iter, int max_ls,
                          double c1, double tol) {
    if (threadIdx.x != 0) return;
    SolverState& s = *L[blockIdx.x].st;
    s.f = 0.0; s.f_t = 0.0; s.alpha = 0.0; s.gd = 0.0; s.gamma = 1.0; s.gg = 0.0;
    s.c1 = c1; s.tol = tol;
    for (int r = 0; r < kMaxM; ++r) { s.cc[r] = 0.0; s.ee[r] = 0.0; s.order[r] = 0; }
    s.cost_hist = L[blockIdx.x].cost_hist;
    s.k = 0; s.evals = 0; s.trials = 0; s.mode = MODE_INIT; s.status = ST_RUNNING;
    s.m_cur = 0; s.m = m; s.max_iter = max_iter; s.max_ls = max_ls; s.accept = 0;
    s.spare = 0; s.launches = 0; s.skip = 0; s.skip_adj = 0;
}

// to_z: z = x_user / scale; else x_user = z * scale.
__global__ __launch_bounds__(kVecThreads) void k_lb_scale(const LbDesc* __restrict__ L,
                                                        const Item* __restrict__ items,
                                                        int n_items, int to_z) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const LbDesc& l = L[w.x];
        const int64_t half = l.nv / 2;
        const int64_t e0 = (int64_t)w.y * kVecChunk;
        const int64_t e1 = min(e0 + kVecChunk, l.nv);
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kVecThreads) {
            const float sc = e < half ? l.scale_mu : l.scale_de;
            if (to_z) l.z[e] = l.x_user[e] / sc;
            else l.x_user[e] = l.z[e] * sc;
        }
    }
}

// ------------------------------------------------------------------------ direction + trial point
// Item (slice, tile_x, tile_y, -): a 32 x 32 tile of both maps.
// INIT: zt = z. NEW_DIR: d = -gamma g - sum ee_r s_r + sum cc_r y_r (FP64 accumulation: the
// combination has cancellation), zt = z + alpha d. BACKTRACK: zt = z + alpha d.
// The tile of zt is also written transposed (the projector's source for column-stepping
// angles) and its sums of squares go to the regulariser partials, replacing a separate
// transpose pass over the trial point.
__global__ __launch_bounds__(kTrThreads) void k_lb_direction(const LbDesc* __restrict__ L,
                                                            const SliceDesc* __restrict__ D,
                                                            const Item* __restrict__ items,
                                                            int n_items) {
    __shared__ float tile[2][kTrTile][kTrTile + 1];
    __shared__ double red[kTrThreads / 64];
    // thread -> 4 consecutive columns (cx .. cx+3) of row ry of the 32 x 32 tile, both maps
    const int cx = (threadIdx.x & 7) * 4, ry = threadIdx.x >> 3;
    const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const LbDesc& l = L[w.x];
        const SliceDesc& dsc = D[w.x];
        const SolverState& s = *l.st;
        if (s.skip) continue;
        const int mode = s.mode;
        const int mc = mode == MODE_NEW_DIR ? s.m_cur : 0;
        const double alpha = s.alpha, gamma = s.gamma;
        const int n = l.n, tx = w.y, ty = w.z;
        const size_t nn = (size_t)n * n;
        const int j = ty * kTrTile + ry, i0 = tx * kTrTile + cx;
        const bool vec = (n & 3) == 0 && j < n && i0 + 3 < n;   // whole aligned float4 in range
        // element e(c, q) of this thread: map c, column i0 + q, row j
        float zt[2][4];
        if (vec) {
            double dv[2][4];
            const size_t e0 = (size_t)j * n + i0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float4 g4 = mode == MODE_NEW_DIR ? *(const float4*)(l.g + c * nn + e0)
                                                       : make_float4(0.f, 0.f, 0.f, 0.f);
                const float4 d4 = mode == MODE_BACKTRACK ? *(const float4*)(l.d + c * nn + e0)
                                                         : make_float4(0.f, 0.f, 0.f, 0.f);
                dv[c][0] = mode == MODE_NEW_DIR ? -gamma * g4.x : (double)d4.x;
                dv[c][1] = mode == MODE_NEW_DIR ? -gamma * g4.y : (double)d4.y;
                dv[c][2] = mode == MODE_NEW_DIR ? -gamma * g4.z : (double)d4.z;
                dv[c][3] = mode == MODE_NEW_DIR ? -gamma * g4.w : (double)d4.w;
            }
            // history combination, next slot's vectors loaded while this one is applied
            float4 sv[2], yv[2];
            auto load_slot = [&](int q) {
                const size_t o = (size_t)s.order[q] * l.nv + e0;
                sv[0] = *(const float4*)(l.S + o);
                yv[0] = *(const float4*)(l.Y + o);
                sv[1] = *(const float4*)(l.S + o + nn);
                yv[1] = *(const float4*)(l.Y + o + nn);
            };
            if (mc > 0) load_slot(0);
            for (int q = 0; q < mc; ++q) {
                const float4 s0 = sv[0], y0 = yv[0], s1 = sv[1], y1 = yv[1];
                if (q + 1 < mc) load_slot(q + 1);
                const double ee = -s.ee[q], cc = s.cc[q];
                dv[0][0] = fma(cc, (double)y0.x, fma(ee, (double)s0.x, dv[0][0]));
                dv[0][1] = fma(cc, (double)y0.y, fma(ee, (double)s0.y, dv[0][1]));
                dv[0][2] = fma(cc, (double)y0.z, fma(ee, (double)s0.z, dv[0][2]));
                dv[0][3] = fma(cc, (double)y0.w, fma(ee, (double)s0.w, dv[0][3]));
                dv[1][0] = fma(cc, (double)y1.x, fma(ee, (double)s1.x, dv[1][0]));
                dv[1][1] = fma(cc, (double)y1.y, fma(ee, (double)s1.y, dv[1][1]));
                dv[1][2] = fma(cc, (double)y1.z, fma(ee, (double)s1.z, dv[1][2]));
                dv[1][3] = fma(cc, (double)y1.w, fma(ee, (double)s1.w, dv[1][3]));
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float4 z4 = *(const float4*)(l.z + c * nn + e0);
                float4 t4;
                if (mode == MODE_INIT) {
                    t4 = z4;
                } else {
                    t4.x = (float)fma(alpha, dv[c][0], (double)z4.x);
                    t4.y = (float)fma(alpha, dv[c][1], (double)z4.y);
                    t4.z = (float)fma(alpha, dv[c][2], (double)z4.z);
                    t4.w = (float)fma(alpha, dv[c][3], (double)z4.w);
                    if (mode == MODE_NEW_DIR)
                        *(float4*)(l.d + c * nn + e0) =
                            make_float4((float)dv[c][0], (float)dv[c][1], (float)dv[c][2], (float)dv[c][3]);
                }
                *(float4*)(l.zt + c * nn + e0) = t4;
                zt[c][0] = t4.x; zt[c][1] = t4.y; zt[c][2] = t4.z; zt[c][3] = t4.w;
            }
        } else {
            // edge tiles or n not a multiple of 4: element by element
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = i0 + u;
                    float t = 0.f;
                    if (j < n && i < n) {
                        const size_t e = c * nn + (size_t)j * n + i;
                        const float z = l.z[e];
                        if (mode == MODE_INIT) {
                            t = z;
                        } else {
                            double dv;
                            if (mode == MODE_NEW_DIR) {
                                dv = -gamma * (double)l.g[e];
                                for (int q = 0; q < mc; ++q) {
                                    const int64_t o = (int64_t)s.order[q] * l.nv + e;
                                    dv = fma(-s.ee[q], (double)l.S[o], dv);
                                    dv = fma(s.cc[q], (double)l.Y[o], dv);
                                }
                                l.d[e] = (float)dv;
                            } else {
                                dv = (double)l.d[e];
                            }
                            t = (float)fma(alpha, dv, (double)z);
                        }
                        l.zt[e] = t;
                    }
                    zt[c][u] = t;
                }
        }
        double sq[2] = {0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                tile[c][ry][cx + u] = zt[c][u];
                sq[c] = fma((double)zt[c][u], (double)zt[c][u], sq[c]);
            }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            float* dst = dsc.xT + c * nn;
            for (int r = ly; r < kTrTile; r += 8) {
                const int i = tx * kTrTile + r, jj = ty * kTrTile + lx;
                if (i < n && jj < n) dst[(size_t)i * n + jj] = tile[c][lx][r];
            }
        }
        sq[0] = block_sum(sq[0], red);
        sq[1] = block_sum(sq[1], red);
        if (threadIdx.x == 0) {
            const int ntx = (n + kTrTile - 1) / kTrTile;
            double* p = dsc.part_reg + 2 * (size_t)(ty * ntx + tx);
            p[0] = sq[0];
            p[1] = sq[1];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ accept: update + dots
// s_new = zt - z, y_new = gt - g into the spare slot; z <- zt, g <- gt; per-block partial
// inner products: [0] g.g [1] s.s [2] y.y [3] s.y [4] z_old.z_old [5] s.g [6] y.g and, for
// every committed slot r: [7+4r] s_r.y [8+4r] y_r.y [9+4r] s_r.g [10+4r] y_r.g (g = new g).
// Each product is reduced across the wavefront with shuffles as soon as it is complete; the
// four wavefront sums meet once in LDS. Partials are stored [block][product].
__global__ __launch_bounds__(kVecThreads) void k_lb_update(const LbDesc* __restrict__ L,
                                                         const Item* __restrict__ items,
                                                         int n_items) {
    constexpr int NW = kVecThreads / 64;
    __shared__ double wsum[NW][max_dots(kMaxM)];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const LbDesc& l = L[w.x];
        const SolverState& st = *l.st;
        if (st.skip_adj) continue;
        const int init = st.mode == MODE_INIT;
        const int mc = init ? 0 : st.m_cur;
        const int64_t nv = l.nv;
        const int64_t e0 = (int64_t)w.y * kVecChunk;
        const int64_t e1 = min(e0 + kVecChunk, nv);
        constexpr int PER = kVecChunk / kVecThreads;
        float yv[PER], gv[PER];
        double acc[kDotsFixed];
#pragma unroll
        for (int q = 0; q < kDotsFixed; ++q) acc[q] = 0.0;
        const int64_t sp = (int64_t)st.spare * nv;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int64_t e = e0 + threadIdx.x + (int64_t)u * kVecThreads;
            yv[u] = 0.f; gv[u] = 0.f;
            if (e < e1) {
                const float gt = l.gt[e];
                gv[u] = gt;
                acc[0] = fma((double)gt, (double)gt, acc[0]);
                if (!init) {
                    const float zo = l.z[e], zn = l.zt[e], go = l.g[e];
                    const float sv = zn - zo, y = gt - go;
                    yv[u] = y;
                    l.S[sp + e] = sv;
                    l.Y[sp + e] = y;
                    l.z[e] = zn;
                    acc[1] = fma((double)sv, (double)sv, acc[1]);
                    acc[2] = fma((double)y, (double)y, acc[2]);
                    acc[3] = fma((double)sv, (double)y, acc[3]);
                    acc[4] = fma((double)zo, (double)zo, acc[4]);
                    acc[5] = fma((double)sv, (double)gt, acc[5]);
                    acc[6] = fma((double)y, (double)gt, acc[6]);
                }
                l.g[e] = gt;
            }
        }
#pragma unroll
        for (int q = 0; q < kDotsFixed; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) wsum[wid][q] = v;
        }
        float sb[PER], yb[PER];
        auto load_slot = [&](int r) {
            const int64_t o = (int64_t)st.order[r] * nv;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int64_t e = e0 + threadIdx.x + (int64_t)u * kVecThreads;
                sb[u] = e < e1 ? l.S[o + e] : 0.f;
                yb[u] = e < e1 ? l.Y[o + e] : 0.f;
            }
        };
        if (mc > 0) load_slot(0);
        for (int r = 0; r < mc; ++r) {
            float sr[PER], yr[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) { sr[u] = sb[u]; yr[u] = yb[u]; }
            if (r + 1 < mc) load_slot(r + 1);          // in flight during this slot's sums
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                a0 = fma((double)sr[u], (double)yv[u], a0);
                a1 = fma((double)yr[u], (double)yv[u], a1);
                a2 = fma((double)sr[u], (double)gv[u], a2);
                a3 = fma((double)yr[u], (double)gv[u], a3);
            }
            a0 = wave_sum(a0);
            a1 = wave_sum(a1);
            a2 = wave_sum(a2);
            a3 = wave_sum(a3);
            if (lane == 0) {
                wsum[wid][kDotsFixed + 4 * r + 0] = a0;
                wsum[wid][kDotsFixed + 4 * r + 1] = a1;
                wsum[wid][kDotsFixed + 4 * r + 2] = a2;
                wsum[wid][kDotsFixed + 4 * r + 3] = a3;
            }
        }
        __syncthreads();
        const int nd = kDotsFixed + 4 * mc;
        double* part = l.part + (int64_t)w.y * max_dots(st.m);   // row w.y of [block][dot]
        for (int q = threadIdx.x; q < nd; q += kVecThreads) {
            double v = 0.0;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) v += wsum[ww][q];
            part[q] = v;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ decision / finalize
// One block per slice. (Running these as the epilogue of the last block of the preceding
// kernel needs device-scope release/acquire, which on a multi-XCD GPU writes back and
// invalidates L2 per block and costs far more than the extra launch.)
__global__ __launch_bounds__(kIcThreads) void k_lb_decide(const SliceDesc* __restrict__ D,
                                                         const LbDesc* __restrict__ L) {
    SolverState& s = *L[blockIdx.x].st;
    if (s.skip) return;
    decide_body(D[blockIdx.x], s);
}

__global__ __launch_bounds__(256) void k_lb_finalize(const LbDesc* __restrict__ L) {
    const LbDesc& l = L[blockIdx.x];
    if (l.st->skip_adj) return;
    finalize_body(l);
}

hipError_t launch_lb_decide(const SliceDesc* D, const LbDesc* L, int n_slices, hipStream_t s) {
    k_lb_decide<<<n_slices, kIcThreads, 0, s>>>(D, L);
    return hipGetLastError();
}
hipError_t launch_lb_finalize(const LbDesc* L, int n_slices, hipStream_t s) {
    k_lb_finalize<<<n_slices, 256, 0, s>>>(L);
    return hipGetLastError();
}

// ------------------------------------------------------------------------ descriptor upload
__global__ void k_store_desc(SliceDesc v, SliceDesc* dst) { *dst = v; }
__global__ void k_store_lbdesc(LbDesc v, LbDesc* dst) { *dst = v; }

// ------------------------------------------------------------------------ launchers
hipError_t launch_lb_init(const LbDesc* L, int n_slices, int m, int max_iter, int max_ls,
                          double c1, double tol, hipStream_t s) {
    k_lb_init<<<n_slices, 64, 0, s>>>(L, m, max_iter, max_ls, c1, tol);
    return hipGetLastError();
}
hipError_t launch_lb_scale(const LbDesc* L, const Item* items, int n_items, int grid, int to_z,
                           hipStream_t s) {
    k_lb_scale<<<grid, kVecThreads, 0, s>>>(L, items, n_items, to_z);
    return hipGetLastError();
}
hipError_t launch_lb_direction(const LbDesc* L, const SliceDesc* D, const Item* items, int n_items,
                               int grid, hipStream_t s) {
    k_lb_direction<<<grid, kTrThreads, 0, s>>>(L, D, items, n_items);
    return hipGetLastError();
}
hipError_t launch_lb_update(const LbDesc* L, const Item* items, int n_items, int grid,
                            hipStream_t s) {
    k_lb_update<<<grid, kVecThreads, 0, s>>>(L, items, n_items);
    return hipGetLastError();
}
hipError_t launch_store_desc(const SliceDesc& v, SliceDesc* dst, hipStream_t s) {
    k_store_desc<<<1, 1, 0, s>>>(v, dst);
    return hipGetLastError();
}
hipError_t launch_store_lbdesc(const LbDesc& v, LbDesc* dst, hipStream_t s) {
    k_store_lbdesc<<<1, 1, 0, s>>>(v, dst);
    return hipGetLastError();
}

}  // namespace eit
