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
        const int64_t e0 = (int64_t)w.y * kVecChunk;
        const int64_t e1 = min(e0 + kVecChunk, l.nv);
        const int64_t maps_end = l.n_maps * l.nn;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kVecThreads) {
            const float sc = e < l.nn ? l.scale_mu : (e < maps_end ? l.scale_de : l.scale_off);
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
            // history combination: the vectors of a batch of slots are requested together
            // (one memory round trip per batch), then applied oldest first
            for (int r0 = 0; r0 < mc; r0 += kSlotBatch) {
                float4 sv[kSlotBatch][2], yv[kSlotBatch][2];
#pragma unroll
                for (int b = 0; b < kSlotBatch; ++b) {
                    if (r0 + b < mc) {
                        const size_t o = (size_t)s.order[r0 + b] * l.nv + e0;
                        sv[b][0] = *(const float4*)(l.S + o);
                        yv[b][0] = *(const float4*)(l.Y + o);
                        sv[b][1] = *(const float4*)(l.S + o + nn);
                        yv[b][1] = *(const float4*)(l.Y + o + nn);
                    }
                }
#pragma unroll
                for (int b = 0; b < kSlotBatch; ++b) {
                    if (r0 + b < mc) {
                        const double ee = -s.ee[r0 + b], cc = s.cc[r0 + b];
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const float4 sq = sv[b][c], yq = yv[b][c];
                            dv[c][0] = fma(cc, (double)yq.x, fma(ee, (double)sq.x, dv[c][0]));
                            dv[c][1] = fma(cc, (double)yq.y, fma(ee, (double)sq.y, dv[c][1]));
                            dv[c][2] = fma(cc, (double)yq.z, fma(ee, (double)sq.z, dv[c][2]));
                            dv[c][3] = fma(cc, (double)yq.w, fma(ee, (double)sq.w, dv[c][3]));
                        }
                    }
                }
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
// A thread owns 8 consecutive elements (two float4 when aligned). The committed slots'
// vectors are requested a batch at a time (one memory round trip per batch). Each product is
// reduced across the wavefront as soon as it is complete; the four wavefront sums meet once
// in LDS. Partials are stored [block][product].
__device__ __forceinline__ void ld8(const float* __restrict__ p, int64_t e, int64_t nv, bool vec,
                                    float* v) {
    if (vec) {
        const float4 a = *(const float4*)(p + e), b = *(const float4*)(p + e + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = e + u < nv ? p[e + u] : 0.f;
    }
}
__device__ __forceinline__ void st8(float* __restrict__ p, int64_t e, int64_t nv, bool vec,
                                    const float* v) {
    if (vec) {
        *(float4*)(p + e) = make_float4(v[0], v[1], v[2], v[3]);
        *(float4*)(p + e + 4) = make_float4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e + u < nv) p[e + u] = v[u];
    }
}

// ------------------------------------------------------------------------ direction (vector form)
// Item (slice, chunk) over the optimiser's vector, for the full model of eq. 4 whose vector
// (maps, then offsets) is not a pair of maps: the same direction and trial point as
// k_lb_direction (FP64 combination, history slots requested a batch at a time), a thread
// owning 8 consecutive elements, without the fused transpose. In h-mode with the pair
// evaluation the trial point's map is also written twice into the expanded pair D.xe that
// the two-map kernels evaluate (the single-map evaluation reads the trial point itself).
__global__ __launch_bounds__(kVecThreads) void k_lb_direction_vec(const LbDesc* __restrict__ L,
                                                                 const SliceDesc* __restrict__ D,
                                                                 const Item* __restrict__ items,
                                                                 int n_items) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const LbDesc& l = L[w.x];
        const SliceDesc& dsc = D[w.x];
        const SolverState& s = *l.st;
        if (s.skip) continue;
        const int mode = s.mode;
        const int mc = mode == MODE_NEW_DIR ? s.m_cur : 0;
        const double alpha = s.alpha, gamma = s.gamma;
        const int64_t nv = l.nv;
        const int64_t e = (int64_t)w.y * kVecChunk + 8 * (int64_t)threadIdx.x;
        if (e >= nv) continue;
        const bool vec = (nv & 3) == 0 && e + 8 <= nv;
        float zv[8], tv[8];
        ld8(l.z, e, nv, vec, zv);
        if (mode == MODE_INIT) {
#pragma unroll
            for (int u = 0; u < 8; ++u) tv[u] = zv[u];
        } else {
            double dv[8];
            float tmp[8];
            if (mode == MODE_NEW_DIR) {
                ld8(l.g, e, nv, vec, tmp);
#pragma unroll
                for (int u = 0; u < 8; ++u) dv[u] = -gamma * (double)tmp[u];
                for (int r0 = 0; r0 < mc; r0 += kSlotBatch) {
                    float sb[kSlotBatch][8], yb[kSlotBatch][8];
#pragma unroll
                    for (int b = 0; b < kSlotBatch; ++b) {
                        if (r0 + b < mc) {
                            const int64_t o = (int64_t)s.order[r0 + b] * nv;
                            ld8(l.S + o, e, nv, vec, sb[b]);
                            ld8(l.Y + o, e, nv, vec, yb[b]);
                        }
                    }
#pragma unroll
                    for (int b = 0; b < kSlotBatch; ++b) {
                        if (r0 + b < mc) {
                            const double ee = -s.ee[r0 + b], cc = s.cc[r0 + b];
#pragma unroll
                            for (int u = 0; u < 8; ++u)
                                dv[u] = fma(cc, (double)yb[b][u], fma(ee, (double)sb[b][u], dv[u]));
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) tmp[u] = (float)dv[u];
                st8(l.d, e, nv, vec, tmp);
            } else {
                ld8(l.d, e, nv, vec, tmp);
#pragma unroll
                for (int u = 0; u < 8; ++u) dv[u] = (double)tmp[u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) tv[u] = (float)fma(alpha, dv[u], (double)zv[u]);
        }
        st8(l.zt, e, nv, vec, tv);
        if ((dsc.ext & EXT_HMODE) && dsc.maps != 1 && e < l.nn) {   // pair evaluation only
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e + u < l.nn) {
                    dsc.xe[e + u] = tv[u];
                    dsc.xe[l.nn + e + u] = tv[u];
                }
        }
    }
}

// Gradient at the trial point from the split adjoint's partial planes: the parts are added in
// plane order, then the regulariser reg * zt, then rounded -- the adjoint's own epilogue.
__device__ __forceinline__ void split_gradient(const LbDesc& l, int64_t e, int64_t nv, bool vec,
                                               const float* zn, float* gv) {
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    for (int g = 0; g < l.gsplits; ++g) {
        const double* p = l.gpart + (int64_t)g * nv + e;
        if (vec) {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const double2 v = *(const double2*)(p + 2 * h);
                acc[2 * h] += v.x;
                acc[2 * h + 1] += v.y;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e + u < nv) acc[u] += p[u];
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double reg = e + u < nv / 2 ? l.reg_mu : l.reg_de;
        gv[u] = (float)fma(reg, (double)zn[u], acc[u]);
    }
}

__global__ __launch_bounds__(kVecThreads) void k_lb_update(const LbDesc* __restrict__ L,
                                                         const Item* __restrict__ items,
                                                         int n_items) {
    constexpr int NW = kVecThreads / 64;
    static_assert(kVecChunk == 8 * kVecThreads, "8 elements per thread");
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
        const int64_t e = (int64_t)w.y * kVecChunk + 8 * (int64_t)threadIdx.x;
        // slot offsets k * nv keep 16-byte alignment when nv % 4 == 0
        const bool vec = (nv & 3) == 0 && e + 8 <= nv;
        float yv[8], gv[8];
        double acc[kDotsFixed];
#pragma unroll
        for (int q = 0; q < kDotsFixed; ++q) acc[q] = 0.0;
        if (e < nv) {
            float zn[8];
            if (l.gsplits > 1) {
                ld8(l.zt, e, nv, vec, zn);
                split_gradient(l, e, nv, vec, zn, gv);
            } else {
                ld8(l.gt, e, nv, vec, gv);
                if (!init) ld8(l.zt, e, nv, vec, zn);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[0] = fma((double)gv[u], (double)gv[u], acc[0]);
            if (!init) {
                float zo[8], go[8], sv[8];
                ld8(l.z, e, nv, vec, zo);
                ld8(l.g, e, nv, vec, go);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    sv[u] = zn[u] - zo[u];
                    yv[u] = gv[u] - go[u];
                    acc[1] = fma((double)sv[u], (double)sv[u], acc[1]);
                    acc[2] = fma((double)yv[u], (double)yv[u], acc[2]);
                    acc[3] = fma((double)sv[u], (double)yv[u], acc[3]);
                    acc[4] = fma((double)zo[u], (double)zo[u], acc[4]);
                    acc[5] = fma((double)sv[u], (double)gv[u], acc[5]);
                    acc[6] = fma((double)yv[u], (double)gv[u], acc[6]);
                }
                const int64_t sp = (int64_t)st.spare * nv;
                st8(l.S + sp, e, nv, vec, sv);
                st8(l.Y + sp, e, nv, vec, yv);
                st8(l.z, e, nv, vec, zn);
            } else {
#pragma unroll
                for (int u = 0; u < 8; ++u) yv[u] = 0.f;
            }
            st8(l.g, e, nv, vec, gv);
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) { yv[u] = 0.f; gv[u] = 0.f; }
        }
#pragma unroll
        for (int q = 0; q < kDotsFixed; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) wsum[wid][q] = v;
        }
        for (int r0 = 0; r0 < mc; r0 += kSlotBatch) {
            float sb[kSlotBatch][8], yb[kSlotBatch][8];
#pragma unroll
            for (int b = 0; b < kSlotBatch; ++b) {
                if (r0 + b < mc) {
                    const int64_t o = (int64_t)st.order[r0 + b] * nv;
                    if (e < nv) {
                        ld8(l.S + o, e, nv, vec, sb[b]);
                        ld8(l.Y + o, e, nv, vec, yb[b]);
                    } else {
#pragma unroll
                        for (int u = 0; u < 8; ++u) { sb[b][u] = 0.f; yb[b][u] = 0.f; }
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < kSlotBatch; ++b) {
                if (r0 + b < mc) {
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        a0 = fma((double)sb[b][u], (double)yv[u], a0);
                        a1 = fma((double)yb[b][u], (double)yv[u], a1);
                        a2 = fma((double)sb[b][u], (double)gv[u], a2);
                        a3 = fma((double)yb[b][u], (double)gv[u], a3);
                    }
                    a0 = wave_sum(a0);
                    a1 = wave_sum(a1);
                    a2 = wave_sum(a2);
                    a3 = wave_sum(a3);
                    if (lane == 0) {
                        const int r = r0 + b;
                        wsum[wid][kDotsFixed + 4 * r + 0] = a0;
                        wsum[wid][kDotsFixed + 4 * r + 1] = a1;
                        wsum[wid][kDotsFixed + 4 * r + 2] = a2;
                        wsum[wid][kDotsFixed + 4 * r + 3] = a3;
                    }
                }
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

__global__ __launch_bounds__(kFinThreads) void k_lb_finalize(const LbDesc* __restrict__ L) {
    const LbDesc& l = L[blockIdx.x];
    if (l.st->skip_adj) return;
    finalize_body(l);
}

// Read-back helpers for batches: the host reads every slice's state in one copy from a
// contiguous array instead of one copy per slice. k_gather_status: (k, evals, trials, mode,
// status) -- consecutive int32 fields of SolverState -- of slice i into out[5 i ..]; one
// thread per slice. k_gather_states: the whole state of slice blockIdx.x into out[blockIdx.x].
__global__ void k_gather_status(const LbDesc* __restrict__ L, int n, int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t* src = &L[i].st->k;
#pragma unroll
    for (int q = 0; q < 5; ++q) out[5 * i + q] = src[q];
}
__global__ void k_gather_states(const LbDesc* __restrict__ L, SolverState* __restrict__ out) {
    const int* src = (const int*)L[blockIdx.x].st;
    int* dst = (int*)(out + blockIdx.x);
    for (int q = threadIdx.x; q < (int)(sizeof(SolverState) / 4); q += blockDim.x) dst[q] = src[q];
}

hipError_t launch_lb_decide(const SliceDesc* D, const LbDesc* L, int n_slices, hipStream_t s) {
    k_lb_decide<<<n_slices, kIcThreads, 0, s>>>(D, L);
    return hipGetLastError();
}
hipError_t launch_gather_status(const LbDesc* L, int n_slices, int32_t* out, hipStream_t s) {
    if (n_slices <= 0) return hipSuccess;
    k_gather_status<<<(n_slices + 255) / 256, 256, 0, s>>>(L, n_slices, out);
    return hipGetLastError();
}
hipError_t launch_gather_states(const LbDesc* L, int n_slices, SolverState* out, hipStream_t s) {
    if (n_slices <= 0) return hipSuccess;
    k_gather_states<<<n_slices, 256, 0, s>>>(L, out);
    return hipGetLastError();
}
hipError_t launch_lb_finalize(const LbDesc* L, int n_slices, hipStream_t s) {
    k_lb_finalize<<<n_slices, kFinThreads, 0, s>>>(L);
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
hipError_t launch_lb_direction_vec(const LbDesc* L, const SliceDesc* D, const Item* items,
                                   int n_items, int grid, hipStream_t s) {
    k_lb_direction_vec<<<grid, kVecThreads, 0, s>>>(L, D, items, n_items);
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
