// Device-side L-BFGS control logic (compact representation, Armijo backtracking): the
// line-search decision and the memory update with the next direction's coefficients, each
// run by one block per slice (k_lb_decide, k_lb_finalize in lbfgs.hip).
#pragma once
#include "device_common.h"
#include "reduce.h"
#include "eitomo.h"

namespace eit {

// ------------------------------------------------------------------------ helpers
__device__ inline void steepest(SolverState& s) {
    s.gamma = 1.0;
    for (int r = 0; r < kMaxM; ++r) { s.cc[r] = 0.0; s.ee[r] = 0.0; }
    s.gd = -s.gg;
    s.alpha = 1.0 / sqrt(s.gg);
    s.trials = 0;
    s.mode = MODE_NEW_DIR;
}

__device__ inline void reset_memory(SolverState& s) {
    s.m_cur = 0;
    s.spare = 0;
}

// Value of lane q (the same q in every lane) in every lane: two scalar lane reads instead of
// an LDS permute, which keeps the substitution chains below short.
__device__ __forceinline__ double lane_bcast(double v, int q) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), q);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), q);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Direction coefficients from a_r = s_r.g, b_r = y_r.g (ring order, oldest first). SY and YY
// are the ring-ordered m_cur x m_cur matrices (row stride kMaxM) in LDS. Runs in the first
// wavefront of the block: lane r owns row r, and each substitution step broadcasts the newly
// solved component to the other lanes (m_cur <= kMaxM < 64).
//   c = R^{-1} a (back substitution), v = (D + gamma Y^T Y) c - gamma b,
//   e = R^{-T} v (forward substitution), g.Hg = gamma g.g + sum_r (a_r e_r - gamma b_r c_r).
__device__ inline void compact_direction(SolverState& s, const double* a, const double* b,
                                         const double* SY, const double* YY) {
    const int lane = threadIdx.x;
    const int mc = s.m_cur;
    const int W = kMaxM;
    const double gamma = SY[(mc - 1) * W + (mc - 1)] / YY[(mc - 1) * W + (mc - 1)];
    const bool on = lane < mc;
    const double Rrr = on ? SY[lane * W + lane] : 1.0;
    const double rinv = 1.0 / Rrr;                    // one division per lane, off the chain
    const double ar = on ? a[lane] : 0.0, br = on ? b[lane] : 0.0;
    double acc = ar, c = 0.0;
    for (int q = mc - 1; q >= 0; --q) {               // c_q known once rows > q are folded in
        const double cq = lane_bcast(acc * rinv, q);
        if (lane == q) c = cq;
        if (lane < q) acc -= SY[lane * W + q] * cq;
    }
    double v = on ? Rrr * c - gamma * br : 0.0;
    for (int q = 0; q < mc; ++q) {
        const double cq = lane_bcast(c, q);
        if (on) v += gamma * YY[lane * W + q] * cq;
    }
    double acc2 = v, e = 0.0;
    for (int q = 0; q < mc; ++q) {
        const double eq = lane_bcast(acc2 * rinv, q);
        if (lane == q) e = eq;
        if (on && lane > q) acc2 -= SY[q * W + lane] * eq;
    }
    const double t = wave_sum(on ? ar * e - gamma * br * c : 0.0);
    if (lane < kMaxM) {
        s.ee[lane] = on ? e : 0.0;
        s.cc[lane] = on ? gamma * c : 0.0;
    }
    if (lane == 0) {
        s.gamma = gamma;
        s.gd = -(gamma * s.gg + t);
        s.alpha = 1.0;
        s.trials = 0;
        s.mode = MODE_NEW_DIR;
        if (!(s.gd < 0.0)) {                            // not a descent direction
            reset_memory(s);
            steepest(s);
        }
    }
}

__device__ inline void finish(SolverState& s, int status) {
    s.status = status;
    s.skip = 1;
    s.skip_adj = 1;
}

// ------------------------------------------------------------------------ decision
// Block-wide: reduce the cost at the trial point (FP64, fixed order) and run the Armijo test
// F(zt) <= F(z) + c1 alpha g.d. One block per slice, after the IC launch.
__device__ inline void decide_body(const SliceDesc& d, SolverState& s) {
    __shared__ double red[kIcThreads / 64];
    double a = 0.0, r0 = 0.0, r1 = 0.0;
    for (int i = threadIdx.x; i < d.n_theta; i += blockDim.x) a += d.part_ic[i];
    for (int b = threadIdx.x; b < d.n_reg_blocks; b += blockDim.x) {
        r0 += d.part_reg[2 * b];
        r1 += d.part_reg[2 * b + 1];
    }
    a = block_sum(a, red);
    r0 = block_sum(r0, red);
    r1 = block_sum(r1, red);
    if (threadIdx.x != 0) return;
    const double ft = a + d.lam_mu * r0 + d.lam_de * r1;
    s.f_t = ft;
    s.launches += 1;
    s.evals += 1;
    if (s.mode == MODE_INIT) {
        if (!isfinite(ft)) {
            s.accept = 0;
            finish(s, EIT_ERR_NONFINITE);
        } else {
            s.accept = 1;
            s.skip_adj = 0;
        }
        return;
    }
    s.trials += 1;
    const bool ok = ft <= s.f + s.c1 * s.alpha * s.gd;      // false for NaN
    if (ok) {
        s.accept = 1;
        s.skip_adj = 0;
        return;
    }
    s.accept = 0;
    s.skip_adj = 1;
    if (s.trials >= s.max_ls) {
        if (s.m_cur > 0) {           // drop the memory, retry along -g
            reset_memory(s);
            steepest(s);
        } else {
            finish(s, EIT_ERR_LINESEARCH);
        }
    } else {
        s.alpha *= 0.5;
        s.mode = MODE_BACKTRACK;
    }
}

// ------------------------------------------------------------------------ accept: finalize
constexpr int kFinThreads = 1024;
// Block-wide (kFinThreads threads), one block per slice:
// reduce the partial inner products in a fixed order, commit the pair if
// s.y > 1e-10 ||s|| ||y||, advance the iteration counter, test the stopping rules and
// compute the next direction's coefficients. The scalar logic runs in one thread on an LDS
// copy of the state.
__device__ inline void finalize_body(const LbDesc& l) {
    constexpr int W = kMaxM + 1;
    __shared__ double dots[max_dots(kMaxM)];
    constexpr int NSUB = kFinThreads / 64;
    __shared__ double redp[NSUB][64];
    __shared__ double sSY[W * W], sYY[W * W];
    __shared__ double oSY[kMaxM * kMaxM], oYY[kMaxM * kMaxM];
    __shared__ double av[kMaxM], bv[kMaxM];
    __shared__ int sorder[kMaxM];
    __shared__ int go, sm2;
    __shared__ SolverState s;          // working copy: the scalar logic touches LDS only
    SolverState& gs = *l.st;
    {
        const int* src = (const int*)&gs;
        int* dst = (int*)&s;
        for (int i = threadIdx.x; i < (int)(sizeof(SolverState) / 4); i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const int init = s.mode == MODE_INIT;
    const int mc = init ? 0 : s.m_cur;
    const int nd = kDotsFixed + 4 * mc;
    const int stride = max_dots(s.m);
    // products q0 .. q0+63 at a time: product q = q0 + t % 64 summed by the NSUB threads
    // t = q - q0 + 64 k over interleaved block rows (independent loads, all in flight), then
    // combined in a fixed order
    for (int q0 = 0; q0 < nd; q0 += 64) {
        const int ql = threadIdx.x & 63, sub = threadIdx.x >> 6, q = q0 + ql;
        double v = 0.0;
        if (q < nd) {
#pragma unroll 16
            for (int b = sub; b < l.n_vblocks; b += NSUB) v += l.part[(int64_t)b * stride + q];
        }
        redp[sub][ql] = v;
        __syncthreads();
        if ((int)threadIdx.x < 64 && q < nd) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < NSUB; ++k) t += redp[k][ql];
            dots[q] = t;
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < W * W; i += blockDim.x) {
        sSY[i] = s.SY[i];
        sYY[i] = s.YY[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        go = 0;
        s.f = s.f_t;
        s.gg = dots[0];
        if (init) {
            if (s.cost_hist) s.cost_hist[0] = s.f;
            reset_memory(s);
            steepest(s);
            if (s.max_iter <= 0) finish(s, ST_DONE);
            else if (s.max_ls <= 0) finish(s, EIT_ERR_LINESEARCH);
            else s.skip_adj = 1;
        } else {
            const double ss = dots[1], yy = dots[2], sy = dots[3], zz = dots[4];
            for (int r = 0; r < mc; ++r) {
                av[r] = dots[kDotsFixed + 4 * r + 2];
                bv[r] = dots[kDotsFixed + 4 * r + 3];
                sorder[r] = s.order[r];
            }
            int m_new = mc;
            if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
                const int sp = s.spare;
                for (int r = 0; r < mc; ++r) {
                    const int o = sorder[r];
                    sSY[o * W + sp] = dots[kDotsFixed + 4 * r + 0];
                    const double yyr = dots[kDotsFixed + 4 * r + 1];
                    sYY[o * W + sp] = yyr;
                    sYY[sp * W + o] = yyr;
                }
                sSY[sp * W + sp] = sy;
                sYY[sp * W + sp] = yy;
                if (mc < s.m) {
                    sorder[mc] = sp;
                    av[mc] = dots[5];
                    bv[mc] = dots[6];
                    m_new = mc + 1;
                    int nxt = 0;                      // smallest slot id not in the ring
                    for (;; ++nxt) {
                        bool used = false;
                        for (int r = 0; r < m_new; ++r) used |= (sorder[r] == nxt);
                        if (!used) break;
                    }
                    s.spare = nxt;
                } else {
                    const int evict = sorder[0];
                    for (int r = 0; r + 1 < mc; ++r) {
                        sorder[r] = sorder[r + 1];
                        av[r] = av[r + 1];
                        bv[r] = bv[r + 1];
                    }
                    sorder[mc - 1] = sp;
                    av[mc - 1] = dots[5];
                    bv[mc - 1] = dots[6];
                    s.spare = evict;
                }
            }
            s.m_cur = m_new;
            sm2 = m_new;
            for (int r = 0; r < m_new; ++r) s.order[r] = sorder[r];
            s.k += 1;
            if (s.cost_hist) s.cost_hist[s.k] = s.f;
            if (s.k >= s.max_iter) finish(s, ST_DONE);
            else if (s.tol > 0.0 && zz > 0.0 && sqrt(ss / zz) < s.tol) finish(s, ST_DONE);
            else if (s.m_cur == 0) { steepest(s); s.skip_adj = 1; }
            else go = 1;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < W * W; i += blockDim.x) {
        s.SY[i] = sSY[i];
        s.YY[i] = sYY[i];
    }
    if (go) {
        const int m2 = sm2;
        for (int i = threadIdx.x; i < m2 * m2; i += blockDim.x) {
            const int r = i / m2, q = i % m2;
            oSY[r * kMaxM + q] = sSY[sorder[r] * W + sorder[q]];
            oYY[r * kMaxM + q] = sYY[sorder[r] * W + sorder[q]];
        }
    }
    __syncthreads();
    if (go && threadIdx.x < 64) {
        compact_direction(s, av, bv, oSY, oYY);
        if (threadIdx.x == 0) s.skip_adj = 1;
    }
    __syncthreads();
    {   // write the working copy back
        const int* src = (const int*)&s;
        int* dst = (int*)&gs;
        for (int i = threadIdx.x; i < (int)(sizeof(SolverState) / 4); i += blockDim.x) dst[i] = src[i];
    }
}


}  // namespace eit
