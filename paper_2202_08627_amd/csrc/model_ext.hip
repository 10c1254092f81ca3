// The paper's full forward model (theory section, eq. 4) on top of the two-map kernels:
//   s_mod[a][j][k] = T[a][k] f_k(m_j - m_o[a] - m_r[k] - Delta[a][k]),
// with three extensions of the plain model, each optional (SliceDesc::ext):
//   * h-mode (homogeneous object): one map h with mu = h and delta = gamma h. The projector's
//     and the adjoint's single-map forms project h once (P_mu and P_delta are that projection
//     scaled by scale_mu and gamma scale_mu) and backproject the sum of the two scaled seeds
//     (chain rule: d/dh = d/dmu + gamma d/ddelta). Slices wider than kSingleMapMaxDet run the
//     two-map kernels on the expanded pair [h, h] and add the two adjoint planes instead;
//   * per-angle drift m_o and per-pixel ring term m_r of the sample mask: unknowns whose
//     derivatives are sums of G_Delta = dS/dDelta over pixels (m_o) or angles (m_r), since u
//     depends on m_o, m_r and Delta with the same coefficient;
//   * a tabulated (measured) flat IC: F[k][q] at u_q = u0 + q du over one mask period (the
//     experiment section scans it in 33 steps), interpolated by cubic convolution (Keys 1981,
//     a = -1/2, continuously differentiable) and held at its end values outside the scan.
// Also the single-shot retrieval of eq. 3 for the h-mode (one mask position).
#include "device_common.h"

namespace eit {

// ------------------------------------------------------------------------ flat IC
// (f, f') of pixel k at u: Gaussian (A, c, 1/(2 s^2), 1/s^2) or the table.
__device__ __forceinline__ void flat_eval(const SliceDesc& d, int k, float4 fl, double u, double& f,
                                          double& fp) {
    if (d.ext & EXT_TABLE) {
        const int Q = d.nq;
        const double lo = d.tab_u0, hi = d.tab_u0 + (Q - 1) * d.tab_du;
        const bool inside = u >= lo && u <= hi;
        const double uc = fmin(fmax(u, lo), hi);
        const double xq = (uc - lo) / d.tab_du;
        const int q = min(max((int)floor(xq), 0), Q - 2);
        const double t = xq - q, t2 = t * t, t3 = t2 * t;
        const double* F = d.ftab + (size_t)k * Q;
        const double f0 = F[max(q - 1, 0)], f1 = F[q], f2 = F[q + 1], f3 = F[min(q + 2, Q - 1)];
        // Keys' cubic convolution weights of samples q-1 .. q+2 and their t-derivatives
        const double w0 = 0.5 * (-t3 + 2.0 * t2 - t), w1 = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
        const double w2 = 0.5 * (-3.0 * t3 + 4.0 * t2 + t), w3 = 0.5 * (t3 - t2);
        const double v0 = 0.5 * (-3.0 * t2 + 4.0 * t - 1.0), v1 = 0.5 * (9.0 * t2 - 10.0 * t);
        const double v2 = 0.5 * (-9.0 * t2 + 8.0 * t + 1.0), v3 = 0.5 * (3.0 * t2 - 2.0 * t);
        f = w0 * f0 + w1 * f1 + w2 * f2 + w3 * f3;
        fp = inside ? (v0 * f0 + v1 * f1 + v2 * f2 + v3 * f3) / d.tab_du : 0.0;
    } else {
        const double uu = u - (double)fl.y;
        f = (double)fl.x * exp(-uu * uu * (double)fl.z);
        fp = -uu * (double)fl.w * f;
    }
}

// ------------------------------------------------------------------------ IC model (eq. 4)
// Item (slice, angle, -, -). As the plain IC stage (FP64 model from FP32 projections, seeds
// in place of the projections), with the offsets of the point and the flat of the plan.
// Also: g_mo[a] = sum_k G_Delta[a][k] (drift, fixed-order block sum) and g_dl[a][k] =
// G_Delta[a][k] (ring; summed over angles by k_ext_ring_grad). G_Delta of the angle's row
// waits in dynamically sized LDS (2 n_det doubles of the widest slice in the launch), and the
// block has 256 threads when no slice has more than 256 detector pixels, else 512.
// Single-map evaluation (d.maps == 1, h-mode): plane 0 holds R h, read as P_mu = scale_mu R h
// and P_delta = scale_de R h (scale_de = gamma scale_mu), and the seed written back to plane 0
// is the sum of the two scaled seeds, which the one-map adjoint turns into the h gradient. The
// mu part waits in LDS until every thread has read its neighbours' projections.
constexpr int kExtMaxDet = 4096;
static_assert(kSingleMapMaxDet * 2 <= kExtMaxDet, "single-map rows fit the LDS bound");
template <int NT>
__global__ __launch_bounds__(NT) void k_ic_ext(const SliceDesc* __restrict__ D,
                                               const Item* __restrict__ items,
                                               int n_items, int want_seeds) {
    extern __shared__ double gdl[];
    __shared__ double red[NT / 64];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped(d)) continue;
        const int a = w.y, nd = d.n_det, M = d.n_mask, nt = d.n_theta;
        const bool one = d.maps == 1;
        float* Pm = d.P + (size_t)a * nd;
        float* Pd = one ? Pm : d.P + ((size_t)nt + a) * nd;
        double* gmu = gdl + nd;              // single-map: scaled mu seeds of the row
        const float* se = d.s_exp + (size_t)a * M * nd;
        const double sm = d.scale_mu, sdl = d.scale_de;
        const double kap = (double)d.kappa;
        const double mo = (d.ext & EXT_DRIFT) ? d.off_scale * (double)d.off[a] : 0.0;
        const float* mr = (d.ext & EXT_RING) ? d.off + ((d.ext & EXT_DRIFT) ? nt : 0) : nullptr;
        double r2 = 0.0, gsum = 0.0;
        for (int k = threadIdx.x; k < nd; k += NT) {
            const double pm = sm * (double)Pm[k];
            const double pp = k + 1 < nd ? sdl * (double)Pd[k + 1] : 0.0;
            const double pn = k > 0 ? sdl * (double)Pd[k - 1] : 0.0;
            const double T = exp(-pm);
            const double dl = kap * 0.5 * (pp - pn);
            const double base = -mo - (mr ? d.off_scale * (double)mr[k] : 0.0) - dl;
            const float4 fl = d.flat[k];
            double sf = 0.0, sfp = 0.0;
            for (int j = 0; j < M; ++j) {
                double f, fp;
                flat_eval(d, k, fl, d.mask[j] + base, f, fp);
                const double r = fma(T, f, -(double)se[(size_t)j * nd + k]);
                r2 = fma(r, r, r2);
                sf = fma(r, f, sf);
                sfp = fma(r, fp, sfp);
            }
            const double gD = -2.0 * T * sfp;                 // G_Delta
            if (want_seeds) {
                if (one) gmu[k] = sm * (-2.0 * T * sf);
                else Pm[k] = (float)(sm * (-2.0 * T * sf));   // G_Pmu, scaled
                gdl[k] = gD;
                if (mr) d.g_dl[(size_t)a * nd + k] = gD;
            }
            gsum += gD;
        }
        __syncthreads();   // every read of Pd done, gdl complete
        if (want_seeds) {
            for (int k = threadIdx.x; k < nd; k += NT) {
                const double gp = k + 1 < nd ? gdl[k + 1] : 0.0;
                const double gn = k > 0 ? gdl[k - 1] : 0.0;
                const double gd = sdl * (-kap * 0.5 * (gp - gn));   // G_Pdelta, scaled
                Pd[k] = (float)(one ? gmu[k] + gd : gd);
            }
        }
        r2 = block_sum(r2, red);
        if (want_seeds && (d.ext & EXT_DRIFT)) {
            gsum = block_sum(gsum, red);
            if (threadIdx.x == 0) d.g_mo[a] = gsum;
        }
        if (threadIdx.x == 0) d.part_ic[a] = r2;
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ expansion
// Item (slice, chunk): h-mode point [h] -> the pair [h, h] the two-map kernels evaluate.
__global__ __launch_bounds__(kVecThreads) void k_ext_expand(const SliceDesc* __restrict__ D,
                                                           const Item* __restrict__ items,
                                                           int n_items) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped(d)) continue;
        const int64_t nn = (int64_t)d.n * d.n;
        const int64_t e0 = (int64_t)w.y * kVecChunk, e1 = min(e0 + kVecChunk, nn);
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kVecThreads) {
            const float v = d.xu[e];
            d.xe[e] = v;
            d.xe[nn + e] = v;
        }
    }
}

// ------------------------------------------------------------------------ contraction
// Item (slice, chunk) over the parameter vector: the gradient in the parameter layout from
// the adjoint's planes (computed without the regulariser), the point xu and the offset
// sums. Maps: g_mu, g_delta (+ 2 lambda x), or in h-mode g_mu + g_delta (+ 2 lambda h), the
// single-map evaluation's one plane already being that sum;
// drift: off_scale * g_mo[a]. The ring entries are written by k_ext_ring_grad. The planes are
// g, or with a split adjoint the FP64 partial planes added here in part order.
__device__ __forceinline__ double adj_plane(const SliceDesc& d, int64_t e, int64_t nv2) {
    if (d.adj_splits <= 1) return (double)d.g[e];
    double v = 0.0;
    for (int g = 0; g < d.adj_splits; ++g) v += d.bp_part[g * nv2 + e];
    return v;
}

__global__ __launch_bounds__(kVecThreads) void k_ext_contract(const SliceDesc* __restrict__ D,
                                                             const Item* __restrict__ items,
                                                             int n_items) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped_adj(d)) continue;
        const int64_t nn = (int64_t)d.n * d.n;
        const bool hm = (d.ext & EXT_HMODE) != 0;
        const int64_t maps_end = hm ? nn : 2 * nn;
        const int64_t mo_end = maps_end + ((d.ext & EXT_DRIFT) ? d.n_theta : 0);
        const int64_t e0 = (int64_t)w.y * kContractChunk, e1 = min(e0 + kContractChunk, d.nvu);
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kVecThreads) {
            double v;
            if (e < maps_end) {
                if (hm && d.maps == 1) {        // one plane: the adjoint of the summed seeds
                    v = fma(d.reg_mu, (double)d.xu[e], adj_plane(d, e, nn));
                } else if (hm) {
                    v = adj_plane(d, e, 2 * nn) + adj_plane(d, nn + e, 2 * nn);
                    v = fma(d.reg_mu, (double)d.xu[e], v);
                } else {
                    v = fma(e < nn ? d.reg_mu : d.reg_de, (double)d.xu[e], adj_plane(d, e, 2 * nn));
                }
            } else if (e < mo_end) {
                v = d.off_scale * d.g_mo[e - maps_end];
            } else {
                continue;                                      // ring term: k_ext_ring_grad
            }
            d.gu[e] = (float)v;
        }
    }
}

// Item (slice, pixel block): the ring term's gradient off_scale * sum_a g_dl[a][k] for 64
// pixels k. The block's 16 wavefronts take every 16th angle (coalesced rows of g_dl), each
// with four independent partial sums so that its loads overlap; the partials are added in a
// fixed order (wavefront, then partial).
constexpr int kRingThreads = 1024, kRingPix = 64, kRingAcc = 4;
__global__ __launch_bounds__(kRingThreads) void k_ext_ring_grad(const SliceDesc* __restrict__ D,
                                                               const Item* __restrict__ items,
                                                               int n_items) {
    constexpr int NW = kRingThreads / kRingPix;
    __shared__ double part[NW][kRingPix];
    const int lane = threadIdx.x % kRingPix, wv = threadIdx.x / kRingPix;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        if (skipped_adj(d) || !(d.ext & EXT_RING)) continue;
        const int nd = d.n_det, nt = d.n_theta;
        const int k = w.y * kRingPix + lane;
        double acc[kRingAcc] = {0.0, 0.0, 0.0, 0.0};
        if (k < nd) {
            int a = wv;
            for (; a + (kRingAcc - 1) * NW < nt; a += kRingAcc * NW) {
#pragma unroll
                for (int q = 0; q < kRingAcc; ++q) acc[q] += d.g_dl[(size_t)(a + q * NW) * nd + k];
            }
            for (int q = 0; a < nt; a += NW, ++q) acc[q] += d.g_dl[(size_t)a * nd + k];
        }
        part[wv][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        __syncthreads();
        if (wv == 0 && k < nd) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) v += part[q][lane];
            const int64_t nn = (int64_t)d.n * d.n;
            const int64_t base = ((d.ext & EXT_HMODE) ? nn : 2 * nn) + ((d.ext & EXT_DRIFT) ? nt : 0);
            d.gu[base + k] = (float)(d.off_scale * v);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ eq. 3 single shot
// Item (slice, angle). h-mode with one mask position j0: r_k = s[a][j0][k] / f_k(m_j0), then
// T = circular convolution of r with the real kernel whose DFT is 1 / (1 + i beta sin q)
// (eq. 3 with the central difference's symbol; beta = kappa gamma f'/f of the detector-
// averaged flat, folded into the kernel on the host), R[h] = -log(max(T, 1e-6)) into the
// first sinogram plane, zeros into the second (the filtered backprojection follows).
constexpr int kEq3Threads = 256;
constexpr double kEq3TFloor = 1e-6;
__global__ __launch_bounds__(kEq3Threads) void k_eq3_retrieve(const SliceDesc* __restrict__ D,
                                                             const Item* __restrict__ items,
                                                             int n_items,
                                                             const double* __restrict__ kern,
                                                             const double* __restrict__ inv_flat,
                                                             int j0) {
    __shared__ double r[kExtMaxDet];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        const int a = w.y, nd = d.n_det;
        const float* se = d.s_exp + ((size_t)a * d.n_mask + j0) * nd;
        __syncthreads();
        for (int k = threadIdx.x; k < nd; k += kEq3Threads) r[k] = (double)se[k] * inv_flat[k];
        __syncthreads();
        float* P0 = d.P + (size_t)a * nd;
        float* P1 = d.P + ((size_t)d.n_theta + a) * nd;
        for (int k = threadIdx.x; k < nd; k += kEq3Threads) {
            double T = 0.0;
            for (int l = 0; l < nd; ++l) {
                const int src = k - l < 0 ? k - l + nd : k - l;
                T = fma(kern[l], r[src], T);
            }
            P0[k] = (float)(-log(fmax(T, kEq3TFloor)));
            P1[k] = 0.f;
        }
    }
}

// Item (slice, chunk) over the parameter vector: the parameter vector of a single-shot start
// from the backprojected planes in g: the maps (h alone in h-mode: the first plane), offsets 0.
__global__ __launch_bounds__(kVecThreads) void k_ext_take_maps(const SliceDesc* __restrict__ D,
                                                              const Item* __restrict__ items,
                                                              int n_items) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        const int64_t nn = (int64_t)d.n * d.n;
        const int64_t maps_end = (d.ext & EXT_HMODE) ? nn : 2 * nn;
        const int64_t e0 = (int64_t)w.y * kVecChunk, e1 = min(e0 + kVecChunk, d.nvu);
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kVecThreads)
            d.gu[e] = e < maps_end ? d.g[e] : 0.f;
    }
}

// ------------------------------------------------------------------------ launchers
hipError_t launch_ext_expand(const SliceDesc* D, const Item* items, int n_items, int grid,
                             hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_ext_expand<<<grid, kVecThreads, 0, s>>>(D, items, n_items);
    return hipGetLastError();
}
hipError_t launch_ic_ext(const SliceDesc* D, const Item* items, int n_items, int grid,
                         int want_seeds, int max_det, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (max_det < 1 || max_det > kExtMaxDet) return hipErrorInvalidValue;
    // G_Delta, then the single-map mu seeds (single-map slices have n_det <= kExtMaxDet / 2):
    // 2 max_det doubles, or kExtMaxDet when the widest slice is wider than that
    const size_t lds = sizeof(double) * (size_t)(max_det <= kExtMaxDet / 2 ? 2 * max_det : kExtMaxDet);
    if (max_det <= 256)
        k_ic_ext<256><<<grid, 256, lds, s>>>(D, items, n_items, want_seeds);
    else
        k_ic_ext<512><<<grid, 512, lds, s>>>(D, items, n_items, want_seeds);
    return hipGetLastError();
}
hipError_t launch_ext_contract(const SliceDesc* D, const Item* items, int n_items, int grid,
                               hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_ext_contract<<<grid, kVecThreads, 0, s>>>(D, items, n_items);
    return hipGetLastError();
}
hipError_t launch_ext_ring_grad(const SliceDesc* D, const Item* items, int n_items, int grid,
                                hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_ext_ring_grad<<<grid, kRingThreads, 0, s>>>(D, items, n_items);
    return hipGetLastError();
}
hipError_t launch_eq3_retrieve(const SliceDesc* D, const Item* items, int n_items, int grid,
                               const double* kern, const double* inv_flat, int mask_index,
                               hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_eq3_retrieve<<<grid, kEq3Threads, 0, s>>>(D, items, n_items, kern, inv_flat, mask_index);
    return hipGetLastError();
}
hipError_t launch_ext_take_maps(const SliceDesc* D, const Item* items, int n_items, int grid,
                                hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_ext_take_maps<<<grid, kVecThreads, 0, s>>>(D, items, n_items);
    return hipGetLastError();
}

}  // namespace eit
