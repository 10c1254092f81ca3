// Non-iterative ("single shot") reconstruction: retrieval of transmission and refraction
// from each pixel's illumination curve, ramp filtering, backprojection. It serves as the
// input of the learned warm start.
//
// Retrieval (per projection pixel (a, k), FP64): with y_j = log s_j - log A_k +
// (m_j - c_k)^2 / (2 s_k^2), the model s_j = T A_k exp(-(m_j - Delta - c_k)^2 / (2 s_k^2))
// is the line y_j = alpha + beta (m_j - c_k), beta = Delta / s_k^2,
// alpha = log T - Delta^2 / (2 s_k^2); a fit weighted by w_j = s_j (Poisson: var(log s) ~ 1/s)
// gives Delta = beta s_k^2 and log T = alpha + Delta^2 / (2 s_k^2). Samples with s_j <= 0 get
// zero weight; a singular fit gives T = 1, Delta = 0.
// Channels: P_mu = -log T; P_delta = trapezoid integral of Delta / kappa along t minus the
// linear ramp that makes both ends zero (the refraction is the detector derivative of the
// projected phase).
// Filtering: Ram-Lak kernel of Kak & Slaney for unit spacing, h[0] = 1/4,
// h[odd n] = -1/(pi^2 n^2), h[even n != 0] = 0, linear (zero-padded) convolution along t,
// scaled by pi / n_theta; then the gather backprojector.
#include "device_common.h"

namespace eit {

constexpr int kSsThreads = 256;

// Item (slice, angle). Reads s_exp and the flat parameters (the plan's float tables are
// FP32; the fit itself runs in FP64), writes the two retrieved sinogram rows into d.P.
__global__ __launch_bounds__(kSsThreads) void k_ss_retrieve(const SliceDesc* __restrict__ D,
                                                           const Item* __restrict__ items,
                                                           int n_items) {
    __shared__ double q[4096];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        const int a = w.y, nd = d.n_det, M = d.n_mask;
        const float* se = d.s_exp + (size_t)a * M * nd;
        float* Pm = d.P + (size_t)a * nd;
        float* Pd = d.P + ((size_t)d.n_theta + a) * nd;
        for (int k = threadIdx.x; k < nd; k += kSsThreads) {
            const float4 fl = d.flat[k];           // A, c, 1/(2 s^2), 1/s^2
            const double h2 = (double)fl.z, logA = log((double)fl.x);
            double S0 = 0, S1 = 0, S2 = 0, Y0 = 0, Y1 = 0;
            for (int j = 0; j < M; ++j) {
                const double s = (double)se[(size_t)j * nd + k];
                if (!(s > 0.0)) continue;
                const double x = (double)d.mask[j] - (double)fl.y;
                const double y = log(s) - logA + x * x * h2;
                S0 += s; S1 += s * x; S2 += s * x * x; Y0 += s * y; Y1 += s * x * y;
            }
            const double det = S0 * S2 - S1 * S1;
            double logT = 0.0, dl = 0.0;
            if (det > 1e-12 * fmax(S0 * S2, 1e-300)) {
                const double alpha = (S2 * Y0 - S1 * Y1) / det;
                const double beta = (S0 * Y1 - S1 * Y0) / det;
                const double s2 = 1.0 / (double)fl.w;              // sigma^2
                dl = beta * s2;
                logT = alpha + dl * dl / (2.0 * s2);
            }
            Pm[k] = (float)(-logT);
            q[k] = dl / (double)d.kappa;
        }
        __syncthreads();
        if (threadIdx.x == 0) {               // trapezoid cumulative sum, fixed order
            double acc = 0.0, prev = q[0];
            q[0] = 0.0;
            for (int k = 1; k < nd; ++k) {
                const double cur = q[k];
                acc += 0.5 * (prev + cur);
                prev = cur;
                q[k] = acc;
            }
        }
        __syncthreads();
        const double last = q[nd - 1];
        for (int k = threadIdx.x; k < nd; k += kSsThreads)
            Pd[k] = (float)(q[k] - last * (double)k / (double)(nd > 1 ? nd - 1 : 1));
        __syncthreads();
    }
}

// Item (slice, angle). Ram-Lak filter of both sinogram rows of the angle in d.P, in place
// (the row is staged in LDS first), scaled by pi / n_theta (FP64 accumulation: the filter
// output is a difference of sums).
__global__ __launch_bounds__(kSsThreads) void k_ss_filter(const SliceDesc* __restrict__ D,
                                                         const Item* __restrict__ items,
                                                         int n_items) {
    __shared__ double row[4096];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x)
    for (int c = 0; c < 2; ++c) {
        const Item w = items[it];
        const SliceDesc& d = D[w.x];
        const int a = w.y, nd = d.n_det;
        const float* in = d.P + ((size_t)c * d.n_theta + a) * nd;
        __syncthreads();
        for (int k = threadIdx.x; k < nd; k += kSsThreads) row[k] = (double)in[k];
        __syncthreads();
        const double scale = M_PI / (double)d.n_theta;
        const double ipi2 = 1.0 / (M_PI * M_PI);
        for (int k = threadIdx.x; k < nd; k += kSsThreads) {
            double acc = 0.25 * row[k];
            // odd offsets only: k' = k - n for n = +-1, +-3, ...
            for (int n = 1; n <= nd; n += 2) {
                const double hn = -ipi2 / ((double)n * (double)n);
                double v = 0.0;
                if (k - n >= 0) v += row[k - n];
                if (k + n < nd) v += row[k + n];
                acc = fma(hn, v, acc);
            }
            d.P[((size_t)c * d.n_theta + a) * nd + k] = (float)(scale * acc);
        }
    }
}

hipError_t launch_ss_retrieve(const SliceDesc* D, const Item* items, int n_items, int grid,
                              hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_ss_retrieve<<<grid, kSsThreads, 0, s>>>(D, items, n_items);
    return hipGetLastError();
}

hipError_t launch_ss_filter(const SliceDesc* D, const Item* items, int n_items, int grid,
                            hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    k_ss_filter<<<grid, kSsThreads, 0, s>>>(D, items, n_items);
    return hipGetLastError();
}

}  // namespace eit
