// Image-quality measures of the combined-results and experiment sections, on the device:
// the Fourier ring correlation (eq. 6) with its resolution estimate, and the
// contrast-to-noise ratio (eq. 7).
//
// FRC(r) = sum_{ring r} Re(F1 F2*) / sqrt(sum_{ring r} |F1|^2 * sum_{ring r} |F2|^2) for two
// n x n images, F the 2-D DFT, ring r the integer frequencies (kx, ky) (DFT order, signed
// in [-n/2, n/2)) with round(sqrt(kx^2 + ky^2)) = r, r = 0 .. n/2. The curve is smoothed over
// rings 1 .. n/2 by a Gaussian of width sigma rings (weights renormalised at the ends) and the
// resolution is n / r_c pixels, r_c the first ring (linear interpolation) where the smoothed
// curve drops below the cutoff.
// The DFT runs as a row pass and a column pass (FP64, twiddles from a per-block LDS table),
// the ring sums in a fixed order (one block per ring), so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "eit_internal.h"
#include "eitomo.h"
#include "reduce.h"

namespace eit {

constexpr int kQThreads = 256;

__device__ __forceinline__ void twiddles(double2* tw, int n) {
    for (int m = threadIdx.x; m < n; m += blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)m / (double)n, &s, &c);
        tw[m] = make_double2(c, s);
    }
}

// Block per row j: R[img][j][kx] = sum_i x[img][j][i] e^{-2 pi i kx i / n} (img = 0, 1).
__global__ __launch_bounds__(kQThreads) void k_frc_rows(int n, const float* __restrict__ a,
                                                       const float* __restrict__ b,
                                                       double2* __restrict__ R) {
    extern __shared__ double2 sm[];
    double2* tw = sm;                                  // [n]
    double* row = (double*)(sm + n);                   // [2][n]
    const int j = blockIdx.x;
    twiddles(tw, n);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        row[i] = (double)a[(size_t)j * n + i];
        row[n + i] = (double)b[(size_t)j * n + i];
    }
    __syncthreads();
    for (int kx = threadIdx.x; kx < n; kx += blockDim.x) {
        double r0 = 0.0, i0 = 0.0, r1 = 0.0, i1 = 0.0;
        int idx = 0;
        for (int i = 0; i < n; ++i) {
            const double2 w = tw[idx];                 // e^{-i phi} = (cos, -sin)
            r0 = fma(row[i], w.x, r0);
            i0 = fma(-row[i], w.y, i0);
            r1 = fma(row[n + i], w.x, r1);
            i1 = fma(-row[n + i], w.y, i1);
            idx += kx;
            if (idx >= n) idx -= n;
        }
        R[(size_t)j * n + kx] = make_double2(r0, i0);
        R[(size_t)n * n + (size_t)j * n + kx] = make_double2(r1, i1);
    }
}

// Block per column kx: F[img][ky][kx] = sum_j R[img][j][kx] e^{-2 pi i ky j / n}, then the
// per-frequency products Q[ky][kx] = (Re F1 F2*, |F1|^2, |F2|^2).
__global__ __launch_bounds__(kQThreads) void k_frc_cols(int n, const double2* __restrict__ R,
                                                       double* __restrict__ Q) {
    extern __shared__ double2 sm[];
    double2* tw = sm;                                  // [n]
    double2* col = sm + n;                             // [2][n]
    const int kx = blockIdx.x;
    twiddles(tw, n);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        col[j] = R[(size_t)j * n + kx];
        col[n + j] = R[(size_t)n * n + (size_t)j * n + kx];
    }
    __syncthreads();
    for (int ky = threadIdx.x; ky < n; ky += blockDim.x) {
        double r0 = 0.0, i0 = 0.0, r1 = 0.0, i1 = 0.0;
        int idx = 0;
        for (int j = 0; j < n; ++j) {
            const double2 w = tw[idx];
            const double2 p = col[j], q = col[n + j];
            // (p.x + i p.y)(w.x - i w.y)
            r0 = fma(p.x, w.x, fma(p.y, w.y, r0));
            i0 = fma(p.y, w.x, fma(-p.x, w.y, i0));
            r1 = fma(q.x, w.x, fma(q.y, w.y, r1));
            i1 = fma(q.y, w.x, fma(-q.x, w.y, i1));
            idx += ky;
            if (idx >= n) idx -= n;
        }
        double* o = Q + 3 * ((size_t)ky * n + kx);
        o[0] = r0 * r1 + i0 * i1;
        o[1] = r0 * r0 + i0 * i0;
        o[2] = r1 * r1 + i1 * i1;
    }
}

__device__ __forceinline__ int signed_freq(int q, int n) { return 2 * q < n ? q : q - n; }
__device__ __forceinline__ int freq_index(int k, int n) { return k >= 0 ? k : k + n; }

// Block per ring r: sums of Q over the ring (each thread a set of ky rows, the |kx| interval of
// the ring on that row, every candidate checked by the exact rounding test), then FRC(r).
__global__ __launch_bounds__(kQThreads) void k_frc_rings(int n, const double* __restrict__ Q,
                                                        double* __restrict__ curve) {
    __shared__ double red[kQThreads / 64];
    const int r = blockIdx.x;
    const double lo = r - 0.5, hi = r + 0.5;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int qy = threadIdx.x; qy < n; qy += blockDim.x) {
        const int ky = signed_freq(qy, n);
        const double rem_hi = hi * hi - (double)ky * ky;
        if (rem_hi <= 0.0) continue;
        const int kmax = (int)floor(sqrt(rem_hi)) + 1;
        const double rem_lo = lo * lo - (double)ky * ky;
        const int kmin = rem_lo > 0.0 ? max((int)floor(sqrt(rem_lo)) - 1, 0) : 0;
        for (int ak = kmin; ak <= kmax; ++ak)
            for (int sgn = 0; sgn < (ak == 0 ? 1 : 2); ++sgn) {
                const int kx = sgn ? -ak : ak;
                if (2 * kx >= n || 2 * kx < -n) continue;            // not a DFT frequency
                const double rad = sqrt((double)kx * kx + (double)ky * ky);
                if ((int)rint(rad) != r) continue;
                const double* o = Q + 3 * ((size_t)qy * n + freq_index(kx, n));
                s0 += o[0];
                s1 += o[1];
                s2 += o[2];
            }
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
        const double den = sqrt(s1 * s2);
        curve[r] = den > 0.0 ? s0 / den : 0.0;
    }
}

// One block: Gaussian smoothing over rings 1 .. nr-1 and the cutoff crossing.
__global__ __launch_bounds__(kQThreads) void k_frc_resolution(int n, int nr, const double* __restrict__ curve,
                                                             double* __restrict__ smooth, double sigma,
                                                             double cutoff, double* __restrict__ res) {
    for (int q = threadIdx.x; q < nr; q += blockDim.x) {
        if (q == 0) { smooth[0] = curve[0]; continue; }
        double num = 0.0, den = 0.0;
        for (int r = 1; r < nr; ++r) {
            const double t = (double)(r - q) / sigma;
            const double w = exp(-0.5 * t * t);
            num = fma(w, curve[r], num);
            den += w;
        }
        smooth[q] = num / den;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double rc = (double)(nr - 1);
    for (int q = 1; q < nr; ++q)
        if (smooth[q] < cutoff) {
            rc = q == 1 ? 1.0 : (q - 1) + (smooth[q - 1] - cutoff) / (smooth[q - 1] - smooth[q]);
            break;
        }
    res[0] = (double)n / rc;
    res[1] = rc;
}

// One block: CNR of the two discs (pixel centres within rho of (x, y), centred coordinates),
// means first, then the population variances about them.
__global__ __launch_bounds__(kQThreads) void k_cnr(int n, const float* __restrict__ img, double x1,
                                                  double y1, double x2, double y2, double rho,
                                                  double* __restrict__ out) {
    __shared__ double red[kQThreads / 64];
    const double c = 0.5 * (n - 1), r2 = rho * rho;
    double cnt[2] = {0.0, 0.0}, sum[2] = {0.0, 0.0};
    const double cx[2] = {x1, x2}, cy[2] = {y1, y2};
    for (size_t e = threadIdx.x; e < (size_t)n * n; e += blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        for (int d = 0; d < 2; ++d) {
            const double dx = i - c - cx[d], dy = j - c - cy[d];
            if (dx * dx + dy * dy <= r2) { cnt[d] += 1.0; sum[d] += (double)img[e]; }
        }
    }
    double mean[2];
    for (int d = 0; d < 2; ++d) {
        const double nc = block_sum(cnt[d], red);
        mean[d] = block_sum(sum[d], red) / nc;
        cnt[d] = nc;
    }
    double var[2] = {0.0, 0.0};
    for (size_t e = threadIdx.x; e < (size_t)n * n; e += blockDim.x) {
        const int i = (int)(e % n), j = (int)(e / n);
        for (int d = 0; d < 2; ++d) {
            const double dx = i - c - cx[d], dy = j - c - cy[d];
            if (dx * dx + dy * dy <= r2) {
                const double v = (double)img[e] - mean[d];
                var[d] = fma(v, v, var[d]);
            }
        }
    }
    for (int d = 0; d < 2; ++d) var[d] = block_sum(var[d], red) / cnt[d];
    if (threadIdx.x == 0) out[0] = fabs(mean[0] - mean[1]) / sqrt(var[0] + var[1]);
}

}  // namespace eit

namespace {
size_t frc_bytes(int n) {
    const size_t nn = (size_t)n * n;
    return 2 * nn * sizeof(double2) + 3 * nn * sizeof(double);
}
int qfail(int code, const char* msg);
}  // namespace

namespace eit {
int report_failure(int code, const char* msg);
}

namespace {
int qfail(int code, const char* msg) { return eit::report_failure(code, msg); }
}  // namespace

extern "C" size_t eit_frc_workspace_bytes(int32_t n) {
    if (n < 2 || n > EIT_MAX_FRC_N) return 0;
    return frc_bytes(n);
}

extern "C" int eit_frc(int32_t n, const float* a, const float* b, double* curve, double* smooth,
                       double* res, double cutoff, double sigma, void* ws, size_t ws_bytes,
                       void* stream) {
    using namespace eit;
    if (n < 2 || n > EIT_MAX_FRC_N) return qfail(EIT_ERR_SHAPE, "FRC image size outside [2, EIT_MAX_FRC_N]");
    if (!a || !b || !curve || !smooth || !res || !ws)
        return qfail(EIT_ERR_INVALID_ARG, "FRC: a NULL pointer");
    if (!(sigma > 0.0) || !std::isfinite(sigma) || !std::isfinite(cutoff))
        return qfail(EIT_ERR_INVALID_ARG, "FRC: sigma must be finite and > 0, cutoff finite");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return qfail(EIT_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (ws_bytes < frc_bytes(n)) return qfail(EIT_ERR_NOMEM, "FRC workspace too small");
    hipStream_t st = (hipStream_t)stream;
    double2* R = (double2*)ws;
    double* Q = (double*)(R + 2 * (size_t)n * n);
    const int nr = n / 2 + 1;
    k_frc_rows<<<n, kQThreads, (size_t)n * sizeof(double2) + 2 * (size_t)n * sizeof(double), st>>>(n, a, b, R);
    if (hipGetLastError() != hipSuccess) return qfail(EIT_ERR_DEVICE, "FRC row pass launch failed");
    k_frc_cols<<<n, kQThreads, 3 * (size_t)n * sizeof(double2), st>>>(n, R, Q);
    if (hipGetLastError() != hipSuccess) return qfail(EIT_ERR_DEVICE, "FRC column pass launch failed");
    k_frc_rings<<<nr, kQThreads, 0, st>>>(n, Q, curve);
    if (hipGetLastError() != hipSuccess) return qfail(EIT_ERR_DEVICE, "FRC ring pass launch failed");
    k_frc_resolution<<<1, kQThreads, 0, st>>>(n, nr, curve, smooth, sigma, cutoff, res);
    if (hipGetLastError() != hipSuccess) return qfail(EIT_ERR_DEVICE, "FRC resolution launch failed");
    return EIT_OK;
}

extern "C" int eit_cnr(int32_t n, const float* img, double x1, double y1, double x2, double y2,
                       double rho, double* out, void* stream) {
    using namespace eit;
    if (n < 1 || n > EIT_MAX_N) return qfail(EIT_ERR_SHAPE, "CNR image size outside [1, EIT_MAX_N]");
    if (!img || !out) return qfail(EIT_ERR_INVALID_ARG, "CNR: a NULL pointer");
    if (!(rho > 0.0) || !std::isfinite(rho) || !std::isfinite(x1) || !std::isfinite(y1) ||
        !std::isfinite(x2) || !std::isfinite(y2))
        return qfail(EIT_ERR_INVALID_ARG, "CNR: centres must be finite and rho > 0");
    // both discs must hold a pixel centre: checked on the host
    const double c = 0.5 * (n - 1);
    for (int d = 0; d < 2; ++d) {
        const double x = d ? x2 : x1, y = d ? y2 : y1;
        bool any = false;
        const int i0 = std::max(0, (int)std::floor(c + x - rho)), i1 = std::min(n - 1, (int)std::ceil(c + x + rho));
        const int j0 = std::max(0, (int)std::floor(c + y - rho)), j1 = std::min(n - 1, (int)std::ceil(c + y + rho));
        for (int j = j0; j <= j1 && !any; ++j)
            for (int i = i0; i <= i1 && !any; ++i) {
                const double dx = i - c - x, dy = j - c - y;
                any = dx * dx + dy * dy <= rho * rho;
            }
        if (!any) return qfail(EIT_ERR_INVALID_ARG, "CNR: a disc holds no pixel centre");
    }
    k_cnr<<<1, kQThreads, 0, (hipStream_t)stream>>>(n, img, x1, y1, x2, y2, rho, out);
    if (hipGetLastError() != hipSuccess) return qfail(EIT_ERR_DEVICE, "CNR launch failed");
    return EIT_OK;
}
