// C ABI of the EI tomography library (declared in include/eitomo.h): host-side validation,
// FP64 table construction, workspace layout, launch sequencing and the reconstruction
// driver (one captured HIP graph per cost/gradient evaluation, replayed until the
// device-side optimiser reports completion).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "eit_internal.h"
#include "eitomo.h"

using namespace eit;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(EIT_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

namespace eit {
// Error reporting for the library's other translation units.
int report_failure(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace eit

namespace {

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    }
};

// Projector variants tried in order when the caller does not choose one; the last (one
// angle per group, window <= 64/cos(45 deg) + 16 + 4 columns) fits every geometry.
const int kProjPrefSmall[] = {1, 7, 8};
const int kProjPrefLarge[] = {0, 1, 7, 8};
int default_adj_variant(int n) { (void)n; return 0; }

int grid_for(int n_items, int cap) { return std::max(1, std::min(n_items, cap)); }
constexpr int kGridCap = 256 * 16;   // persistent-grid cap: CUs x resident blocks

// Adjoint angle split: automatic choice doubles the split while the launch has fewer than
// kSplitTarget blocks (4 per CU) and every part keeps at least 2 angle chunks.
constexpr int kSplitTarget = 1024;
constexpr int kMaxSplits = 64;
int auto_splits(int tiles, int nchunks) {
    int g = 1;
    while (tiles * g < kSplitTarget && 2 * g <= std::min(8, nchunks / 2)) g *= 2;
    return g;
}

}  // namespace

// ============================================================================ plan
struct eit_plan {
    int n, n_theta, n_det, n_mask;
    double kappa;
    int proj_v, adj_v;
    ProjTile pt;
    AdjTile at;
    int n_groups, n_dblk, n_strips, win_w, win_shift;
    size_t proj_lds;
    int n_tx, n_ty, kwin;
    int adj_splits;        // adjoint blocks per voxel tile (angle ranges)
    int n_pairs;           // mirror-pair adjoint: angle pair slots (0 otherwise)
    int n_trx;             // transpose tiles per side
    int64_t nv;            // 2 n^2
    int n_vblocks;
    // device tables
    ProjAngle* pang = nullptr;
    int32_t* groups = nullptr;
    int32_t* win_lo = nullptr;
    AdjAngle* aang = nullptr;
    int2* apairs = nullptr;
    float4* flat = nullptr;
    double* mask = nullptr;
    // single-slice item lists (slice 0)
    Item* it_tr = nullptr;
    Item* it_pr = nullptr;
    Item* it_ic = nullptr;
    Item* it_bp = nullptr;
    Item* it_vec = nullptr;
    int n_it_tr, n_it_pr, n_it_ic, n_it_bp, n_it_vec;
    int device;
    // full model of eq. 4 (ext == 0: the plain two-map model of eq. 2)
    int ext = 0;
    int n_maps = 2;        // maps in the parameter vector (1 in h-mode)
    int eval_maps = 2;     // maps the kernels evaluate: 1 in h-mode (R h once), else 2
    double gamma = 0.0;    // h-mode: delta = gamma h
    double off_scale = 1.0;
    int nq = 0;            // tabulated flat samples per pixel
    double tab_u0 = 0.0, tab_du = 0.0;
    int eq3_mask = 0;
    bool gauss = true;     // Gaussian flat parameters given (the two-map single shot needs them)
    int64_t nvu = 0;       // parameter-vector entries (= nv for the plain model)
    double* ftab = nullptr;       // [n_det][nq]
    double* eq3_kern = nullptr;   // [n_det] circular kernel of eq. 3 (h-mode)
    double* eq3_invf = nullptr;   // [n_det] 1 / f_k(m_j0)
    Item* it_uvec = nullptr;      // chunks of the parameter vector
    Item* it_hvec = nullptr;      // chunks of one map
    Item* it_ring = nullptr;      // pixel blocks of the ring term's gradient
    Item* it_cvec = nullptr;      // small chunks of the parameter vector (contraction)
    int n_it_uvec = 0, n_it_hvec = 0, n_it_ring = 0, n_it_cvec = 0;
};

namespace {

template <class T>
int upload(T** dst, const std::vector<T>& v) {
    *dst = nullptr;
    if (v.empty()) return EIT_OK;
    HIP_TRY(hipMalloc((void**)dst, v.size() * sizeof(T)));
    HIP_TRY(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return EIT_OK;
}

void free_plan(eit_plan* p) {
    if (!p) return;
    void* ptrs[] = {p->pang, p->groups, p->win_lo, p->aang, p->apairs, p->flat, p->mask,
                    p->it_tr, p->it_pr, p->it_ic, p->it_bp, p->it_vec, p->ftab, p->eq3_kern,
                    p->eq3_invf, p->it_uvec, p->it_hvec, p->it_ring, p->it_cvec};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Projector angle record in the stepping frame (see ProjAngle).
ProjAngle make_pangle(double th, int n, bool row) {
    const double c = 0.5 * (n - 1);
    const double cs = std::cos(th), sn = std::sin(th);
    ProjAngle a{};
    if (row) {
        a.inv = 1.0 / cs;
        a.base = c * sn / cs + c;
        a.slope = -sn / cs;
        a.w = (float)(1.0 / std::fabs(cs));
        a.src = 0;
    } else {
        a.inv = 1.0 / sn;
        a.base = c * cs / sn + c;
        a.slope = -cs / sn;
        a.w = (float)(1.0 / std::fabs(sn));
        a.src = 1;
    }
    a.slope_f = (float)a.slope;
    return a;
}

// Mirror pairs for the mirror-pair adjoint: angle b is the mirror of a when cos b = -cos a and
// sin b = sin a (to 1e-12), i.e. b = pi - a as a set of lines. Angles are taken in order; an
// angle not yet used is paired with the first unused later angle that mirrors it. mate[a] is
// that partner (a first of a pair), -1 (no partner in the set), or -2 (second of a pair).
void mirror_pairs(const std::vector<double>& theta, std::vector<int32_t>& mate) {
    const int nt = (int)theta.size();
    std::vector<int> order(nt);
    std::vector<double> cs(nt), sn(nt);
    for (int a = 0; a < nt; ++a) {
        order[a] = a;
        cs[a] = std::cos(theta[a]);
        sn[a] = std::sin(theta[a]);
    }
    // candidates sorted by sin, then index: a mirror has the same sin
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        return sn[x] < sn[y] || (sn[x] == sn[y] && x < y);
    });
    std::vector<double> key(nt);
    for (int q = 0; q < nt; ++q) key[q] = sn[order[q]];
    const double tol = 1e-12;
    mate.assign(nt, -1);
    for (int a = 0; a < nt; ++a) {
        if (mate[a] != -1) continue;
        const int lo = (int)(std::lower_bound(key.begin(), key.end(), sn[a] - tol) - key.begin());
        int best = -1;
        for (int q = lo; q < nt && key[q] <= sn[a] + tol; ++q) {
            const int b = order[q];
            if (b > a && mate[b] == -1 && std::fabs(cs[b] + cs[a]) <= tol && (best < 0 || b < best))
                best = b;
        }
        if (best >= 0) {
            mate[a] = best;
            mate[best] = -2;
        }
    }
}

}  // namespace

namespace {

struct HostTables {
    std::vector<ProjAngle> pang;
    std::vector<int32_t> groups, win_lo;
    std::vector<AdjAngle> aang;
    std::vector<int2> apairs;
    std::vector<int32_t> mate;     // per angle: mirror partner (first of a pair), -1, or -2
    std::vector<float4> flat;
    std::vector<double> maskd;
    std::vector<Item> it_tr, it_pr, it_ic, it_bp, it_vec;
    std::vector<double> ftab, eq3_kern, eq3_invf;
    std::vector<Item> it_uvec, it_hvec, it_ring, it_cvec;
};

// Cubic-convolution value and slope (Keys 1981, a = -1/2) of a tabulated flat row F[0..Q) at u,
// held at the end values (slope 0) outside the scanned period.
void table_flat(const double* F, int Q, double u0, double du, double u, double* f, double* fp) {
    const double lo = u0, hi = u0 + (Q - 1) * du;
    const bool inside = u >= lo && u <= hi;
    const double xq = (std::min(std::max(u, lo), hi) - lo) / du;
    const int q = std::min(std::max((int)std::floor(xq), 0), Q - 2);
    const double t = xq - q, t2 = t * t, t3 = t2 * t;
    const double F0 = F[std::max(q - 1, 0)], F1 = F[q], F2 = F[q + 1], F3 = F[std::min(q + 2, Q - 1)];
    *f = 0.5 * ((-t3 + 2 * t2 - t) * F0 + (3 * t3 - 5 * t2 + 2) * F1 + (-3 * t3 + 4 * t2 + t) * F2 +
                (t3 - t2) * F3);
    *fp = inside ? 0.5 * ((-3 * t2 + 4 * t - 1) * F0 + (9 * t2 - 10 * t) * F1 +
                          (-9 * t2 + 8 * t + 1) * F2 + (3 * t2 - 2 * t) * F3) / du
                 : 0.0;
}

// Model options: validation and the full model's tables (touches no device).
int build_model(const eit_setup* setup, const eit_model* m, eit_plan* p, HostTables& h,
                const std::vector<double>& mpos) {
    const int nt = p->n_theta, nd = p->n_det;
    p->ext = 0;
    p->n_maps = 2;
    p->eval_maps = 2;
    p->nvu = p->nv;
    if (!m) return EIT_OK;
    if (m->hmode) {
        if (!finite_pos(m->gamma)) return fail(EIT_ERR_INVALID_ARG, "h-mode gamma must be finite and > 0");
        p->ext |= EXT_HMODE;
        p->gamma = m->gamma;
        p->n_maps = 1;
        p->eval_maps = nd <= kSingleMapMaxDet ? 1 : 2;
    }
    if (m->fit_drift) p->ext |= EXT_DRIFT;
    if (m->fit_ring) p->ext |= EXT_RING;
    if (m->offset_scale != 0.0 && !finite_pos(m->offset_scale))
        return fail(EIT_ERR_INVALID_ARG, "offset_scale must be finite and > 0 (or 0 for 1)");
    p->off_scale = m->offset_scale > 0.0 ? m->offset_scale : 1.0;
    if (m->n_table != 0) {
        if (m->n_table < 4 || m->n_table > EIT_MAX_NTABLE)
            return fail(EIT_ERR_SHAPE, "n_table=%d outside [4, %d]", m->n_table, EIT_MAX_NTABLE);
        if (!m->flat_table) return fail(EIT_ERR_INVALID_ARG, "flat_table is NULL");
        if (!std::isfinite(m->table_u0) || !finite_pos(m->table_du))
            return fail(EIT_ERR_INVALID_ARG, "table_u0 must be finite and table_du finite and > 0");
        const size_t cnt = (size_t)nd * m->n_table;
        for (size_t i = 0; i < cnt; ++i)
            if (!std::isfinite(m->flat_table[i])) return fail(EIT_ERR_INVALID_ARG, "flat_table[%zu] not finite", i);
        p->ext |= EXT_TABLE;
        p->nq = m->n_table;
        p->tab_u0 = m->table_u0;
        p->tab_du = m->table_du;
        h.ftab.assign(m->flat_table, m->flat_table + cnt);
    }
    if (m->eq3_mask < 0 || m->eq3_mask >= p->n_mask)
        return fail(EIT_ERR_INVALID_ARG, "eq3_mask=%d outside [0, n_mask)", m->eq3_mask);
    p->eq3_mask = m->eq3_mask;
    if (!(p->ext & EXT_TABLE) && !p->gauss)
        return fail(EIT_ERR_INVALID_ARG, "flat-field IC parameters are NULL and no table is given");
    p->nvu = (int64_t)p->n_maps * p->n * p->n + ((p->ext & EXT_DRIFT) ? nt : 0) +
             ((p->ext & EXT_RING) ? nd : 0);
    if (p->ext & EXT_HMODE) {
        // eq. 3: r = s / f_k(m_j0) convolved with the real kernel whose DFT is
        // 1 / (1 + i beta sin(2 pi q / n_det)), beta = kappa gamma f'/f of the detector-averaged flat
        const double mj = mpos[p->eq3_mask];
        std::vector<double> f(nd), fp(nd);
        double fs = 0.0, fps = 0.0;
        for (int k = 0; k < nd; ++k) {
            if (p->ext & EXT_TABLE) {
                table_flat(&h.ftab[(size_t)k * p->nq], p->nq, p->tab_u0, p->tab_du, mj, &f[k], &fp[k]);
            } else {
                const double uu = mj - setup->flat_ctr[k], sg = setup->flat_sigma[k];
                f[k] = setup->flat_amp[k] * std::exp(-uu * uu / (2.0 * sg * sg));
                fp[k] = -uu / (sg * sg) * f[k];
            }
            fs += f[k];
            fps += fp[k];
        }
        const double beta = fs != 0.0 ? p->kappa * p->gamma * (fps / nd) / (fs / nd) : 0.0;
        h.eq3_invf.resize(nd);
        for (int k = 0; k < nd; ++k) h.eq3_invf[k] = f[k] > 0.0 ? 1.0 / f[k] : 0.0;
        h.eq3_kern.assign(nd, 0.0);
        for (int q = 0; q < nd; ++q) {
            const double sq = std::sin(2.0 * M_PI * q / nd);
            const double den = 1.0 + beta * beta * sq * sq;
            for (int l = 0; l < nd; ++l) {
                const double ph = 2.0 * M_PI * (double)(((long long)q * l) % nd) / nd;
                h.eq3_kern[l] += (std::cos(ph) + beta * sq * std::sin(ph)) / den;
            }
        }
        for (int l = 0; l < nd; ++l) h.eq3_kern[l] /= nd;
    }
    return EIT_OK;
}

// Validation and FP64 table construction; touches no device (testable on the host).
int build_host(const eit_dims* dims, const eit_setup* setup, const eit_tiling* tiling,
               eit_plan* p, HostTables& h, const eit_model* model = nullptr) {
    if (!dims || !setup) return fail(EIT_ERR_INVALID_ARG, "dims or setup is NULL");
    const int n = dims->n, nt = dims->n_theta, nd = dims->n_det, nm = dims->n_mask;
    if (n < 2 || n > EIT_MAX_N) return fail(EIT_ERR_SHAPE, "n=%d outside [2, %d]", n, EIT_MAX_N);
    if (nt < 1 || nt > EIT_MAX_NTHETA)
        return fail(EIT_ERR_SHAPE, "n_theta=%d outside [1, %d]", nt, EIT_MAX_NTHETA);
    if (nd < 2 || nd > EIT_MAX_NDET)
        return fail(EIT_ERR_SHAPE, "n_det=%d outside [2, %d]", nd, EIT_MAX_NDET);
    if (nm < 1 || nm > EIT_MAX_NMASK)
        return fail(EIT_ERR_SHAPE, "n_mask=%d outside [1, %d]", nm, EIT_MAX_NMASK);
    if (!std::isfinite(dims->kappa)) return fail(EIT_ERR_INVALID_ARG, "kappa is not finite");
    p->gauss = setup->flat_amp && setup->flat_ctr && setup->flat_sigma;
    if (!p->gauss && !(model && model->n_table != 0))
        return fail(EIT_ERR_INVALID_ARG, "flat-field IC parameters are NULL");
    std::vector<double> theta(nt), mpos(nm);
    for (int a = 0; a < nt; ++a) {
        theta[a] = setup->theta ? setup->theta[a] : a * M_PI / nt;
        if (!std::isfinite(theta[a])) return fail(EIT_ERR_INVALID_ARG, "theta[%d] not finite", a);
    }
    for (int j = 0; j < nm; ++j) {
        mpos[j] = setup->mask_pos ? setup->mask_pos[j] : (j + 0.5) / nm - 0.5;
        if (!std::isfinite(mpos[j])) return fail(EIT_ERR_INVALID_ARG, "mask_pos[%d] not finite", j);
    }
    for (int k = 0; k < nd && p->gauss; ++k) {
        if (!finite_pos(setup->flat_amp[k]) || !finite_pos(setup->flat_sigma[k]) ||
            !std::isfinite(setup->flat_ctr[k]))
            return fail(EIT_ERR_INVALID_ARG, "flat-field parameters of pixel %d invalid", k);
    }
    const bool pv_given = tiling && tiling->proj_variant >= 0;
    int pv = pv_given ? tiling->proj_variant : (n <= 128 ? kProjPrefSmall[0] : kProjPrefLarge[0]);
    int av = tiling && tiling->adj_variant >= 0 ? tiling->adj_variant : default_adj_variant(n);
    if (pv >= proj_variant_count()) return fail(EIT_ERR_INVALID_ARG, "proj_variant %d unknown", pv);
    if (av >= adj_variant_count()) return fail(EIT_ERR_INVALID_ARG, "adj_variant %d unknown", av);
    if (!pv_given) {
        // first preferred variant whose staging window fits
        const int* pref = n <= 128 ? kProjPrefSmall : kProjPrefLarge;
        const int np = n <= 128 ? 3 : 4;
        for (int q = 0; q < np; ++q) {
            eit_tiling t{pref[q], av, tiling ? tiling->adj_splits : 0};
            eit_plan probe{};
            HostTables hh;
            const std::string keep = g_err;
            if (build_host(dims, setup, &t, &probe, hh, model) == EIT_OK) { pv = pref[q]; break; }
            g_err = keep;
        }
    }
    p->n = n; p->n_theta = nt; p->n_det = nd; p->n_mask = nm; p->kappa = dims->kappa;
    p->proj_v = pv; p->adj_v = av; p->device = -1;
    p->pt = proj_variant(pv);
    p->at = adj_variant(av);
    const int A = p->pt.A, W = p->pt.W, R = p->pt.R;

    // ---- projector tables: row/column flag decided once here in FP64 (ties -> rows)
    std::vector<ProjAngle>& pang = h.pang;
    pang.assign(nt, ProjAngle{});
    std::vector<int> cls(nt);
    for (int a = 0; a < nt; ++a) {
        const double cs = std::cos(theta[a]), sn = std::sin(theta[a]);
        const bool row = std::fabs(cs) >= std::fabs(sn);
        pang[a] = make_pangle(theta[a], n, row);
        cls[a] = (row ? 0 : 2) + (pang[a].inv > 0 ? 0 : 1);
    }
    // groups: runs of consecutive angles of one class, chunked by A
    std::vector<int32_t>& groups = h.groups;
    groups.clear();
    for (int a = 0; a < nt;) {
        int b = a;
        while (b < nt && cls[b] == cls[a] && b - a < A) ++b;
        for (int q = 0; q < A; ++q) groups.push_back(a + q < b ? a + q : -1);
        a = b;
    }
    p->n_groups = (int)groups.size() / A;
    p->n_dblk = (nd + W - 1) / W;
    p->n_strips = (n + R - 1) / R;
    std::vector<int32_t>& win_lo = h.win_lo;
    win_lo.assign((size_t)p->n_groups * p->n_dblk * p->n_strips, 0);
    int win_w = 2;
    for (int g = 0; g < p->n_groups; ++g)
        for (int b = 0; b < p->n_dblk; ++b) {
            const int k0 = b * W, k1 = std::min(b * W + W - 1, nd - 1);
            const double t0 = k0 - 0.5 * (nd - 1), t1 = k1 - 0.5 * (nd - 1);
            for (int s = 0; s < p->n_strips; ++s) {
                const double p0 = (double)s * R, p1 = p0 + R - 1;
                double umin = 1e300, umax = -1e300;
                for (int q = 0; q < A; ++q) {
                    const int a = groups[(size_t)g * A + q];
                    if (a < 0) continue;
                    const ProjAngle& pa = pang[a];
                    for (double t : {t0, t1})
                        for (double pp : {p0, p1}) {
                            const double u = t * pa.inv + pa.base + pp * pa.slope;
                            umin = std::min(umin, u);
                            umax = std::max(umax, u);
                        }
                }
                const int lo = (int)std::floor(umin - 1e-3) - 1;
                win_lo[((size_t)g * p->n_dblk + b) * p->n_strips + s] = lo;
                win_w = std::max(win_w, (int)std::floor(umax + 1e-3) - lo + 2);
            }
        }
    p->win_w = win_w;
    p->win_shift = 0;
    while ((1 << p->win_shift) < p->pt.PW) ++p->win_shift;
    p->proj_lds = (size_t)R * (size_t)p->pt.LP * (p->pt.DUP ? sizeof(float4) : sizeof(float2));
    if (win_w > p->pt.LP) {
        return fail(EIT_ERR_SHAPE, "projector window %d wider than variant %d's pitch %d", win_w,
                    pv, p->pt.LP);
    }

    // ---- adjoint tables
    std::vector<AdjAngle>& aang = h.aang;
    aang.assign(nt, AdjAngle{});
    double span = 0.0;
    const double c = 0.5 * (n - 1), cdet = 0.5 * (nd - 1);
    for (int a = 0; a < nt; ++a) {
        const double cs = std::cos(theta[a]), sn = std::sin(theta[a]);
        const bool row = std::fabs(cs) >= std::fabs(sn);
        const double wv = row ? std::fabs(cs) : std::fabs(sn);
        AdjAngle q{};
        q.cs = cs; q.sn = sn; q.cd = cdet - c * (cs + sn);
        q.cd_s = cdet - c * (-cs + sn);
        q.cs_f = (float)cs; q.sn_f = (float)sn;
        q.iw = (float)(1.0 / wv);
        q.iw2 = (float)(1.0 / (wv * wv));
        q.iwm = (float)(1.0 / wv - 1.0 / (wv * wv));
        q.omw = (float)(1.0 - 1.0 / wv);
        aang[a] = q;
        span = std::max(span, (p->at.TX - 1) * std::fabs(cs) + (p->at.TY - 1) * std::fabs(sn));
    }
    p->kwin = (int)std::ceil(span) + 4;
    if (p->kwin > adj_pitch_limit(av)) {
        return fail(EIT_ERR_SHAPE, "adjoint window %d exceeds variant capacity", p->kwin);
    }
    p->n_tx = (n + p->at.TX - 1) / p->at.TX;
    // the mirror-pair adjoint runs tiles of the top half only (rows j with 2j <= n-1)
    p->n_ty = p->at.MIR ? ((n + 1) / 2 + p->at.TY - 1) / p->at.TY : (n + p->at.TY - 1) / p->at.TY;
    h.apairs.clear();
    h.mate.assign(nt, -1);
    if (p->at.MIR) {
        mirror_pairs(theta, h.mate);
        for (int a = 0; a < nt; ++a)
            if (h.mate[a] != -2) h.apairs.push_back(make_int2(a, h.mate[a]));
    }
    p->n_pairs = (int)h.apairs.size();
    {
        const int units = p->at.MIR ? p->n_pairs : nt;
        const int nchunks = (units + p->at.AC - 1) / p->at.AC;
        const int want = tiling ? tiling->adj_splits : 0;
        if (want > kMaxSplits)
            return fail(EIT_ERR_INVALID_ARG, "adj_splits=%d above %d", want, kMaxSplits);
        p->adj_splits = want >= 1 ? std::min(want, nchunks) : auto_splits(p->n_tx * p->n_ty, nchunks);
    }

    // ---- detector tables
    std::vector<float4>& flat = h.flat;
    flat.assign(nd, float4{});
    for (int k = 0; k < nd && p->gauss; ++k) {
        const double sg = setup->flat_sigma[k];
        flat[k] = make_float4((float)setup->flat_amp[k], (float)setup->flat_ctr[k],
                              (float)(1.0 / (2.0 * sg * sg)), (float)(1.0 / (sg * sg)));
    }
    h.maskd = mpos;

    // ---- single-slice work items
    p->n_trx = (n + kTrTile - 1) / kTrTile;
    p->nv = 2LL * n * n;
    p->n_vblocks = (int)((p->nv + kVecChunk - 1) / kVecChunk);
    std::vector<Item>&it_tr = h.it_tr, &it_pr = h.it_pr, &it_ic = h.it_ic, &it_bp = h.it_bp,
                     &it_vec = h.it_vec;
    for (int ty = 0; ty < p->n_trx; ++ty)
        for (int tx = 0; tx < p->n_trx; ++tx) it_tr.push_back(make_int4(0, tx, ty, 0));
    for (int g = 0; g < p->n_groups; ++g)
        for (int b = 0; b < p->n_dblk; ++b) it_pr.push_back(make_int4(0, g, b, 0));
    for (int a = 0; a < nt; ++a) it_ic.push_back(make_int4(0, a, 0, 0));
    for (int ty = 0; ty < p->n_ty; ++ty)
        for (int tx = 0; tx < p->n_tx; ++tx)
            for (int g = 0; g < p->adj_splits; ++g) it_bp.push_back(make_int4(0, tx, ty, g));
    for (int b = 0; b < p->n_vblocks; ++b) it_vec.push_back(make_int4(0, b, 0, 0));
    p->n_it_tr = (int)it_tr.size(); p->n_it_pr = (int)it_pr.size(); p->n_it_ic = nt;
    p->n_it_bp = (int)it_bp.size(); p->n_it_vec = (int)it_vec.size();

    // ---- full model of eq. 4: parameter vector and its work items
    if (int rc = build_model(setup, model, p, h, mpos)) return rc;
    p->n_vblocks = (int)((p->nvu + kVecChunk - 1) / kVecChunk);
    for (int b = 0; b < p->n_vblocks; ++b) h.it_uvec.push_back(make_int4(0, b, 0, 0));
    const int hb = (int)(((int64_t)n * n + kVecChunk - 1) / kVecChunk);
    for (int b = 0; b < hb; ++b) h.it_hvec.push_back(make_int4(0, b, 0, 0));
    p->n_it_uvec = (int)h.it_uvec.size();
    p->n_it_hvec = hb;
    if (p->ext & EXT_RING)
        for (int b = 0; b < (nd + kRingPixPerItem - 1) / kRingPixPerItem; ++b)
            h.it_ring.push_back(make_int4(0, b, 0, 0));
    p->n_it_ring = (int)h.it_ring.size();
    if (p->ext)
        for (int64_t b = 0; b < (p->nvu + kContractChunk - 1) / kContractChunk; ++b)
            h.it_cvec.push_back(make_int4(0, (int)b, 0, 0));
    p->n_it_cvec = (int)h.it_cvec.size();
    return EIT_OK;
}

}  // namespace

namespace {
int create_plan(const eit_dims* dims, const eit_setup* setup, const eit_model* model,
                const eit_tiling* tiling, eit_plan** out) {
    if (!out) return fail(EIT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    eit_plan* p = new eit_plan();
    HostTables h;
    int rc = build_host(dims, setup, tiling, p, h, model);
    if (rc) {
        delete p;
        return rc;
    }
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return fail(EIT_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    if ((rc = upload(&p->pang, h.pang)) || (rc = upload(&p->groups, h.groups)) ||
        (rc = upload(&p->win_lo, h.win_lo)) || (rc = upload(&p->aang, h.aang)) ||
        (rc = upload(&p->apairs, h.apairs)) ||
        (rc = upload(&p->flat, h.flat)) || (rc = upload(&p->mask, h.maskd)) ||
        (rc = upload(&p->it_tr, h.it_tr)) || (rc = upload(&p->it_pr, h.it_pr)) ||
        (rc = upload(&p->it_ic, h.it_ic)) || (rc = upload(&p->it_bp, h.it_bp)) ||
        (rc = upload(&p->it_vec, h.it_vec)) || (rc = upload(&p->ftab, h.ftab)) ||
        (rc = upload(&p->eq3_kern, h.eq3_kern)) || (rc = upload(&p->eq3_invf, h.eq3_invf)) ||
        (rc = upload(&p->it_uvec, h.it_uvec)) || (rc = upload(&p->it_hvec, h.it_hvec)) ||
        (rc = upload(&p->it_ring, h.it_ring)) || (rc = upload(&p->it_cvec, h.it_cvec))) {
        free_plan(p);
        return rc;
    }
    *out = p;
    return EIT_OK;
}
}  // namespace

extern "C" int eit_plan_create(const eit_dims* dims, const eit_setup* setup,
                               const eit_tiling* tiling, eit_plan** out) {
    return create_plan(dims, setup, nullptr, tiling, out);
}

extern "C" int eit_plan_create_model(const eit_dims* dims, const eit_setup* setup,
                                     const eit_model* model, const eit_tiling* tiling,
                                     eit_plan** out) {
    if (!model) return fail(EIT_ERR_INVALID_ARG, "model is NULL");
    return create_plan(dims, setup, model, tiling, out);
}

extern "C" int64_t eit_param_count(const eit_plan* p) { return p ? p->nvu : 0; }

extern "C" int eit_plan_inspect(const eit_dims* dims, const eit_setup* setup,
                                const eit_tiling* tiling, eit_plan_info* info,
                                double* proj_angles, int32_t* groups, int32_t* win_lo,
                                double* adj_angles) {
    if (!info) return fail(EIT_ERR_INVALID_ARG, "info is NULL");
    eit_plan tmp{};
    HostTables h;
    int rc = build_host(dims, setup, tiling, &tmp, h);
    if (rc) return rc;
    info->proj_variant = tmp.proj_v; info->adj_variant = tmp.adj_v;
    info->proj_a = tmp.pt.A; info->proj_w = tmp.pt.W; info->proj_r = tmp.pt.R;
    info->adj_tx = tmp.at.TX; info->adj_ty = tmp.at.TY; info->adj_ac = tmp.at.AC;
    info->n_groups = tmp.n_groups; info->n_dblk = tmp.n_dblk; info->n_strips = tmp.n_strips;
    info->win_w = tmp.win_w; info->win_pitch = tmp.pt.LP;
    info->proj_lds_bytes = (int64_t)tmp.proj_lds;
    info->kwin = tmp.kwin; info->n_tx = tmp.n_tx; info->n_ty = tmp.n_ty;
    info->kwin_pitch_limit = adj_pitch_limit(tmp.adj_v);
    info->adj_splits = tmp.adj_splits;
    info->adj_mirror = tmp.at.MIR;
    info->n_pairs = tmp.n_pairs;
    if (proj_angles)
        for (size_t a = 0; a < h.pang.size(); ++a) {
            const ProjAngle& q = h.pang[a];
            double* o = proj_angles + 6 * a;
            o[0] = q.inv; o[1] = q.base; o[2] = q.slope; o[3] = q.slope_f; o[4] = q.w; o[5] = q.src;
        }
    if (groups) std::copy(h.groups.begin(), h.groups.end(), groups);
    if (win_lo) std::copy(h.win_lo.begin(), h.win_lo.end(), win_lo);
    if (adj_angles)
        for (size_t a = 0; a < h.aang.size(); ++a) {
            const AdjAngle& q = h.aang[a];
            double* o = adj_angles + 10 * a;
            o[0] = q.cs; o[1] = q.sn; o[2] = q.cd; o[3] = q.cs_f; o[4] = q.sn_f;
            o[5] = q.iw; o[6] = q.iw2; o[7] = q.iwm; o[8] = q.cd_s; o[9] = h.mate[a];
        }
    return EIT_OK;
}

namespace {
void purge_graphs(const eit_plan* p);
}  // namespace

extern "C" void eit_plan_destroy(eit_plan* p) {
    if (!p) return;
    purge_graphs(p);
    free_plan(p);
}

// ============================================================================ workspace
namespace {

struct EvalLayout {
    size_t desc, xT, P, part_ic, part_reg, cost, bp_part, end;
    size_t xe, ge, g_mo, g_dl;      // full model only (0 otherwise)
};

EvalLayout eval_layout(const eit_plan* p, bool need_P, size_t base = 0) {
    Layout L;
    L.off = base;
    EvalLayout e{};
    e.desc = L.take(sizeof(SliceDesc));
    e.xT = L.take(sizeof(float) * (size_t)p->nv);
    e.P = need_P ? L.take(sizeof(float) * 2 * (size_t)p->n_theta * p->n_det) : 0;
    e.part_ic = L.take(sizeof(double) * (size_t)p->n_theta);
    e.part_reg = L.take(sizeof(double) * 2 * (size_t)p->n_trx * p->n_trx);
    e.cost = L.take(sizeof(double));
    e.bp_part = p->adj_splits > 1 ? L.take(sizeof(double) * p->adj_splits * (size_t)p->nv) : 0;
    if (p->ext) {
        e.xe = (p->ext & EXT_HMODE) ? L.take(sizeof(float) * (size_t)p->nv) : 0;
        e.ge = L.take(sizeof(float) * (size_t)p->nv);
        e.g_mo = (p->ext & EXT_DRIFT) ? L.take(sizeof(double) * (size_t)p->n_theta) : 0;
        e.g_dl = (p->ext & EXT_RING) ? L.take(sizeof(double) * (size_t)p->n_theta * p->n_det) : 0;
    }
    e.end = L.off;
    return e;
}

struct SolveLayout {
    EvalLayout ev;
    size_t lbdesc, state, z, zt, g, gt, d, S, Y, part, end;
};

SolveLayout solve_layout(const eit_plan* p, int m, size_t base = 0) {
    SolveLayout s{};
    s.ev = eval_layout(p, true, base);
    Layout L;
    L.off = s.ev.end;
    const size_t vb = sizeof(float) * (size_t)p->nvu;
    s.lbdesc = L.take(sizeof(LbDesc));
    s.state = L.take(sizeof(SolverState));
    s.z = L.take(vb); s.zt = L.take(vb); s.g = L.take(vb); s.gt = L.take(vb); s.d = L.take(vb);
    s.S = L.take(vb * (m + 1));
    s.Y = L.take(vb * (m + 1));
    s.part = L.take(sizeof(double) * max_dots(m) * (size_t)p->n_vblocks);
    s.end = L.off;
    return s;
}

char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

SliceDesc base_desc(const eit_plan* p) {
    SliceDesc d{};
    d.n = p->n; d.n_theta = p->n_theta; d.n_det = p->n_det; d.n_mask = p->n_mask;
    d.kappa = (float)p->kappa;
    d.scale_mu = 1.0; d.scale_de = 1.0;
    d.proj_tile = p->proj_v; d.adj_tile = p->adj_v;
    d.n_groups = p->n_groups; d.n_dblk = p->n_dblk; d.n_strips = p->n_strips;
    d.win_w = p->win_w; d.win_shift = p->win_shift;
    d.n_tx = p->n_tx; d.n_ty = p->n_ty; d.kwin = p->kwin;
    d.adj_splits = p->adj_splits;
    d.n_pairs = p->n_pairs; d.apairs = p->apairs;
    d.pang = p->pang; d.groups = p->groups; d.win_lo = p->win_lo; d.aang = p->aang;
    d.flat = p->flat; d.mask = p->mask;
    d.n_reg_blocks = p->n_trx * p->n_trx;
    d.ext = p->ext;
    d.nq = p->nq; d.tab_u0 = p->tab_u0; d.tab_du = p->tab_du; d.ftab = p->ftab;
    d.off_scale = 1.0;
    d.nvu = p->nvu;
    d.maps = 2;
    return d;
}

// Full-model buffers of a descriptor whose evaluation buffers start at `base`: the expanded
// maps, the adjoint's planes and the offset sums. x_param is the parameter vector of the point.
void set_ext_buffers(const eit_plan* p, SliceDesc& d, void* base, const EvalLayout& L,
                     const float* x_param) {
    const size_t nn = (size_t)p->n * p->n;
    d.xu = x_param;
    d.xe = (p->ext & EXT_HMODE) ? (float*)at(base, L.xe) : nullptr;
    d.maps = p->eval_maps;
    // the pair evaluation reads the expanded [h, h]; the single-map one reads h in place
    d.x = d.xe && d.maps == 2 ? d.xe : x_param;
    d.off = (p->ext & (EXT_DRIFT | EXT_RING)) ? x_param + p->n_maps * nn : nullptr;
    d.g = (float*)at(base, L.ge);
    d.g_mo = (p->ext & EXT_DRIFT) ? (double*)at(base, L.g_mo) : nullptr;
    d.g_dl = (p->ext & EXT_RING) ? (double*)at(base, L.g_dl) : nullptr;
}

// The adjoint's partial-sum planes of a descriptor whose evaluation buffers start at `base`.
void set_split_buffers(SliceDesc& d, void* base, const EvalLayout& L) {
    d.bp_part = d.adj_splits > 1 ? (double*)at(base, L.bp_part) : nullptr;
}

// Adjoint launch, then (split plans) the pass that adds the parts into d.g.
int enqueue_backproject(const eit_plan* p, const SliceDesc* dd, int add_reg, hipStream_t st) {
    HIP_TRY(launch_backproject(p->adj_v, 2, dd, p->it_bp, p->n_it_bp, grid_for(p->n_it_bp, kGridCap),
                               add_reg, st));
    if (p->adj_splits > 1)
        HIP_TRY(launch_bp_combine(dd, p->it_vec, p->n_it_vec, grid_for(p->n_it_vec, kGridCap),
                                  add_reg, st));
    return EIT_OK;
}

int check_ws(const void* ws, size_t have, size_t need) {
    if (!ws) return fail(EIT_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(EIT_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    if (have < need) return fail(EIT_ERR_NOMEM, "workspace %zu bytes < required %zu", have, need);
    return EIT_OK;
}

}  // namespace

extern "C" size_t eit_workspace_bytes(const eit_plan* p, int32_t op, int32_t m) {
    if (!p) return 0;
    switch (op) {
        case EIT_OP_PROJECT: return eval_layout(p, false).end;
        case EIT_OP_BACKPROJECT: return eval_layout(p, false).end;
        case EIT_OP_COST_GRAD: return eval_layout(p, true).end;
        case EIT_OP_SINGLE_SHOT: return eval_layout(p, true).end;
        case EIT_OP_RECONSTRUCT:
            if (m < 1 || m > EIT_MAX_LBFGS_M) return 0;
            return solve_layout(p, m).end;
        default: return 0;
    }
}

// ============================================================================ single evaluations
namespace {

int enqueue_eval(const eit_plan* p, const SliceDesc* dd, bool seeds, bool grad, hipStream_t st) {
    HIP_TRY(launch_transpose(dd, p->it_tr, p->n_it_tr, grid_for(p->n_it_tr, kGridCap), st));
    HIP_TRY(launch_project(p->proj_v, 2, dd, p->it_pr, p->n_it_pr, grid_for(p->n_it_pr, kGridCap),
                           p->proj_lds, st));
    HIP_TRY(launch_ic(dd, p->it_ic, p->n_it_ic, grid_for(p->n_it_ic, kGridCap), seeds ? 1 : 0, st));
    if (grad) return enqueue_backproject(p, dd, 1, st);
    return EIT_OK;
}

}  // namespace

extern "C" int eit_project(const eit_plan* p, const float* x, float* sino, void* ws,
                           size_t ws_bytes, void* stream) {
    if (!p) return fail(EIT_ERR_INVALID_ARG, "plan is NULL");
    if (!x || !sino) return fail(EIT_ERR_INVALID_ARG, "x or sino is NULL");
    const EvalLayout L = eval_layout(p, false);
    if (int rc = check_ws(ws, ws_bytes, L.end)) return rc;
    hipStream_t st = (hipStream_t)stream;
    SliceDesc d = base_desc(p);
    d.x = x;
    d.xT = (float*)at(ws, L.xT);
    d.P = sino;
    d.part_reg = (double*)at(ws, L.part_reg);
    SliceDesc* dd = (SliceDesc*)at(ws, L.desc);
    HIP_TRY(launch_store_desc(d, dd, st));
    HIP_TRY(launch_transpose(dd, p->it_tr, p->n_it_tr, grid_for(p->n_it_tr, kGridCap), st));
    HIP_TRY(launch_project(p->proj_v, 2, dd, p->it_pr, p->n_it_pr, grid_for(p->n_it_pr, kGridCap),
                           p->proj_lds, st));
    return EIT_OK;
}

extern "C" int eit_backproject(const eit_plan* p, const float* sino, float* x_out, void* ws,
                               size_t ws_bytes, void* stream) {
    if (!p) return fail(EIT_ERR_INVALID_ARG, "plan is NULL");
    if (!sino || !x_out) return fail(EIT_ERR_INVALID_ARG, "sino or x_out is NULL");
    const EvalLayout L = eval_layout(p, false);
    if (int rc = check_ws(ws, ws_bytes, L.end)) return rc;
    hipStream_t st = (hipStream_t)stream;
    SliceDesc d = base_desc(p);
    d.P = const_cast<float*>(sino);   // read only by the adjoint
    d.g = x_out;
    set_split_buffers(d, ws, L);
    SliceDesc* dd = (SliceDesc*)at(ws, L.desc);
    HIP_TRY(launch_store_desc(d, dd, st));
    return enqueue_backproject(p, dd, 0, st);
}

extern "C" int eit_cost_and_grad(const eit_plan* p, const float* x, const float* s_exp,
                                 double lam_mu, double lam_delta, double* cost_dev, float* grad,
                                 void* ws, size_t ws_bytes, void* stream) {
    if (!p) return fail(EIT_ERR_INVALID_ARG, "plan is NULL");
    if (!x || !s_exp || !cost_dev) return fail(EIT_ERR_INVALID_ARG, "x, s_exp or cost_dev is NULL");
    if (!(lam_mu >= 0.0) || !(lam_delta >= 0.0) || !std::isfinite(lam_mu) || !std::isfinite(lam_delta))
        return fail(EIT_ERR_INVALID_ARG, "lam_mu / lam_delta must be finite and >= 0");
    const EvalLayout L = eval_layout(p, true);
    if (int rc = check_ws(ws, ws_bytes, L.end)) return rc;
    hipStream_t st = (hipStream_t)stream;
    SliceDesc d = base_desc(p);
    d.x = x;
    d.xT = (float*)at(ws, L.xT);
    d.P = (float*)at(ws, L.P);
    d.s_exp = s_exp;
    d.g = grad;
    d.part_ic = (double*)at(ws, L.part_ic);
    d.part_reg = (double*)at(ws, L.part_reg);
    d.cost = cost_dev;
    d.lam_mu = lam_mu; d.lam_de = lam_delta;
    d.reg_mu = 2.0 * lam_mu; d.reg_de = 2.0 * lam_delta;
    set_split_buffers(d, ws, L);
    SliceDesc* dd = (SliceDesc*)at(ws, L.desc);
    if (p->ext) {
        // full model: the maps through the two-map kernels (h-mode: h once through the
        // single-map kernels, or expanded to [h, h]; P_delta scaled by gamma), the eq. 4 IC
        // stage, the adjoint without regulariser and the contraction to the parameter layout
        set_ext_buffers(p, d, ws, L, x);
        d.gu = grad;
        if (p->ext & EXT_HMODE) {
            d.scale_de = p->gamma;
            d.lam_de = 0.0;
            d.reg_de = 0.0;
        }
        HIP_TRY(launch_store_desc(d, dd, st));
        if ((p->ext & EXT_HMODE) && p->eval_maps == 2)
            HIP_TRY(launch_ext_expand(dd, p->it_hvec, p->n_it_hvec, grid_for(p->n_it_hvec, kGridCap), st));
        HIP_TRY(launch_transpose(dd, p->it_tr, p->n_it_tr, grid_for(p->n_it_tr, kGridCap), st));
        HIP_TRY(launch_project(p->proj_v, p->eval_maps, dd, p->it_pr, p->n_it_pr,
                               grid_for(p->n_it_pr, kGridCap), p->proj_lds, st));
        HIP_TRY(launch_ic_ext(dd, p->it_ic, p->n_it_ic, grid_for(p->n_it_ic, kGridCap),
                              grad ? 1 : 0, p->n_det, st));
        HIP_TRY(launch_cost_reduce(dd, 1, st));
        if (!grad) return EIT_OK;
        // the contraction adds a split adjoint's partial planes itself (no combine pass)
        HIP_TRY(launch_backproject(p->adj_v, p->eval_maps, dd, p->it_bp, p->n_it_bp,
                                   grid_for(p->n_it_bp, kGridCap), 0, st));
        HIP_TRY(launch_ext_contract(dd, p->it_cvec, p->n_it_cvec, grid_for(p->n_it_cvec, kGridCap), st));
        HIP_TRY(launch_ext_ring_grad(dd, p->it_ring, p->n_it_ring, grid_for(p->n_it_ring, kGridCap), st));
        return EIT_OK;
    }
    HIP_TRY(launch_store_desc(d, dd, st));
    if (int rc = enqueue_eval(p, dd, grad != nullptr, false, st)) return rc;
    HIP_TRY(launch_cost_reduce(dd, 1, st));
    if (grad) return enqueue_backproject(p, dd, 1, st);
    return EIT_OK;
}

extern "C" int eit_single_shot(const eit_plan* p, const float* s_exp, float* x_out, void* ws,
                               size_t ws_bytes, void* stream) {
    if (!p) return fail(EIT_ERR_INVALID_ARG, "plan is NULL");
    if (!s_exp || !x_out) return fail(EIT_ERR_INVALID_ARG, "s_exp or x_out is NULL");
    const EvalLayout L = eval_layout(p, true);
    if (int rc = check_ws(ws, ws_bytes, L.end)) return rc;
    hipStream_t st = (hipStream_t)stream;
    SliceDesc d = base_desc(p);
    d.P = (float*)at(ws, L.P);
    d.s_exp = s_exp;
    d.g = x_out;
    set_split_buffers(d, ws, L);
    SliceDesc* dd = (SliceDesc*)at(ws, L.desc);
    const int gi = grid_for(p->n_it_ic, kGridCap);
    if (p->ext) {
        // h-mode: eq. 3 from one mask position; two maps: the per-pixel fit (Gaussian flats).
        // Both planes are backprojected into the workspace and the maps copied out, offsets 0.
        if (!(p->ext & EXT_HMODE) && !p->gauss)
            return fail(EIT_ERR_INVALID_ARG, "the two-map single shot needs the Gaussian flat parameters");
        d.g = (float*)at(ws, L.ge);
        d.gu = x_out;
        HIP_TRY(launch_store_desc(d, dd, st));
        if (p->ext & EXT_HMODE)
            HIP_TRY(launch_eq3_retrieve(dd, p->it_ic, p->n_it_ic, gi, p->eq3_kern, p->eq3_invf,
                                        p->eq3_mask, st));
        else
            HIP_TRY(launch_ss_retrieve(dd, p->it_ic, p->n_it_ic, gi, st));
        HIP_TRY(launch_ss_filter(dd, p->it_ic, p->n_it_ic, gi, st));
        if (int rc = enqueue_backproject(p, dd, 0, st)) return rc;
        HIP_TRY(launch_ext_take_maps(dd, p->it_uvec, p->n_it_uvec, grid_for(p->n_it_uvec, kGridCap), st));
        return EIT_OK;
    }
    HIP_TRY(launch_store_desc(d, dd, st));
    HIP_TRY(launch_ss_retrieve(dd, p->it_ic, p->n_it_ic, gi, st));
    HIP_TRY(launch_ss_filter(dd, p->it_ic, p->n_it_ic, gi, st));
    return enqueue_backproject(p, dd, 0, st);
}

// ============================================================================ reconstruct
namespace {

int validate_opts(const eit_opts* o) {
    if (!o) return fail(EIT_ERR_INVALID_ARG, "opts is NULL");
    if (o->max_iter < 0) return fail(EIT_ERR_INVALID_ARG, "max_iter < 0");
    if (o->lbfgs_m < 1 || o->lbfgs_m > EIT_MAX_LBFGS_M)
        return fail(EIT_ERR_INVALID_ARG, "lbfgs_m=%d outside [1, %d]", o->lbfgs_m, EIT_MAX_LBFGS_M);
    if (o->max_ls_trials < 0) return fail(EIT_ERR_INVALID_ARG, "max_ls_trials < 0");
    if (!(o->lam >= 0.0) || !std::isfinite(o->lam)) return fail(EIT_ERR_INVALID_ARG, "lam must be finite and >= 0");
    if (!finite_pos(o->mu_scale) || !finite_pos(o->delta_scale))
        return fail(EIT_ERR_INVALID_ARG, "mu_scale / delta_scale must be finite and > 0");
    if (!(o->tol_rel_step >= 0.0) || !std::isfinite(o->tol_rel_step))
        return fail(EIT_ERR_INVALID_ARG, "tol_rel_step must be finite and >= 0");
    if (!(o->c1 > 0.0 && o->c1 < 1.0)) return fail(EIT_ERR_INVALID_ARG, "c1 must be in (0, 1)");
    return EIT_OK;
}

// One evaluation step of the optimiser for n_slices slices described by (D, L).
struct StepPlan {
    const SliceDesc* D;
    const LbDesc* L;
    int n_slices;
    // per projector / adjoint variant groups (batch may mix variants)
    struct Launch { int variant; const Item* items; int n; size_t lds; int maps; };
    void* gather = nullptr;    // batches: device array the slices' states are gathered into
    std::vector<Launch> proj, adj;
    const Item* it_tr; int n_tr;
    const Item* it_ic; int n_ic;
    const Item* it_vec; int n_vec;
    // full model of eq. 4: vector-form direction, separate transpose, eq. 4 IC stage, adjoint
    // without regulariser, contraction (which adds a split adjoint's parts), ring sums
    bool ext = false;
    const Item* it_ring = nullptr; int n_ring = 0; // pixel blocks of ring-term gradients
    const Item* it_cvec = nullptr; int n_cvec = 0; // contraction chunks
    int max_det = 0;                               // widest slice (n_det) of the launch
};

// ev: optional array of EIT_N_PHASES + 1 events recorded around the phases.
int enqueue_step(const StepPlan& sp, hipStream_t st, hipEvent_t* ev) {
    auto mark = [&](int i) -> int {
        if (ev) HIP_TRY(hipEventRecord(ev[i], st));
        return EIT_OK;
    };
    if (int rc = mark(0)) return rc;
    if (sp.ext) {
        HIP_TRY(launch_lb_direction_vec(sp.L, sp.D, sp.it_vec, sp.n_vec, grid_for(sp.n_vec, kGridCap), st));
        if (int rc = mark(1)) return rc;
        HIP_TRY(launch_transpose(sp.D, sp.it_tr, sp.n_tr, grid_for(sp.n_tr, kGridCap), st));
        if (int rc = mark(2)) return rc;
        for (const auto& l : sp.proj)
            HIP_TRY(launch_project(l.variant, l.maps, sp.D, l.items, l.n, grid_for(l.n, kGridCap), l.lds, st));
        if (int rc = mark(3)) return rc;
        HIP_TRY(launch_ic_ext(sp.D, sp.it_ic, sp.n_ic, grid_for(sp.n_ic, kGridCap), 1, sp.max_det, st));
        if (int rc = mark(4)) return rc;
        HIP_TRY(launch_lb_decide(sp.D, sp.L, sp.n_slices, st));
        if (int rc = mark(5)) return rc;
        for (const auto& l : sp.adj)
            HIP_TRY(launch_backproject(l.variant, l.maps, sp.D, l.items, l.n, grid_for(l.n, kGridCap), 0, st));
        // the contraction adds a split adjoint's partial planes itself
        HIP_TRY(launch_ext_contract(sp.D, sp.it_cvec, sp.n_cvec, grid_for(sp.n_cvec, kGridCap), st));
        HIP_TRY(launch_ext_ring_grad(sp.D, sp.it_ring, sp.n_ring, grid_for(sp.n_ring, kGridCap), st));
        if (int rc = mark(6)) return rc;
        HIP_TRY(launch_lb_update(sp.L, sp.it_vec, sp.n_vec, grid_for(sp.n_vec, kGridCap), st));
        if (int rc = mark(7)) return rc;
        HIP_TRY(launch_lb_finalize(sp.L, sp.n_slices, st));
        return mark(8);
    }
    // direction, trial point, its transposed copy and ||zt||^2 partials in one pass
    HIP_TRY(launch_lb_direction(sp.L, sp.D, sp.it_tr, sp.n_tr, grid_for(sp.n_tr, kGridCap), st));
    if (int rc = mark(1)) return rc;
    if (int rc = mark(2)) return rc;
    for (const auto& l : sp.proj)
        HIP_TRY(launch_project(l.variant, l.maps, sp.D, l.items, l.n, grid_for(l.n, kGridCap), l.lds, st));
    if (int rc = mark(3)) return rc;
    HIP_TRY(launch_ic(sp.D, sp.it_ic, sp.n_ic, grid_for(sp.n_ic, kGridCap), 1, st));
    if (int rc = mark(4)) return rc;
    HIP_TRY(launch_lb_decide(sp.D, sp.L, sp.n_slices, st));
    if (int rc = mark(5)) return rc;
    for (const auto& l : sp.adj)
        HIP_TRY(launch_backproject(l.variant, l.maps, sp.D, l.items, l.n, grid_for(l.n, kGridCap), 1, st));
    if (int rc = mark(6)) return rc;
    HIP_TRY(launch_lb_update(sp.L, sp.it_vec, sp.n_vec, grid_for(sp.n_vec, kGridCap), st));
    if (int rc = mark(7)) return rc;
    HIP_TRY(launch_lb_finalize(sp.L, sp.n_slices, st));
    return mark(8);
}

struct PhaseTimer {
    std::vector<hipEvent_t> ev;     // (steps) x (EIT_N_PHASES + 1)
    double ms[EIT_N_PHASES] = {0};
    int steps = 0;
    ~PhaseTimer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    int next(hipEvent_t** out) {
        const size_t base = ev.size();
        for (int i = 0; i <= EIT_N_PHASES; ++i) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            ev.push_back(e);
        }
        *out = &ev[base];
        ++steps;
        return EIT_OK;
    }
    int collect() {
        for (int s = 0; s < steps; ++s)
            for (int i = 0; i < EIT_N_PHASES; ++i) {
                float t = 0.f;
                HIP_TRY(hipEventElapsedTime(&t, ev[(size_t)s * (EIT_N_PHASES + 1) + i],
                                            ev[(size_t)s * (EIT_N_PHASES + 1) + i + 1]));
                ms[i] += t;
            }
        return EIT_OK;
    }
};

// ---------------------------------------------------------------------------- step graphs
// A captured graph holds kStepsPerGraph consecutive evaluation steps; the launch gap between
// graphs is larger than between kernels of one graph. Its kernels read every per-call value
// (data pointers, options, optimiser state) from descriptors at fixed workspace offsets, so
// a graph depends only on the plans (item tables, tiles), the workspace address and the
// L-BFGS memory (which fixes the workspace layout). Graphs are therefore kept, keyed by
// those, and replayed by later calls instead of being captured and instantiated each time.
// At most kGraphCacheMax are kept (least recently used dropped); destroying a plan drops its
// graphs. Captures run on a library-owned stream per device, so the caller's stream, the
// null stream included, only ever replays.
constexpr int kStepsPerGraph = 4;
constexpr size_t kGraphCacheMax = 16;

struct GraphKey {
    std::vector<const eit_plan*> plans;
    const void* ws = nullptr;
    int m = 0;
    int device = 0;
    bool operator==(const GraphKey& o) const {
        return plans == o.plans && ws == o.ws && m == o.m && device == o.device;
    }
};
struct GraphEntry {
    GraphKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
std::vector<hipStream_t> g_capture_streams;    // per device, created on first use

void destroy_entry(GraphEntry& e) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
}

void purge_graphs(const eit_plan* p) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    bool any = false;
    for (const auto& e : g_graphs)
        any = any || std::find(e.key.plans.begin(), e.key.plans.end(), p) != e.key.plans.end();
    if (!any) return;
    (void)hipDeviceSynchronize();           // no replay of a dropped graph may still be queued
    for (auto& e : g_graphs)
        if (std::find(e.key.plans.begin(), e.key.plans.end(), p) != e.key.plans.end()) destroy_entry(e);
    g_graphs.erase(std::remove_if(g_graphs.begin(), g_graphs.end(),
                                  [](const GraphEntry& e) { return e.exec == nullptr; }),
                   g_graphs.end());
}

// Library-owned streams per device, created on first use and kept until the process ends:
// one for captures (under g_graph_mu), one that replays graphs for null-stream callers.
std::vector<hipStream_t> g_replay_streams;
std::mutex g_stream_mu;

int owned_stream(std::vector<hipStream_t>& v, int dev, hipStream_t* out) {
    std::lock_guard<std::mutex> lk(g_stream_mu);
    if ((int)v.size() <= dev) v.resize(dev + 1, nullptr);
    if (!v[dev]) HIP_TRY(hipStreamCreateWithFlags(&v[dev], hipStreamNonBlocking));
    *out = v[dev];
    return EIT_OK;
}
int capture_stream(int dev, hipStream_t* out) { return owned_stream(g_capture_streams, dev, out); }
int replay_stream(int dev, hipStream_t* out) { return owned_stream(g_replay_streams, dev, out); }

int enqueue_step(const StepPlan& sp, hipStream_t st, hipEvent_t* ev);

// The graph of key, captured on first use.
int step_graph(const StepPlan& sp, GraphKey key, hipGraphExec_t* out) {
    HIP_TRY(hipGetDevice(&key.device));
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& e : g_graphs)
        if (e.key == key) {
            e.used = ++g_graph_clock;
            *out = e.exec;
            return EIT_OK;
        }
    hipStream_t cs;
    if (int rc = capture_stream(key.device, &cs)) return rc;
    GraphEntry ent;
    ent.key = key;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = EIT_OK;
    for (int q = 0; q < kStepsPerGraph && !rc; ++q) rc = enqueue_step(sp, cs, nullptr);
    hipError_t e = hipStreamEndCapture(cs, &ent.graph);
    if (rc) { destroy_entry(ent); return rc; }
    if (e != hipSuccess) { destroy_entry(ent); return fail(EIT_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e)); }
    e = hipGraphInstantiate(&ent.exec, ent.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        destroy_entry(ent);
        return fail(EIT_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    if (g_graphs.size() >= kGraphCacheMax) {
        auto lru = std::min_element(g_graphs.begin(), g_graphs.end(),
                                    [](const GraphEntry& a, const GraphEntry& b) { return a.used < b.used; });
        (void)hipDeviceSynchronize();       // the dropped graph may still be replaying
        destroy_entry(*lru);
        g_graphs.erase(lru);
    }
    ent.used = ++g_graph_clock;
    g_graphs.push_back(ent);
    *out = ent.exec;
    return EIT_OK;
}

// Replays the step until every slice's optimiser has stopped. Reads back (status, k) of each
// slice only between rounds of launches; each round enqueues as many steps as the slowest
// slice still needs iterations (every accepted iteration needs at least one evaluation).
int drive_on(const StepPlan& sp, const std::vector<SolverState*>& states, int max_iter, int max_ls,
             hipGraphExec_t exec, hipStream_t st, int* launches_out, PhaseTimer* pt);

// Graph replays for a null-stream caller run on a library-owned non-blocking stream, ordered
// after (and before) the caller's work through an event.
int drive(const StepPlan& sp, const std::vector<SolverState*>& states, int max_iter, int max_ls,
          bool use_graph, const GraphKey& key, hipStream_t st, int* launches_out, PhaseTimer* pt) {
    if (pt) use_graph = false;
    hipGraphExec_t exec = nullptr;
    if (use_graph)
        if (int rc = step_graph(sp, key, &exec)) return rc;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (!use_graph || st != nullptr)
        return drive_on(sp, states, max_iter, max_ls, exec, st, launches_out, pt);
    hipStream_t side = nullptr;
    hipEvent_t ev = nullptr;
    if (int rc = replay_stream(dev, &side)) return rc;
    int rc = EIT_OK;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, ev, 0);
    if (e != hipSuccess) rc = fail(EIT_ERR_DEVICE, "stream ordering: %s", hipGetErrorString(e));
    if (!rc) rc = drive_on(sp, states, max_iter, max_ls, exec, side, launches_out, nullptr);
    if (!rc) {
        e = hipEventRecord(ev, side);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
        if (e != hipSuccess) rc = fail(EIT_ERR_DEVICE, "stream ordering: %s", hipGetErrorString(e));
    }
    if (ev) (void)hipEventDestroy(ev);
    return rc;
}

int drive_on(const StepPlan& sp, const std::vector<SolverState*>& states, int max_iter, int max_ls,
             hipGraphExec_t exec, hipStream_t st, int* launches_out, PhaseTimer* pt) {
    // Steps past a slice's end are no-ops (its skip flags are set), so a round may run up to
    // kStepsPerGraph - 1 idle steps.
    const bool use_graph = exec != nullptr;
    const long long cap = (long long)(max_iter + 2) * (max_ls + 2) * 2 + 16;
    long long total = 0;
    int rc = EIT_OK;
    int want = max_iter + 1;
    std::vector<int32_t> host(5 * states.size());
    while (rc == EIT_OK) {
        for (int i = 0; i < want && rc == EIT_OK;) {
            if (use_graph) {
                hipError_t e = hipGraphLaunch(exec, st);
                if (e != hipSuccess) rc = fail(EIT_ERR_DEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
                i += kStepsPerGraph;
                total += kStepsPerGraph;
            } else {
                hipEvent_t* ev = nullptr;
                if (pt) rc = pt->next(&ev);
                if (!rc) rc = enqueue_step(sp, st, ev);
                ++i;
                ++total;
            }
        }
        if (rc) break;
        if (sp.gather && states.size() > 1) {      // one copy for the whole batch
            hipError_t e = launch_gather_status(sp.L, (int)states.size(), (int32_t*)sp.gather, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(host.data(), sp.gather, host.size() * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) { rc = fail(EIT_ERR_DEVICE, "state read-back: %s", hipGetErrorString(e)); break; }
        } else {
            for (size_t q = 0; q < states.size(); ++q) {
                // k, evals, trials, mode, status are consecutive int32 fields
                hipError_t e = hipMemcpyAsync(&host[5 * q], &states[q]->k, 5 * sizeof(int32_t),
                                              hipMemcpyDeviceToHost, st);
                if (e != hipSuccess) { rc = fail(EIT_ERR_DEVICE, "state read-back: %s", hipGetErrorString(e)); break; }
            }
        }
        if (rc) break;
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) { rc = fail(EIT_ERR_DEVICE, "stream sync: %s", hipGetErrorString(e)); break; }
        int remaining = 0;
        for (size_t q = 0; q < states.size(); ++q)
            if (host[5 * q + 4] == ST_RUNNING)
                remaining = std::max(remaining, std::max(1, max_iter - host[5 * q]));
        if (rc || remaining == 0) break;
        if (total > cap) { rc = fail(EIT_ERR_DEVICE, "optimiser did not stop within %lld steps", cap); break; }
        want = remaining;
    }
    if (launches_out) *launches_out = (int)std::min<long long>(total, 1 << 30);
    return rc;
}


// Adjoint split of one solver slice: the parts land in the partial planes and the update
// forms the gradient from them (gt is then unused).
void set_solver_split(SliceDesc& d, LbDesc& l, void* base, const SolveLayout& S, int splits) {
    d.adj_splits = splits;
    set_split_buffers(d, base, S.ev);
    l.gpart = d.bp_part;
    l.gsplits = splits;
    l.reg_mu = d.reg_mu;
    l.reg_de = d.reg_de;
    if (d.ext) {            // full model: the combine pass and the contraction form gt
        l.gpart = nullptr;
        l.gsplits = 1;
    }
}

// Descriptors of one slice's optimiser run whose buffers start at `base` with layout S.
void solver_descs(const eit_plan* p, const eit_opts* o, void* base, const SolveLayout& S,
                  const float* s_exp, float* x, double* cost_hist, SliceDesc& d, LbDesc& l) {
    SolverState* state = (SolverState*)at(base, S.state);
    d = base_desc(p);
    d.x = (const float*)at(base, S.zt);
    d.xT = (float*)at(base, S.ev.xT);
    d.P = (float*)at(base, S.ev.P);
    d.s_exp = s_exp;
    d.g = (float*)at(base, S.gt);
    d.part_ic = (double*)at(base, S.ev.part_ic);
    d.part_reg = (double*)at(base, S.ev.part_reg);
    d.cost = &state->f_t;
    d.scale_mu = o->mu_scale; d.scale_de = o->delta_scale;
    d.lam_mu = o->lam; d.lam_de = o->lam;
    d.reg_mu = 2.0 * o->lam; d.reg_de = 2.0 * o->lam;
    d.skip = &state->skip;
    d.skip_adj = &state->skip_adj;
    l = LbDesc{};
    l.nv = p->nv; l.n = p->n; l.n_vblocks = p->n_vblocks;
    l.scale_mu = (float)o->mu_scale; l.scale_de = (float)o->delta_scale;
    l.nn = (int64_t)p->n * p->n; l.n_maps = 2; l.scale_off = 1.f;
    l.z = (float*)at(base, S.z); l.zt = (float*)at(base, S.zt); l.g = (float*)at(base, S.g);
    l.gt = (float*)at(base, S.gt); l.d = (float*)at(base, S.d);
    l.S = (float*)at(base, S.S); l.Y = (float*)at(base, S.Y);
    l.part = (double*)at(base, S.part);
    l.st = state;
    l.x_user = x;
    l.cost_hist = cost_hist;
    if (p->ext) {
        // full model: the optimiser's vectors are parameter vectors (maps, then offsets); the
        // update reads the contracted gradient gt, the split's parts are combined beforehand
        set_ext_buffers(p, d, base, S.ev, (const float*)at(base, S.zt));
        d.gu = (float*)at(base, S.gt);
        d.off_scale = p->off_scale;
        if (p->ext & EXT_HMODE) {
            d.scale_de = p->gamma * o->mu_scale;
            d.lam_de = 0.0;
            d.reg_de = 0.0;
        }
        l.nv = p->nvu;
        l.n_maps = p->n_maps;
        l.scale_off = (float)p->off_scale;
    }
    set_solver_split(d, l, base, S, p->adj_splits);
}

void fill_report(const SolverState& hs, int launches, eit_report* rep) {
    rep->status = hs.status == ST_DONE ? EIT_OK : hs.status;
    rep->iters = hs.k;
    rep->evals = hs.evals;
    rep->launches = launches;
    rep->cost = hs.f;
    rep->gnorm = std::sqrt(hs.gg);
    for (int i = 0; i < EIT_N_PHASES; ++i) rep->phase_ms[i] = 0.0;
    rep->phase_steps = 0;
}

}  // namespace

extern "C" int eit_reconstruct(const eit_plan* p, const float* s_exp, const eit_opts* o, float* x,
                               double* cost_hist, eit_report* rep, void* ws, size_t ws_bytes,
                               void* stream) {
    if (!p) return fail(EIT_ERR_INVALID_ARG, "plan is NULL");
    if (!s_exp || !x) return fail(EIT_ERR_INVALID_ARG, "s_exp or x is NULL");
    if (int rc = validate_opts(o)) return rc;
    const SolveLayout S = solve_layout(p, o->lbfgs_m);
    if (int rc = check_ws(ws, ws_bytes, S.end)) return rc;
    hipStream_t st = (hipStream_t)stream;

    SolverState* state = (SolverState*)at(ws, S.state);
    SliceDesc d;
    LbDesc l;
    solver_descs(p, o, ws, S, s_exp, x, cost_hist, d, l);
    SliceDesc* dd = (SliceDesc*)at(ws, S.ev.desc);
    LbDesc* ld = (LbDesc*)at(ws, S.lbdesc);
    HIP_TRY(launch_store_desc(d, dd, st));
    HIP_TRY(launch_store_lbdesc(l, ld, st));
    HIP_TRY(launch_lb_init(ld, 1, o->lbfgs_m, o->max_iter, o->max_ls_trials, o->c1, o->tol_rel_step, st));
    const int gv = grid_for(p->n_it_uvec, kGridCap);
    HIP_TRY(launch_lb_scale(ld, p->it_uvec, p->n_it_uvec, gv, 1, st));

    StepPlan sp;
    sp.D = dd; sp.L = ld; sp.n_slices = 1;
    sp.proj.push_back({p->proj_v, p->it_pr, p->n_it_pr, p->proj_lds, p->eval_maps});
    sp.adj.push_back({p->adj_v, p->it_bp, p->n_it_bp, 0, p->eval_maps});
    sp.it_tr = p->it_tr; sp.n_tr = p->n_it_tr;
    sp.it_ic = p->it_ic; sp.n_ic = p->n_it_ic;
    sp.it_vec = p->it_uvec; sp.n_vec = p->n_it_uvec;
    sp.ext = p->ext != 0;
    sp.it_ring = p->it_ring; sp.n_ring = p->n_it_ring;
    sp.it_cvec = p->it_cvec; sp.n_cvec = p->n_it_cvec;
    sp.max_det = p->n_det;
    int launches = 0;
    PhaseTimer timer;
    PhaseTimer* pt = o->profile ? &timer : nullptr;
    GraphKey key;
    key.plans = {p};
    key.ws = ws;
    key.m = o->lbfgs_m;
    if (int rc = drive(sp, {state}, o->max_iter, o->max_ls_trials, o->use_graph != 0, key, st,
                       &launches, pt))
        return rc;
    HIP_TRY(launch_lb_scale(ld, p->it_uvec, p->n_it_uvec, gv, 0, st));
    SolverState hs;
    HIP_TRY(hipMemcpyAsync(&hs, state, sizeof(SolverState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (rep) {
        fill_report(hs, launches, rep);
        if (pt) {
            if (int rc = pt->collect()) return rc;
            for (int i = 0; i < EIT_N_PHASES; ++i) rep->phase_ms[i] = pt->ms[i];
            rep->phase_steps = pt->steps;
        }
    }
    if (hs.status < 0)
        return fail(hs.status, hs.status == EIT_ERR_NONFINITE ? "cost is not finite at the start"
                                                              : "line search failed from an empty memory");
    return EIT_OK;
}

// ============================================================================ misc
extern "C" const char* eit_last_error(void) { return g_err.c_str(); }

extern "C" int eit_variant_info(int32_t kind, int32_t v, int32_t* a, int32_t* b, int32_t* c,
                                int32_t* dd) {
    if (kind == 0) {
        const int n = proj_variant_count();
        if (v >= 0 && v < n) {
            ProjTile t = proj_variant(v);
            if (a) *a = t.A;
            if (b) *b = t.W;
            if (c) *c = t.R;
            if (dd) *dd = t.PW;
        }
        return n;
    }
    if (kind == 2) {                       // projector LDS layout
        const int n = proj_variant_count();
        if (v >= 0 && v < n) {
            if (a) *a = proj_variant(v).DUP;
            if (b) *b = proj_variant(v).LP;
            if (c) *c = proj_variant(v).IL;
        }
        return n;
    }
    if (kind == 3) {                       // adjoint kernel form
        const int n = adj_variant_count();
        if (v >= 0 && v < n && a) *a = adj_variant(v).MIR;
        return n;
    }
    if (kind == 1) {
        const int n = adj_variant_count();
        if (v >= 0 && v < n) {
            AdjTile t = adj_variant(v);
            if (a) *a = t.TX;
            if (b) *b = t.TY;
            if (c) *c = t.AC;
            if (dd) *dd = t.VPT;
        }
        return n;
    }
    return 0;
}

// ============================================================================ batch
namespace {

struct BatchLayout {
    size_t descs = 0, lbdescs = 0, items = 0, gather = 0, end = 0;
    std::vector<size_t> slice;        // per-slice solve layout base
    std::vector<int> order;           // slices by decreasing work
    std::vector<int> splits;          // adjoint split per slice
    std::vector<Item> items_h;        // all work items, grouped by launch
    // item ranges (offset, count) in items_h
    std::pair<int, int> r_dir, r_ic, r_vec;
    std::pair<int, int> r_ring{0, 0}; // full model: pixel blocks of ring-term gradients
    std::pair<int, int> r_cvec{0, 0}; // full model: contraction chunks
    bool ext = false;                 // full-model batch (every plan has model options)
    // variant, off, count, lds, maps evaluated
    std::vector<std::tuple<int, int, int, size_t, int>> r_proj, r_adj;
};

int batch_layout(int32_t n, const eit_plan* const* plans, int32_t m, BatchLayout& B) {
    if (n < 1) return fail(EIT_ERR_INVALID_ARG, "n_slices must be >= 1");
    if (!plans) return fail(EIT_ERR_INVALID_ARG, "plans is NULL");
    if (m < 1 || m > EIT_MAX_LBFGS_M) return fail(EIT_ERR_INVALID_ARG, "lbfgs_m=%d out of range", m);
    for (int i = 0; i < n; ++i)
        if (!plans[i]) return fail(EIT_ERR_INVALID_ARG, "plans[%d] is NULL", i);
    B.ext = plans[0]->ext != 0;
    for (int i = 1; i < n; ++i)
        if ((plans[i]->ext != 0) != B.ext)
            return fail(EIT_ERR_INVALID_ARG, "plans[%d]: a batch takes either only plain plans or only "
                        "full-model plans", i);
    B.order.resize(n);
    for (int i = 0; i < n; ++i) B.order[i] = i;
    auto work = [&](int i) { return (double)plans[i]->n * plans[i]->n * plans[i]->n_theta; };
    std::stable_sort(B.order.begin(), B.order.end(), [&](int a, int b) { return work(a) > work(b); });
    // items: direction tiles, IC angles, vector chunks, then projector / adjoint per variant
    auto& H = B.items_h;
    H.clear();
    B.r_dir.first = 0;
    for (int i : B.order)
        for (int ty = 0; ty < plans[i]->n_trx; ++ty)
            for (int tx = 0; tx < plans[i]->n_trx; ++tx) H.push_back(make_int4(i, tx, ty, 0));
    B.r_dir.second = (int)H.size();
    B.r_ic.first = (int)H.size();
    for (int i : B.order)
        for (int a = 0; a < plans[i]->n_theta; ++a) H.push_back(make_int4(i, a, 0, 0));
    B.r_ic.second = (int)H.size() - B.r_ic.first;
    B.r_vec.first = (int)H.size();
    for (int i : B.order)
        for (int b = 0; b < plans[i]->n_vblocks; ++b) H.push_back(make_int4(i, b, 0, 0));
    B.r_vec.second = (int)H.size() - B.r_vec.first;
    B.r_proj.clear();
    B.r_adj.clear();
    for (int v = 0; v < proj_variant_count(); ++v)
        for (int mp = 2; mp >= 1; --mp) {          // one launch per (variant, maps evaluated)
            const int off = (int)H.size();
            size_t lds = 0;
            for (int i : B.order) {
                const eit_plan* p = plans[i];
                if (p->proj_v != v || p->eval_maps != mp) continue;
                lds = std::max(lds, p->proj_lds);
                for (int g = 0; g < p->n_groups; ++g)
                    for (int b = 0; b < p->n_dblk; ++b) H.push_back(make_int4(i, g, b, 0));
            }
            if ((int)H.size() > off) B.r_proj.emplace_back(v, off, (int)H.size() - off, lds, mp);
        }
    // the angle split only serves launches with few tiles: a batch that fills the chip
    // without it runs every slice unsplit
    long long tiles = 0;
    for (int i = 0; i < n; ++i) tiles += (long long)plans[i]->n_tx * plans[i]->n_ty;
    B.splits.resize(n);
    for (int i = 0; i < n; ++i) B.splits[i] = tiles >= kSplitTarget ? 1 : plans[i]->adj_splits;
    B.r_ring = {(int)H.size(), 0};
    for (int i : B.order)
        for (int b = 0; b < plans[i]->n_it_ring; ++b) H.push_back(make_int4(i, b, 0, 0));
    B.r_ring.second = (int)H.size() - B.r_ring.first;
    B.r_cvec = {(int)H.size(), 0};
    for (int i : B.order)
        for (int b = 0; b < plans[i]->n_it_cvec; ++b) H.push_back(make_int4(i, b, 0, 0));
    B.r_cvec.second = (int)H.size() - B.r_cvec.first;
    for (int v = 0; v < adj_variant_count(); ++v)
        for (int mp = 2; mp >= 1; --mp) {
            const int off = (int)H.size();
            for (int i : B.order) {
                const eit_plan* p = plans[i];
                if (p->adj_v != v || p->eval_maps != mp) continue;
                for (int ty = 0; ty < p->n_ty; ++ty)
                    for (int tx = 0; tx < p->n_tx; ++tx)
                        for (int g = 0; g < B.splits[i]; ++g) H.push_back(make_int4(i, tx, ty, g));
            }
            if ((int)H.size() > off) B.r_adj.emplace_back(v, off, (int)H.size() - off, (size_t)0, mp);
        }
    Layout L;
    B.descs = L.take(sizeof(SliceDesc) * n);
    B.lbdescs = L.take(sizeof(LbDesc) * n);
    B.items = L.take(sizeof(Item) * H.size());
    B.gather = L.take(sizeof(SolverState) * n);    // state read-back staging
    B.slice.resize(n);
    for (int i = 0; i < n; ++i) {
        const size_t base = L.off;
        B.slice[i] = base;
        L.off = base + solve_layout(plans[i], m).end;
        L.off = align_up(L.off, 256);
    }
    B.end = L.off;
    return EIT_OK;
}

}  // namespace

extern "C" size_t eit_batch_workspace_bytes(int32_t n, const eit_plan* const* plans, int32_t m) {
    BatchLayout B;
    if (batch_layout(n, plans, m, B)) return 0;
    return B.end;
}

extern "C" int eit_reconstruct_batch(int32_t n, const eit_plan* const* plans,
                                     const float* const* s_exp, float* const* x,
                                     const eit_opts* o, eit_report* reps, void* ws,
                                     size_t ws_bytes, void* stream) {
    if (int rc = validate_opts(o)) return rc;
    BatchLayout B;
    if (int rc = batch_layout(n, plans, o->lbfgs_m, B)) return rc;
    if (!s_exp || !x) return fail(EIT_ERR_INVALID_ARG, "s_exp or x is NULL");
    for (int i = 0; i < n; ++i)
        if (!s_exp[i] || !x[i]) return fail(EIT_ERR_INVALID_ARG, "s_exp[%d] or x[%d] is NULL", i, i);
    if (int rc = check_ws(ws, ws_bytes, B.end)) return rc;
    hipStream_t st = (hipStream_t)stream;

    std::vector<SliceDesc> dh(n);
    std::vector<LbDesc> lh(n);
    std::vector<SolverState*> states(n);
    for (int i = 0; i < n; ++i) {
        void* base = at(ws, B.slice[i]);
        const SolveLayout S = solve_layout(plans[i], o->lbfgs_m);
        solver_descs(plans[i], o, base, S, s_exp[i], x[i], nullptr, dh[i], lh[i]);
        set_solver_split(dh[i], lh[i], base, S, B.splits[i]);
        states[i] = lh[i].st;
    }
    SliceDesc* dd = (SliceDesc*)at(ws, B.descs);
    LbDesc* ld = (LbDesc*)at(ws, B.lbdescs);
    Item* it = (Item*)at(ws, B.items);
    HIP_TRY(hipMemcpyAsync(dd, dh.data(), sizeof(SliceDesc) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ld, lh.data(), sizeof(LbDesc) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(it, B.items_h.data(), sizeof(Item) * B.items_h.size(),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));      // host staging arrays may be released after this

    HIP_TRY(launch_lb_init(ld, n, o->lbfgs_m, o->max_iter, o->max_ls_trials, o->c1, o->tol_rel_step, st));
    const Item* it_vec = it + B.r_vec.first;
    const int n_vec = B.r_vec.second;
    HIP_TRY(launch_lb_scale(ld, it_vec, n_vec, grid_for(n_vec, kGridCap), 1, st));

    StepPlan sp;
    sp.D = dd; sp.L = ld; sp.n_slices = n;
    sp.gather = at(ws, B.gather);
    for (auto& r : B.r_proj)
        sp.proj.push_back({std::get<0>(r), it + std::get<1>(r), std::get<2>(r), std::get<3>(r), std::get<4>(r)});
    for (auto& r : B.r_adj)
        sp.adj.push_back({std::get<0>(r), it + std::get<1>(r), std::get<2>(r), std::get<3>(r), std::get<4>(r)});
    sp.it_tr = it + B.r_dir.first; sp.n_tr = B.r_dir.second;
    sp.it_ic = it + B.r_ic.first; sp.n_ic = B.r_ic.second;
    sp.it_vec = it_vec; sp.n_vec = n_vec;
    sp.ext = B.ext;
    sp.it_ring = it + B.r_ring.first; sp.n_ring = B.r_ring.second;
    sp.it_cvec = it + B.r_cvec.first; sp.n_cvec = B.r_cvec.second;
    for (int i = 0; i < n; ++i) sp.max_det = std::max(sp.max_det, plans[i]->n_det);
    int launches = 0;
    PhaseTimer timer;
    PhaseTimer* pt = o->profile ? &timer : nullptr;
    GraphKey key;
    key.plans.assign(plans, plans + n);
    key.ws = ws;
    key.m = o->lbfgs_m;
    if (int rc = drive(sp, states, o->max_iter, o->max_ls_trials, o->use_graph != 0, key, st,
                       &launches, pt))
        return rc;
    HIP_TRY(launch_lb_scale(ld, it_vec, n_vec, grid_for(n_vec, kGridCap), 0, st));
    std::vector<SolverState> hs(n);
    SolverState* gathered = (SolverState*)at(ws, B.gather);
    HIP_TRY(launch_gather_states(ld, n, gathered, st));
    HIP_TRY(hipMemcpyAsync(hs.data(), gathered, sizeof(SolverState) * n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int worst = EIT_OK;
    for (int i = 0; i < n; ++i) {
        if (reps) fill_report(hs[i], launches, &reps[i]);
        if (hs[i].status < 0 && worst == EIT_OK) worst = hs[i].status;
    }
    if (pt && reps) {
        if (int rc = pt->collect()) return rc;
        for (int i = 0; i < EIT_N_PHASES; ++i) reps[0].phase_ms[i] = pt->ms[i];
        reps[0].phase_steps = pt->steps;
    }
    if (worst) return fail(worst, "at least one slice stopped with an error (see reports)");
    return EIT_OK;
}

namespace eit {
// error reporting for the network entry points (unet.cpp) through the same thread-local message
int nn_fail(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace eit
