// Internal declarations shared by the library's HIP translation units.
// Device data layouts, per-slice descriptors and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace eit {

// ---------------------------------------------------------------- projector tables
// Joseph ray-driven projection in the "stepping frame": an angle either steps over the
// rows of x (|cos| >= |sin|) or over the rows of x^T. Along a ray for detector t the
// interpolation coordinate at step p is u(t, p) = t*inv + base + p*slope (voxel units),
// and the ray sum is scaled by the step length w.
struct ProjAngle {
    double inv, base, slope;   // FP64 so per-strip origins stay exact to ~1e-12
    float slope_f, w;          // FP32 copies for the inner loop
    int32_t src;               // 0: step over rows of x, 1: rows of x^T
    int32_t pad;
};

// ---------------------------------------------------------------- adjoint tables
// Gather form of R^T: voxel (i, j) projects to detector coordinate
// u = i*cs + j*sn + cd (bins, fractional); it receives from bins floor(u) and floor(u)+1
// with triangle weights (1/w) max(0, 1 - |k - u|/w).
// Mirror frame of the same angle (cos -> -cos): u_s = -i*cs + j*sn + cd_s. Voxel (i, j) at
// the mirror angle pi - theta and voxel (i, n-1-j) at theta project to u_s and n_det-1-u_s.
struct AdjAngle {
    double cs, sn, cd;         // FP64 for the per-tile window origin
    double cd_s;               // mirror-frame offset
    float cs_f, sn_f;          // FP32 for the inner loop
    float iw, iw2, iwm;        // 1/w, 1/w^2, 1/w - 1/w^2
    float omw;                 // 1 - 1/w
};

// Tile shapes (compile-time variants, chosen per grid-size class).
struct ProjTile { int A, W, R, PW, DUP, LP, IL; };  // angles per group, detectors per block, rows per
                                                   // strip, staged width, 16-byte entries, LDS row
                                                   // pitch, interleaved rays (8 angles per wavefront)
struct AdjTile  { int TX, TY, AC, VPT, MIR; }; // voxel tile, angles (or angle pairs) per staged
                                              // chunk, voxels per thread, mirror pairs 0/1

// ---------------------------------------------------------------- per-slice descriptor
// Everything a kernel needs for one slice. Lives in device memory; kernels index it by the
// slice id of their work item, so one launch can serve many slices.
struct SliceDesc {
    int32_t n, n_theta, n_det, n_mask;
    float kappa;
    double scale_mu, scale_de;     // P_raw = scale * R x   (1 for raw units)
    double reg_mu, reg_de;         // gradient adds reg * x  (2 lambda)
    double lam_mu, lam_de;         // cost adds lam * ||x||^2
    int32_t proj_tile, adj_tile;   // variant ids
    // projector work decomposition
    int32_t n_groups, n_dblk, n_strips, win_w;
    int32_t win_shift;             // log2 of the staging row pitch (>= win_w)
    // adjoint work decomposition
    int32_t n_tx, n_ty, n_chunks, kwin;
    // plan tables (device, owned by the plan)
    const ProjAngle* pang;         // [n_theta]
    const int32_t* groups;         // [n_groups][A] angle ids (-1 = empty slot)
    const int32_t* win_lo;         // [n_groups][n_dblk][n_strips]
    const AdjAngle* aang;          // [n_theta]
    const float4* flat;            // [n_det] (A, c, 1/(2 s^2), 1/s^2)
    const double* mask;            // [n_mask] mask positions
    // per-call buffers (device)
    const float* x;                // [2][n][n] point of evaluation
    float* xT;                     // [2][n][n] transposed copy (projector source)
    float* P;                      // [2][n_theta][n_det] projections, then adjoint seeds
    const float* s_exp;            // [n_theta][n_mask][n_det]
    float* g;                      // [2][n][n] gradient (or backprojection) output
    double* part_ic;               // [n_theta] data-term partials
    double* part_reg;              // [n_reg_blocks][2] ||mu||^2, ||delta||^2 partials
    int32_t n_reg_blocks;
    int32_t maps;                  // maps evaluated: 2 (mu, delta; also the default), or 1 in
                                   // h-mode (R h once; P_delta = gamma scale R h, seeds summed)
    double* cost;                  // scalar cost
    const int32_t* skip;           // optional device flag: nonzero => kernels no-op
    const int32_t* skip_adj;       // optional: nonzero => adjoint no-ops
    // adjoint angle split: G = adj_splits blocks per voxel tile (1 = no split)
    int32_t adj_splits, n_pairs;   // n_pairs: entries of apairs (mirror-pair adjoint only)
    const int2* apairs;            // [n_pairs] (angle, mirror angle or -1)
    double* bp_part;               // [G][maps][n][n] FP64 partial sums of the adjoint (G > 1)
    // Full model of eq. 4 (ext != 0; the plain two-map model leaves every field below zero).
    // The unknowns form one parameter vector xu: the maps (two, or h alone in h-mode, which
    // is evaluated once by the single-map kernels, maps == 1, or as the expanded pair [h, h],
    // with P_delta scaled by gamma), then the per-angle drift m_o and the per-pixel ring term
    // m_r when fitted.
    int32_t ext;                   // EXT_* flags
    int32_t nq;                    // tabulated flat: samples per pixel
    double tab_u0, tab_du;         // sample q of the table sits at u = tab_u0 + q tab_du
    const double* ftab;            // [n_det][nq] measured flat IC (EXT_TABLE)
    const float* xu;               // parameter vector of the evaluation point
    float* xe;                     // [2][n][n] expanded maps (h-mode pair evaluation)
    const float* off;              // offsets of the point: m_o [n_theta] then m_r [n_det]
    double off_scale;              // raw offset = off_scale * off
    double* g_mo;                  // [n_theta] sum over pixels of G_Delta (drift)
    double* g_dl;                  // [n_theta][n_det] G_Delta (ring)
    float* gu;                     // gradient in the parameter vector's layout
    int64_t nvu;                   // entries of the parameter vector
};

// SliceDesc::ext flags.
constexpr int EXT_HMODE = 1, EXT_DRIFT = 2, EXT_RING = 4, EXT_TABLE = 8;
// h-mode plans evaluate R h once (single-map kernels) up to this many detector pixels, beyond
// it through the pair [h, h] (the eq. 4 IC stage keeps two rows of doubles in LDS)
constexpr int kSingleMapMaxDet = 2048;

// Work items: (slice, a, b, c) -- meaning depends on the kernel.
using Item = int4;

// ---------------------------------------------------------------- optimiser state
constexpr int kMaxM = 20;                // largest L-BFGS memory
constexpr int kVecChunk = 2048;          // vector elements per work item (256 threads x 8)
constexpr int kVecThreads = 256;
constexpr int kDotsFixed = 7;            // gg, ss, yy, sy, zz, s.g, y.g
constexpr int kSlotBatch = 10;           // history slots whose vectors are loaded together
constexpr int max_dots(int m) { return kDotsFixed + 4 * m; }

enum SolverMode : int32_t { MODE_INIT = 0, MODE_NEW_DIR = 1, MODE_BACKTRACK = 2 };
enum SolverStatus : int32_t { ST_RUNNING = 0, ST_DONE = 1 };   // errors use EIT_ERR_* (< 0)

// Device-resident L-BFGS state of one slice (compact representation, FP64 scalars).
// The (s, y) vectors live in m+1 slots; `order` lists the committed slots oldest first and
// `spare` is the slot that receives the next candidate pair.
struct SolverState {
    double f, f_t, alpha, gd, gamma, gg, c1, tol;
    double cc[kMaxM], ee[kMaxM];                 // d = -gamma g - sum ee_r s_r + sum cc_r y_r
    double SY[(kMaxM + 1) * (kMaxM + 1)];        // s_i . y_j by slot (i <= j used)
    double YY[(kMaxM + 1) * (kMaxM + 1)];        // y_i . y_j by slot
    double* cost_hist;                           // optional [max_iter + 1]
    int32_t k, evals, trials, mode, status, m_cur, m, max_iter, max_ls, accept, spare, launches;
    int32_t order[kMaxM];
    int32_t skip, skip_adj;                      // step-level no-op flags read by every kernel
};

// Per-slice optimiser buffers.
struct LbDesc {
    int64_t nv;                  // entries of the optimiser's vectors (2 n^2 for the plain model)
    int32_t n, n_vblocks;
    float scale_mu, scale_de;    // z = x / scale: first map, second map (or h-mode's h alone)
    int64_t nn;                  // n^2
    int32_t n_maps;              // maps in the vector (2, or 1 in h-mode); offsets follow
    float scale_off;             // scaling of the offsets (full model)
    float* z;  float* zt;  float* g;  float* gt;  float* d;
    float* S;  float* Y;         // [(m+1)][nv] each
    double* part;                // [n_vblocks][max_dots(m)]
    SolverState* st;
    float* x_user;               // raw-unit iterate (in/out)
    double* cost_hist;           // optional [max_iter + 1]
    // split adjoint (gsplits > 1): the gradient at zt is sum_g gpart[g] + reg * zt, formed
    // here instead of in gt
    const double* gpart;         // [gsplits][nv]
    int32_t gsplits, pad;
    double reg_mu, reg_de;
};

hipError_t launch_lb_init(const LbDesc* L, int n_slices, int m, int max_iter, int max_ls, double c1,
                          double tol, hipStream_t s);
hipError_t launch_lb_scale(const LbDesc* L, const Item* items, int n_items, int grid, int to_z,
                           hipStream_t s);
hipError_t launch_lb_direction(const LbDesc* L, const SliceDesc* D, const Item* items, int n_items,
                               int grid, hipStream_t s);
hipError_t launch_lb_update(const LbDesc* L, const Item* items, int n_items, int grid,
                            hipStream_t s);
hipError_t launch_lb_decide(const SliceDesc* D, const LbDesc* L, int n_slices, hipStream_t s);
hipError_t launch_lb_finalize(const LbDesc* L, int n_slices, hipStream_t s);
// batch read-back: 5 status ints per slice into out[5 n], or whole states into out[n]
hipError_t launch_gather_status(const LbDesc* L, int n_slices, int32_t* out, hipStream_t s);
hipError_t launch_gather_states(const LbDesc* L, int n_slices, SolverState* out, hipStream_t s);
hipError_t launch_lb_direction_vec(const LbDesc* L, const SliceDesc* D, const Item* items,
                                   int n_items, int grid, hipStream_t s);

// full model of eq. 4 (model_ext.hip)
hipError_t launch_ext_expand(const SliceDesc* D, const Item* items, int n_items, int grid,
                             hipStream_t s);
hipError_t launch_ic_ext(const SliceDesc* D, const Item* items, int n_items, int grid,
                         int want_seeds, int max_det, hipStream_t s);   // max_det: widest slice
hipError_t launch_ext_contract(const SliceDesc* D, const Item* items, int n_items, int grid,
                               hipStream_t s);
constexpr int kContractChunk = 256;     // parameter-vector entries per item of the contraction
hipError_t launch_ext_ring_grad(const SliceDesc* D, const Item* items, int n_items, int grid,
                                hipStream_t s);
constexpr int kRingPixPerItem = 64;     // pixels per item of launch_ext_ring_grad
hipError_t launch_eq3_retrieve(const SliceDesc* D, const Item* items, int n_items, int grid,
                               const double* kern, const double* inv_flat, int mask_index,
                               hipStream_t s);
hipError_t launch_ext_take_maps(const SliceDesc* D, const Item* items, int n_items, int grid,
                                hipStream_t s);
hipError_t launch_store_desc(const SliceDesc& v, SliceDesc* dst, hipStream_t s);
hipError_t launch_store_lbdesc(const LbDesc& v, LbDesc* dst, hipStream_t s);

// ---------------------------------------------------------------- launchers (kernels.hip)
hipError_t launch_transpose(const SliceDesc* d_descs, const Item* items, int n_items,
                            int grid, hipStream_t s);
// maps: 2 (the pair of maps) or 1 (map 0 only; its projections land in plane 0)
hipError_t launch_project(int variant, int maps, const SliceDesc* d_descs, const Item* items,
                          int n_items, int grid, size_t lds_bytes, hipStream_t s);
hipError_t launch_ic(const SliceDesc* d_descs, const Item* items, int n_items, int grid,
                     int want_seeds, hipStream_t s);
hipError_t launch_cost_reduce(const SliceDesc* d_descs, int n_slices, hipStream_t s);
// maps: 2 (both seed planes into both gradient planes) or 1 (seed plane 0 into plane 0)
hipError_t launch_backproject(int variant, int maps, const SliceDesc* d_descs, const Item* items,
                              int n_items, int grid, int add_reg, hipStream_t s);
hipError_t launch_bp_combine(const SliceDesc* d_descs, const Item* vec_items, int n_items, int grid,
                             int add_reg, hipStream_t s);

// single-shot reconstruction (single_shot.hip)
hipError_t launch_ss_retrieve(const SliceDesc* D, const Item* items, int n_items, int grid,
                              hipStream_t s);
hipError_t launch_ss_filter(const SliceDesc* D, const Item* items, int n_items, int grid,
                            hipStream_t s);

// projector/adjoint variant registry
int proj_variant_count();
ProjTile proj_variant(int v);
int adj_variant_count();
AdjTile adj_variant(int v);
int adj_pitch_limit(int v);   // compile-time LDS pitch capacity of adjoint variant v

constexpr int kIcThreads = 512;
constexpr int kTrThreads = 256;      // transpose tile 32x32, 256 threads
constexpr int kTrTile = 32;

}  // namespace eit
