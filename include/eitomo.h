/*
 * eitomo.h -- C ABI of the MI355X (gfx950) library for model-based iterative
 * edge-illumination (EI) X-ray tomography (Modregger et al., "Accelerated iterative
 * tomographic reconstruction with x-ray edge illumination", arXiv 2202.08627).
 *
 * The library reconstructs, slice by slice, an absorption map mu and a phase map delta
 * (refractive-index decrement) from edge-illumination data s_exp(t, theta, m) by
 * minimising the least-squares cost of eq. 5 under the forward model of eq. 2 (eq. 4 with
 * the drift m_o and ring term m_r set to zero):
 *     s_mod(t, theta, m) = exp(-R[mu](t, theta)) * f_t(m - kappa * d/dt R[delta](t, theta))
 * where R is the parallel-beam Radon transform of eq. 1 and f_t is the flat-field
 * illumination curve of detector pixel t.
 *
 * Conventions (the paper fixes no discretisation; these are the library's):
 *   - Unit voxel and detector pitch. Voxel (i, j) (column i = x, row j = y) has centre
 *     (i - (n-1)/2, j - (n-1)/2); maps are stored planar and row-major, x[c][j][i],
 *     c = 0 for mu and c = 1 for delta, i.e. float[2][n][n].
 *   - Detector pixel k sits at t_k = k - (n_det-1)/2; angle theta_a (radians); the ray is
 *     the line x cos(theta) + y sin(theta) = t.
 *   - R is Joseph's ray-driven projector: linear interpolation along the axis the ray
 *     crosses more slowly, interpolation indices computed on the fly (no system matrix,
 *     as the algorithmic-improvements section recommends). Sinograms are float[2][n_theta][n_det].
 *   - d/dt is the central difference with zero padding (the paper's finite differences).
 *   - IC data are float[n_theta][n_mask][n_det]; the flat IC of pixel k is the Gaussian
 *     A_k exp(-(u - c_k)^2 / (2 sigma_k^2)), u in mask periods.
 *   - kappa converts the projected-phase slope into a shift in mask periods (z in eq. 2).
 *
 * Memory and ownership: all array arguments documented "device" are device pointers
 * (HIP global memory) owned by the caller; the library never frees them. Arguments
 * documented "host" are host pointers read during the call only. Apart from the plan's
 * own small tables (angle and detector tables allocated in eit_plan_create) the library
 * allocates no device memory: scratch space is the caller's workspace `ws`, at least
 * eit_workspace_bytes() bytes, 256-byte aligned, and it must not be used concurrently by
 * two calls.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream). Calls enqueue work on it
 * and return without synchronising, except eit_reconstruct and eit_reconstruct_batch,
 * which synchronise the stream once at the end to fill the host report.
 *
 * Errors: every int-returning call returns EIT_OK (0) or a negative EIT_ERR_* code;
 * eit_last_error() returns a thread-local message for the last failure on the calling
 * thread. Argument validation happens on the host before any device work is enqueued;
 * on a validation error nothing is enqueued. No C++ exception crosses this interface.
 */
#ifndef EITOMO_H
#define EITOMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EIT_OK 0
#define EIT_ERR_INVALID_ARG (-1) /* null pointer, non-finite or out-of-range scalar */
#define EIT_ERR_SHAPE (-2)       /* inconsistent or unsupported sizes */
#define EIT_ERR_DEVICE (-3)      /* a HIP runtime call failed (message has the hipError_t) */
#define EIT_ERR_NOMEM (-4)       /* workspace too small / plan table allocation failed */
#define EIT_ERR_NONFINITE (-5)   /* cost is NaN or Inf at the starting point */
#define EIT_ERR_LINESEARCH (-6)  /* no step satisfied the Armijo test from an empty memory */

/* Limits checked by eit_plan_create. */
#define EIT_MAX_N 4096
#define EIT_MAX_NDET 4096
#define EIT_MAX_NTHETA 16384
#define EIT_MAX_NMASK 64
#define EIT_MAX_LBFGS_M 20
#define EIT_MAX_NTABLE 1024

typedef struct eit_plan eit_plan;

/* Problem sizes. n: grid n x n voxels; n_theta angles; n_det detector pixels; n_mask
 * sample-mask positions per IC; kappa: refraction scale (mask periods per unit slope of
 * the projected delta). */
typedef struct {
    int32_t n, n_theta, n_det, n_mask;
    double kappa;
} eit_dims;

/* Acquisition set-up (all host, FP64, read during eit_plan_create only).
 * theta: [n_theta] radians, or NULL for theta_a = a*pi/n_theta (180 degrees, endpoint
 *        excluded).
 * mask_pos: [n_mask] mask offsets in periods, or NULL for (j + 0.5)/n_mask - 0.5.
 * flat_amp, flat_ctr, flat_sigma: [n_det] Gaussian flat-field IC parameters per pixel
 *        (required; sigma > 0, amp > 0). */
typedef struct {
    const double* theta;
    const double* mask_pos;
    const double* flat_amp;
    const double* flat_ctr;
    const double* flat_sigma;
} eit_setup;

/* Optional tile-shape selection (autotuner output); NULL or -1 fields = defaults.
 * proj_variant / adj_variant index the library's compiled projector / adjoint tile
 * variants (see eit_variant_info). adj_splits divides the angles of every adjoint voxel
 * tile among that many blocks (1 .. 64, clamped to the number of angle chunks; <= 0 =
 * automatic: doubled, up to 8, while the launch has under 1024 blocks and each part keeps
 * two chunks). With more than one part each block stores FP64 partial sums in the
 * workspace and a following pass adds them in part order, so results do not depend on
 * block scheduling. */
typedef struct {
    int32_t proj_variant;
    int32_t adj_variant;
    int32_t adj_splits;
} eit_tiling;

/* The paper's full forward model (theory section, eq. 4), for eit_plan_create_model:
 *     s_mod(t, theta, m) = exp(-R[mu]) f_t(m - m_o(theta) - m_r(t) - kappa d/dt R[delta])
 * hmode: nonzero for the homogeneous-object assumption that leads to eq. 4 and eq. 3: one
 *        map h with mu = h and delta = gamma*h (gamma > 0). The gradient in h is the mu
 *        gradient plus gamma times the delta gradient.
 * fit_drift: nonzero makes the per-angle offset of the sample mask m_o(theta) (the drift the
 *        paper fits, eq. 4) n_theta more unknowns.
 * fit_ring: nonzero makes the per-pixel offset m_r(t) (eq. 4's ring-artefact term) n_det
 *        more unknowns. With both offsets the cost has the paper's ambiguity m_o + c, m_r - c.
 * n_table: 0 keeps the Gaussian flats of eit_setup; >= 4 (<= EIT_MAX_NTABLE) replaces them
 *        by a measured flat IC, flat_table (host, [n_det][n_table], FP64, read during the
 *        call), sample q taken at mask offset table_u0 + q*table_du (table_du > 0; the
 *        experiment section scans one period in 33 steps). The model interpolates it by
 *        cubic convolution (Keys 1981, a = -1/2) and holds the end values outside the scan
 *        (slope 0 there). eit_setup's Gaussian parameters may then be NULL.
 * offset_scale: optimiser scaling of the offsets, z = m / offset_scale (0 means 1).
 * eq3_mask: h-mode single shot (eq. 3): index of the mask position it reads.
 * Parameter vector (x and gradient of eit_cost_and_grad, x of eit_reconstruct, x_out of
 * eit_single_shot): the maps (float[2][n][n], or float[n][n] h in h-mode), then m_o
 * [n_theta] if fitted, then m_r [n_det] if fitted; eit_param_count gives its length.
 * eit_project and eit_backproject keep applying R and R^T to two maps. A batch
 * (eit_reconstruct_batch) takes either only plain plans or only model plans. */
typedef struct {
    int32_t hmode;
    int32_t fit_drift;
    int32_t fit_ring;
    int32_t n_table;
    double gamma;
    const double* flat_table;
    double table_u0, table_du;
    double offset_scale;
    int32_t eq3_mask;
    int32_t pad;
} eit_model;

/* Optimiser options for eit_reconstruct (L-BFGS on the scaled unknowns
 * z = [mu / mu_scale ; delta / delta_scale], cost weight lam on ||z||^2, i.e.
 * lambda_mu = lam / mu_scale^2 and lambda_delta = lam / delta_scale^2 in eq. 5). */
typedef struct {
    int32_t max_iter;       /* accepted iterations to run (>= 0) */
    int32_t lbfgs_m;        /* memory pairs, 1 .. EIT_MAX_LBFGS_M */
    int32_t max_ls_trials;  /* Armijo backtracking trials per line search (>= 0) */
    int32_t use_graph;      /* nonzero: replay one captured HIP graph per evaluation */
    double lam;             /* >= 0 */
    double mu_scale, delta_scale;   /* > 0 */
    double tol_rel_step;    /* stop when ||z_{k+1}-z_k|| / ||z_k|| < tol (0 = off) */
    double c1;              /* Armijo constant, 0 < c1 < 1 (typ. 1e-4) */
    int32_t profile;        /* nonzero: direct launches bracketed by hipEvents per phase
                               (fills eit_report.phase_ms; use_graph is ignored) */
    int32_t pad;
} eit_opts;

/* Phases of one evaluation step, in launch order (indices of eit_report.phase_ms). */
#define EIT_PHASE_DIRECTION 0   /* L-BFGS direction, trial point, its transpose and norms */
#define EIT_PHASE_TRANSPOSE 1   /* folded into EIT_PHASE_DIRECTION (reported as 0) */
#define EIT_PHASE_PROJECT 2     /* Radon transform of both maps */
#define EIT_PHASE_IC 3          /* IC model, residual, cost partials, adjoint seeds */
#define EIT_PHASE_DECIDE 4      /* cost reduction and Armijo decision */
#define EIT_PHASE_BACKPROJECT 5 /* adjoint backprojection (gradient) */
#define EIT_PHASE_UPDATE 6      /* accepted step: s, y, inner products */
#define EIT_PHASE_FINALIZE 7    /* memory update and next direction coefficients */
#define EIT_N_PHASES 8

/* Host report filled by eit_reconstruct after its final stream synchronisation. */
typedef struct {
    int32_t status;         /* EIT_OK or EIT_ERR_LINESEARCH / EIT_ERR_NONFINITE */
    int32_t iters;          /* accepted iterations */
    int32_t evals;          /* cost+gradient evaluations (line-search trials included) */
    int32_t launches;       /* evaluation steps enqueued (no-op steps included) */
    double cost;            /* final cost F(z) */
    double gnorm;           /* final ||grad_z F|| */
    double phase_ms[EIT_N_PHASES];   /* profile mode: summed device time per phase */
    int32_t phase_steps;    /* profile mode: steps timed */
    int32_t pad;
} eit_report;

/* Create a plan: validates sizes, computes the angle/detector tables in FP64 on the host
 * and uploads them (the plan's only device allocations). Requires a current HIP device.
 * Returns EIT_ERR_SHAPE / EIT_ERR_INVALID_ARG on bad input, EIT_ERR_DEVICE on HIP failure. */
int eit_plan_create(const eit_dims* dims, const eit_setup* setup, const eit_tiling* tiling,
                    eit_plan** out);
void eit_plan_destroy(eit_plan* plan);

/* As eit_plan_create, for the full model of eq. 4 described by *model (required, host, read
 * during the call). Errors as eit_plan_create, plus EIT_ERR_INVALID_ARG for invalid model
 * options and EIT_ERR_SHAPE for n_table outside [4, EIT_MAX_NTABLE]. */
int eit_plan_create_model(const eit_dims* dims, const eit_setup* setup, const eit_model* model,
                          const eit_tiling* tiling, eit_plan** out);

/* Entries of the plan's parameter vector: 2 n^2 for a plain plan; for a model plan the maps
 * (n^2 in h-mode, else 2 n^2) plus n_theta drift and n_det ring offsets when fitted. 0 for
 * a NULL plan. Host only. */
int64_t eit_param_count(const eit_plan* plan);

/* Operation codes for eit_workspace_bytes. */
#define EIT_OP_PROJECT 1
#define EIT_OP_BACKPROJECT 2
#define EIT_OP_COST_GRAD 3
#define EIT_OP_RECONSTRUCT 4
#define EIT_OP_SINGLE_SHOT 5

/* Workspace bytes needed by an operation (lbfgs_m used by EIT_OP_RECONSTRUCT only).
 * Returns 0 for an invalid plan or op. */
size_t eit_workspace_bytes(const eit_plan* plan, int32_t op, int32_t lbfgs_m);

/* Radon transform R (eq. 1) of both maps: x device float[2][n][n] ->
 * sino device float[2][n_theta][n_det]. */
int eit_project(const eit_plan* plan, const float* x, float* sino, void* ws, size_t ws_bytes,
                void* stream);

/* Exact transpose R^T of eit_project's operator (gather form, no atomics):
 * sino device float[2][n_theta][n_det] -> x_out device float[2][n][n].
 * Theory section: the paper minimises eq. 5 with its analytic gradient; by the chain rule
 * through eq. 1 and eq. 2 that gradient is R^T applied to the derivatives of the cost with
 * respect to the projections (the IC residual seeds), which is this operator. It is also the
 * backprojection of the single-shot route's filtered backprojection (Kak & Slaney, the
 * paper's Radon reference). Asynchronous; errors as for eit_project. */
int eit_backproject(const eit_plan* plan, const float* sino, float* x_out, void* ws,
                    size_t ws_bytes, void* stream);

/* Cost of eq. 5 (model of eq. 2/4 with m_o = m_r = 0) at x = [mu; delta] (device
 * float[2][n][n], raw units) for data s_exp (device float[n_theta][n_mask][n_det]):
 *   S = sum (s_mod - s_exp)^2 + lam_mu ||mu||^2 + lam_delta ||delta||^2
 * written as one FP64 value to cost_dev (device double*), reduced deterministically.
 * If grad is non-NULL (device float[2][n][n]) the analytic gradient dS/dx is written too
 * (adjoint backprojection of the IC residual seeds). Asynchronous; never syncs. */
int eit_cost_and_grad(const eit_plan* plan, const float* x, const float* s_exp, double lam_mu,
                      double lam_delta, double* cost_dev, float* grad, void* ws, size_t ws_bytes,
                      void* stream);
/* With a model plan, x and grad are parameter vectors (eit_param_count entries, raw units)
 * and the model is eq. 4 with the plan's options; in h-mode lam_mu weights ||h||^2 and
 * lam_delta is unused; the offsets are not regularised. */

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): eit_cost_and_grad with its scratch
 * buffers in a static device array of EIT_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends, instead of a caller workspace. Same
 * arguments and results as eit_cost_and_grad (same kernels and buffer layout, so the outputs
 * are identical). Calls nothing that allocates. Returns EIT_ERR_NOMEM, before enqueueing
 * anything, when eit_workspace_bytes(plan, EIT_OP_COST_GRAD, 0) exceeds the limit (e.g.
 * 1024^2 / 1800 angles with a split adjoint), EIT_ERR_DEVICE if the array's device address
 * cannot be looked up. All calls on one GPU share the array: calls that overlap on one GPU
 * (two streams, two threads) race and must be serialised by the caller. */
#define EIT_NOALLOC_SCRATCH_BYTES (32u << 20)
int eit_cost_and_grad_noalloc(const eit_plan* plan, const float* x, const float* s_exp,
                              double lam_mu, double lam_delta, double* cost_dev, float* grad,
                              void* stream);

/* Non-iterative reconstruction (the paper's single-shot route: retrieve each projection
 * pixel, then filtered backprojection), used as the start of the learned warm start.
 * With several mask positions per IC both channels are retrieved per pixel: a weighted
 * least-squares fit of log s_j (weights s_j) to the log of the shifted, attenuated Gaussian
 * flat IC gives T and Delta; P_mu = -log T, P_delta = trapezoid integral of Delta/kappa along
 * t minus the ramp that zeroes both ends; each is filtered with the Ram-Lak kernel (Kak &
 * Slaney, unit spacing), scaled by pi/n_theta and backprojected with R^T.
 * s_exp device float[n_theta][n_mask][n_det] -> x_out device float[2][n][n].
 * Workspace: eit_workspace_bytes(plan, EIT_OP_SINGLE_SHOT, 0). Asynchronous. */
int eit_single_shot(const eit_plan* plan, const float* s_exp, float* x_out, void* ws,
                    size_t ws_bytes, void* stream);
/* With an h-mode model plan the route is eq. 3 (single-shot retrieval from one mask
 * position, eq3_mask, for a homogeneous object): r = s / f_t(m) per pixel, then in Fourier
 * space along t, T = F^-1[F[r] / (1 + i kappa gamma (f'/f) sin q)] with f, f' the detector-
 * averaged flat and slope at m (sin q: the symbol of the central difference), R[h] = -log T
 * (T held at >= 1e-6); h = Ram-Lak filtered backprojection of R[h] (as above). x_out is a
 * parameter vector: the map(s), offsets set to 0. A two-map model plan takes the per-pixel
 * fit above and needs the Gaussian flat parameters (EIT_ERR_INVALID_ARG otherwise). */

/* Minimise the cost of eq. 5 from x (device float[2][n][n], raw units): x holds the start on
 * entry and x_K on return. Theory section: the paper minimises eq. 5 with L-BFGS (SciPy's
 * implementation) using the analytic gradient, and states no settings; here L-BFGS with
 * memory opts->lbfgs_m (compact representation, FP64 dot products, H_0 = (s.y / y.y) I),
 * first trial step 1/||g|| from an empty memory and 1 otherwise, Armijo backtracking by
 * halving (constant opts->c1, at most opts->max_ls_trials trials; when every trial fails the
 * memory is cleared and the iteration redone along -g, or the run stops with
 * EIT_ERR_LINESEARCH if the memory was empty), a pair kept only if s.y > 1e-10 |s||y|, entirely
 * device-resident; one accepted step per iteration. Synchronises `stream` at the end and fills
 * *rep (host, may be NULL). cost_hist (device double[max_iter + 1], may be NULL) receives F
 * after the start evaluation and after every accepted iteration. The captured graphs of the
 * evaluation steps are kept per (plan, workspace address, lbfgs_m) and replayed by later calls
 * with the same three (at most 16 kept; eit_plan_destroy drops a plan's). Returns
 * EIT_ERR_NONFINITE if the cost at the start is not finite. */
int eit_reconstruct(const eit_plan* plan, const float* s_exp, const eit_opts* opts, float* x,
                    double* cost_hist, eit_report* rep, void* ws, size_t ws_bytes, void* stream);
/* With a model plan, x is a parameter vector (start in, x_K out); the scaled unknowns are
 * h / mu_scale in h-mode (delta_scale unused) and the offsets / offset_scale, and lam weights
 * the squared norm of the scaled maps only. */

/* Many independent slices (3-D as a stack of 2-D problems, combined-results section) in
 * one sequence of persistent launches, optionally replayed from one captured HIP graph.
 * plans/s_exp/x/reps are host arrays of n_slices entries (s_exp[i], x[i] device pointers
 * as in eit_reconstruct; reps may be NULL). Slices may differ in every size, and in their
 * model options if every plan is a model plan (EIT_ERR_INVALID_ARG for a mix of plain and
 * model plans). Workspace:
 * eit_batch_workspace_bytes. Each slice runs its own optimiser state and line search. */
size_t eit_batch_workspace_bytes(int32_t n_slices, const eit_plan* const* plans, int32_t lbfgs_m);
int eit_reconstruct_batch(int32_t n_slices, const eit_plan* const* plans,
                          const float* const* s_exp, float* const* x, const eit_opts* opts,
                          eit_report* reps, void* ws, size_t ws_bytes, void* stream);

/* Host-only diagnostic (no device needed): validates like eit_plan_create and reports the
 * tiling-dependent sizes and the FP64 tables the plan would upload, so that launch shapes
 * and LDS bounds can be checked on the host. Output arrays may be NULL; if given they need
 * 6*n_theta doubles (per angle: inv, base, slope, slope as float, step weight, source 0/1),
 * n_groups*proj_a int32 (angle ids, -1 = empty), n_groups*n_dblk*n_strips int32 (window
 * origins) and 10*n_theta doubles (per angle: cos, sin, offset, cos as float, sin as float,
 * 1/w, 1/w^2, 1/w - 1/w^2, mirror-frame offset, mirror partner). The mirror-frame offset
 * cd_s places voxel (i, j) at detector coordinate -i cos + j sin + cd_s (the angle pi - theta).
 * The mirror partner is filled for mirror-pair adjoint variants (adj_mirror = 1): the later
 * angle b with cos b = -cos a and sin b = sin a that angle a is paired with, -1 if a has none,
 * -2 if a is itself the partner of an earlier angle; n_pairs counts the angles that are not -2.
 * Otherwise it is -1 for every angle. Call once with NULL arrays to learn the sizes. */
typedef struct {
    int32_t proj_variant, adj_variant;
    int32_t proj_a, proj_w, proj_r;
    int32_t adj_tx, adj_ty, adj_ac;
    int32_t n_groups, n_dblk, n_strips, win_w, win_pitch;
    int32_t kwin, kwin_pitch_limit, n_tx, n_ty;
    int32_t adj_splits;
    int32_t adj_mirror, n_pairs;
    int64_t proj_lds_bytes;
} eit_plan_info;
int eit_plan_inspect(const eit_dims* dims, const eit_setup* setup, const eit_tiling* tiling,
                     eit_plan_info* info, double* proj_angles, int32_t* groups, int32_t* win_lo,
                     double* adj_angles);

/* ---------------------------------------------------------------------------------------
 * Image quality (combined-results and experiment sections), for reconstructions of synthetic
 * phantoms; both run on `stream` and write their results to device memory.
 *
 * Fourier ring correlation of eq. 6 between two n x n images a and b (device float, row-
 * major, 2 <= n <= EIT_MAX_FRC_N): FRC(r) = sum_ring Re(F_a F_b*) / sqrt(sum_ring |F_a|^2 *
 * sum_ring |F_b|^2), F the 2-D DFT, ring r the frequencies (kx, ky) (signed, DFT order) with
 * round(sqrt(kx^2 + ky^2)) = r, r = 0 .. n/2 (the printed equation omits the ring sums and
 * the real part; this is the standard definition the paper cites). curve and smooth: device
 * double[n/2 + 1], the curve and its Gaussian smoothing over rings 1 .. n/2 (width sigma
 * rings, weights renormalised at the ends; ring 0 kept). res: device double[2], the
 * resolution n / r_c in pixels and r_c, the first ring (linear interpolation) at which the
 * smoothed curve drops below cutoff (0.5 in the paper), or n/2 if it never does. Workspace:
 * eit_frc_workspace_bytes(n) (0 for an invalid n), 256-byte aligned. Deterministic (fixed
 * summation orders). */
#define EIT_MAX_FRC_N 1024
size_t eit_frc_workspace_bytes(int32_t n);
int eit_frc(int32_t n, const float* a, const float* b, double* curve, double* smooth, double* res,
            double cutoff, double sigma, void* ws, size_t ws_bytes, void* stream);

/* Contrast-to-noise ratio of eq. 7 in the n x n image img (device float): CNR =
 * |mean_1 - mean_2| / sqrt(std_1^2 + std_2^2) over the pixels whose centres lie within rho of
 * (x1, y1) and of (x2, y2) (centred coordinates: pixel (i, j) at (i - (n-1)/2, j - (n-1)/2)),
 * population standard deviations. out: device double[1]. EIT_ERR_INVALID_ARG if a disc holds
 * no pixel centre (checked on the host). */
int eit_cnr(int32_t n, const float* img, double x1, double y1, double x2, double y2, double rho,
            double* out, void* stream);

/* Thread-local message describing the last non-zero return on this thread. */
const char* eit_last_error(void);

/* Compiled tile variants: kind 0 = projector (a = angles per group, b = detectors per
 * block, c = rows per strip, d = staged entries per row), kind 1 = adjoint (a, b = voxel tile,
 * c = angles per chunk, d = voxels per thread), kind 2 = projector LDS layout (a = 1 if a
 * sample reads one 16-byte entry holding both neighbouring columns, 0 if it reads two 8-byte
 * (mu, delta) pairs; b = entries per LDS row, the widest window the variant accepts, at most
 * the staged width d of kind 0; c = 1 if a wavefront follows 8 detectors of 8 angles instead
 * of 64 detectors of one angle), kind 3 = adjoint kernel form (a = 1 for the mirror-pair
 * kernel: each voxel with its row mirror and each angle with its mirror angle pi - theta; its
 * c of kind 1 counts angle pairs). Returns the number of variants of that kind; fills a/b/c/d
 * (each may be NULL) for index v if in range. */
int eit_variant_info(int32_t kind, int32_t v, int32_t* a, int32_t* b, int32_t* c, int32_t* d);

/* ---------------------------------------------------------------------------------------
 * Learned warm start. Not part of the paper's method: a 2-D U-Net maps the two-channel
 * single-shot reconstruction (eq. 3 style retrieval followed by filtered backprojection,
 * eit_single_shot) to a starting point for the iterative minimisation of eq. 5.
 * Architecture: 4 levels with base, 2*base, 4*base, 8*base channels; two 3x3 convolutions
 * (zero padding) with ReLU per level; 2x2 max pooling down; 2x2 stride-2 transposed
 * convolutions up, concatenated before the skip connection ([up, skip] channel order); a
 * 1x1 head with two outputs added to the input (residual). Products in BF16 on the matrix
 * cores with FP32 accumulation; parameters, gradients and Adam moments in FP32.
 *
 * Parameter vector (FP32, device): layers in the order returned by eit_unet_layers, each
 * its weights followed directly by its bias (cout floats):
 *   kind 0, 3x3 conv:        W[cout][ky*3 + kx][cin]
 *   kind 1, 2x2 up-conv:     W[cout][dy*2 + dx][cin]   (output pixel (2y + dy, 2x + dx))
 *   kind 2, 1x1 head:        W[2][cin]
 * Images: FP32 [batch][2][h][w] (channel 0 = mu, channel 1 = delta, both normalised by the
 * caller), h and w multiples of 8. Workspace: eit_unet_workspace_bytes, device memory owned
 * by the caller; contents on return are scratch. All device pointers must stay valid until
 * the stream has drained. Errors as for the reconstruction calls (EIT_ERR_SHAPE for sizes,
 * EIT_ERR_NOMEM for a short workspace, EIT_ERR_DEVICE for a failed launch). */
typedef struct eit_unet eit_unet;
typedef struct {
    int32_t kind, cin, cout, pad;
    int64_t w_off, b_off;   /* offsets (in floats) of weights and bias in the parameter vector */
} eit_unet_layer;

/* base: channels of the first level, a power of two in [8, 64]. Host-only. */
int eit_unet_create(int32_t base, eit_unet** out);
void eit_unet_destroy(eit_unet* net);
int64_t eit_unet_param_count(const eit_unet* net);
/* Fills up to cap entries of out (may be NULL) and returns the number of layers. */
int eit_unet_layers(const eit_unet* net, eit_unet_layer* out, int32_t cap);
/* 0 for invalid sizes; train != 0 sizes the workspace of eit_unet_train_step. */
size_t eit_unet_workspace_bytes(const eit_unet* net, int32_t batch, int32_t h, int32_t w,
                                int32_t train);
/* y = net(x) for a batch; params is the FP32 parameter vector. Asynchronous on stream. */
int eit_unet_forward(const eit_unet* net, const float* params, const float* x, float* y,
                     int32_t batch, int32_t h, int32_t w, void* ws, size_t ws_bytes, void* stream);
/* One step on the mean squared error over all batch*2*h*w outputs: writes grad (FP32, the
 * parameter layout, overwritten) and *loss (device double). If step >= 1, also applies Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias correction for that step number) with learning
 * rate lr to params in place, updating adam_m and adam_v; step <= 0 computes the gradient
 * only (adam_m / adam_v may then be NULL). Asynchronous on stream. */
int eit_unet_train_step(const eit_unet* net, float* params, float* adam_m, float* adam_v,
                        float* grad, int32_t step, double lr, const float* x,
                        const float* target, int32_t batch, int32_t h, int32_t w, double* loss,
                        void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EITOMO_H */
