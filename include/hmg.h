/*
 * hmg.h -- C-ABI of libhmg, an MI355X (gfx950) implementation of the
 * multigrid-preconditioned Bi-CGSTAB solver for the 2-D Helmholtz equation
 * of I. Livshits, "Shifted Laplacian based multigrid preconditioners for
 * solving indefinite Helmholtz equations" (arXiv:1312.2880).
 *
 * Problem (Section 1, eq:diff and the Sommerfeld condition after it):
 *     Lap u + k(x)^2 u = f  on [0,1]^2,   du/dn - i k u = 0 on the boundary,
 * discretised by the second-order 5-point stencil (eq:disc) with the
 * boundary condition closed by central-difference ghost points.
 *
 * Grid and array conventions used by every call:
 *   - n interior nodes per side; h = 1/(n+1) on the unit square (any h > 0 is
 *     accepted: the domain is then [0, (n+1) h]^2).  Coarse levels halve the
 *     interval count n + 1 until n <= coarsest_n, so n + 1 must stay even
 *     down to there: n = 2^m - 1 (down to 7 by default), or e.g. n = 79
 *     (h = 1/80: levels 79, 39, 19, 9, 4);
 *   - every node (i,j), 0 <= i,j <= n+1, is an unknown, node (i,j) sits at
 *     (i h, j h);
 *   - arrays are row-major with x fastest: element (i,j) at j*(n+2) + i,
 *     (n+2)^2 elements per field;
 *   - wavenumber k: real double per node (k, not k^2), finite and > 0;
 *   - complex fields: hmg_c64 (two doubles, re then im; the layout of C99
 *     double _Complex and of torch.complex128).
 *
 * Ownership: the caller owns every pointer it passes.  Host inputs are copied
 * before the call returns; host outputs are written only on HMG_OK (and on
 * HMG_ERR_NOT_CONVERGED / HMG_ERR_BREAKDOWN for solution arrays, which then
 * hold the last iterate).  Functions with the suffix _dev take device
 * pointers and a hipStream_t (passed as void*, NULL = the grid's own stream);
 * they enqueue work on that stream and may return before it completes unless
 * stated otherwise.  Handles are opaque and released by their destroy call.
 *
 * Errors: every call returns an hmg_status and never throws.  A thread-local
 * message for the last failure is available from hmg_last_error().
 *
 * Threading: hmg_submit / hmg_poll / hmg_cancel are thread-safe; all other
 * calls on one handle must be serialised by the caller.
 */
#ifndef HMG_H
#define HMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } hmg_c64;

typedef enum {
    HMG_OK = 0,
    HMG_ERR_INVALID = 1,        /* bad argument; nothing was done               */
    HMG_ERR_NOMEM = 2,          /* device or host allocation failed             */
    HMG_ERR_DEVICE = 3,         /* a HIP call failed                            */
    HMG_ERR_NOT_CONVERGED = 4,  /* maxit reached; x holds the last iterate      */
    HMG_ERR_BREAKDOWN = 5,      /* a residual norm of the iteration was not
                                   finite (NaN or Inf); x holds the iterate of
                                   that step.  (A Bi-CGSTAB breakdown rho ~ 0
                                   restarts the iteration from the current
                                   residual instead, counted in
                                   hmg_solve_info.restarts.)                    */
    HMG_PENDING = 6,            /* request not finished yet                     */
    HMG_ERR_TOO_LARGE = 7,      /* request footprint above the context budget   */
    HMG_ERR_UNKNOWN_TICKET = 8,
    HMG_ERR_CANCELLED = 9
} hmg_status;

/* Section 5: the three V-cycle variants.  SL-V uses M = L + i beta k^2 for
 * relaxation and residuals; HLM-V uses L for both; HYB-V uses L for residuals
 * everywhere and M for relaxation on the levels near kH = 0.625 and 1.25. */
typedef enum { HMG_SL = 0, HMG_HLM = 1, HMG_HYB = 2 } hmg_variant;

/* FP64: the whole path in double.  MIXED: the V-cycle (preconditioner) in
 * complex float, the outer Bi-CGSTAB, inner products, the true residual and
 * the coarsest-grid solve in double. */
typedef enum { HMG_FP64 = 0, HMG_MIXED = 1 } hmg_precision;

typedef enum { HMG_SM_GS = 0, HMG_SM_KACZ = 1, HMG_SM_LU = 2 } hmg_smoother;

/* Order of the relaxation sweeps.  COLOUR: red-black Gauss-Seidel and
 * 5-colour Kaczmarz (parallel orders).  LEX: lexicographic order, x fastest,
 * the order Section 4 analyses; each sweep equals the sequential sweep up to
 * rounding and runs on the device as a wavefront. */
typedef enum { HMG_ORDER_COLOUR = 0, HMG_ORDER_LEX = 1 } hmg_order;

typedef struct {
    int    variant;          /* hmg_variant, default HMG_HYB                      */
    int    precision;        /* hmg_precision, default HMG_FP64                   */
    double beta;             /* shift of eq:mh, default 0.5                       */
    int    nu_pre, nu_post;  /* Gauss-Seidel sweeps, default 1 + 1               */
    int    kacz_pre, kacz_post; /* Kaczmarz sweeps, default 4 + 4                 */
    int    kacz_band;        /* 1: Kaczmarz on the kH ~ 1.25 levels (default)     */
    int    coarsest_n;       /* in [1, 31]: coarsening stops at the first level
                                with n <= coarsest_n (dense LU), default 7    */
    int    use_graph;        /* 1: replay each Bi-CGSTAB iteration as a hipGraph  */
    int    one_pass_kernels; /* 1: one kernel launch per colour pass / transfer
                                (reference schedule); 0: fused LDS-tiled kernels
                                and the bottom levels as one cycle (default) */
    int    autotune;         /* 1: time the Kaczmarz tile configurations on the
                                level's shape at grid creation (cached per
                                process); 0: fixed default.  The choice
                                changes only the speed: every tile
                                configuration gives the same bits            */
    int    bottom_dense;     /* 1: the cycle on the bottom levels (n <= 31) is a
                                fixed linear map of its right-hand side; form
                                its matrix (complex FP64, m^2 entries for
                                m = (n+2)^2 nodes) at grid creation and apply
                                it as a matrix-vector product (default);
                                0: run the bottom levels in one workgroup     */
    int    relax_order;      /* hmg_order, default HMG_ORDER_COLOUR; HMG_ORDER_LEX
                                runs every level with the one-pass schedule   */
    int    breakdown_at;     /* K > 0: the Bi-CGSTAB breakdown restart (rhat =
                                p = r, scalars reset) is taken after iteration
                                K whatever rho is, to exercise the restart
                                path (Section 6 names no breakdown rule; the
                                library restarts when |rho| <= 1e-14 ||rhat||
                                ||r||); 0: off (default)                       */
    int    true_res_every;   /* K > 0: after every K-th full iteration that
                                misses rtol the residual is recomputed in
                                FP64 as b - L x and the iteration restarts
                                from it (rhat = p = r), or ends when it meets
                                rtol; 0: only when the recursive residual
                                meets rtol (default)                           */
    int    nan_at;           /* K > 0: the residual norm at the end of
                                iteration K is taken as NaN, to exercise the
                                not-finite exit (HMG_ERR_BREAKDOWN); 0: off    */
    int    fp64_levels;      /* MIXED only: the finest fp64_levels levels keep
                                complex-double fields and k; the first level
                                in complex float then takes its right-hand
                                side and returns its correction in double, so
                                it must be a Gauss-Seidel level or the bottom
                                levels (HMG_ERR_INVALID otherwise, and with
                                the one-pass or lexicographic schedules);
                                values beyond the levels above the bottom
                                levels are clamped.  0: every level in float
                                (default)                                      */
    int    ray_n;            /* Section 6.1 ray correction after every V-cycle of
                                a solve: 0 off (default); else the ray grid's
                                interior nodes per side, with (n + 1) a
                                multiple of ray_n + 1, at least 8 fine
                                intervals per ray cell and ray_n <= 7 (the
                                8 (ray_n + 2)^2 <= 648 ray unknowns are
                                solved densely; the Galerkin matrix is
                                factored on the host at grid creation).  The preconditioner becomes
                                z = B_V r; z += P (P^H L P)^{-1} P^H (r - L z),
                                P the 8 plane waves exp(i kr (cos(j pi/4) x +
                                sin(j pi/4) y)), j = 1..8, times the bilinear
                                hats of the ray grid, kr the mean of k          */
    int    hyb_mid;          /* HYB-V only: 1 = M for relaxation on the
                                intermediate scales up to kH ~ 2.5 as well
                                (levels whose kH span meets
                                [0.625/sqrt2, 2.5 sqrt2)), L on the finer and
                                the coarsest ones: the motivation of the
                                hybrid in Section 5 (M's transformation of
                                near-kernel error on intermediate scales, L's
                                accuracy on the coarsest); 0 = the variant's
                                definition, M only for 0.625 <~ kH <~ 1.25
                                (default)                                     */
} hmg_opts;

#define HMG_MAX_LEVELS 24

/* The level plan chosen at grid creation (Section 5 level rules). */
typedef struct {
    int    nlev;
    int    n[HMG_MAX_LEVELS];
    double H[HMG_MAX_LEVELS];
    double kHmin[HMG_MAX_LEVELS], kHmax[HMG_MAX_LEVELS];
    int    smoother[HMG_MAX_LEVELS];      /* hmg_smoother                     */
    double sigma_relax[HMG_MAX_LEVELS];   /* role (A): relaxation operator    */
    double sigma_resid[HMG_MAX_LEVELS];   /* role (B): residual operator      */
    int    pre[HMG_MAX_LEVELS], post[HMG_MAX_LEVELS];
} hmg_plan;

typedef struct {
    double iters;            /* Bi-CGSTAB iterations, counted in halves (Section 6) */
    int    halfsteps;
    double rel_res_true;     /* ||b - L x|| / ||b|| recomputed in FP64 at exit  */
    int    status;           /* hmg_status of this solve                       */
    int    levels;
    int    restarts;         /* breakdown / true-residual restarts             */
    double seconds;          /* wall time of the solve                         */
    int    flags;            /* HMG_INFO_* bits                                */
} hmg_solve_info;

/* hmg_solve_info.flags: the largest k h of the finest grid exceeds 2 pi / 10,
 * i.e. fewer than ten nodes per wavelength somewhere (the resolution the
 * problem statement of Section 1 asks for); the solve is run regardless. */
#define HMG_INFO_KH_ABOVE_GUIDE 1
/* hmg_solve_info.flags: this right-hand side ran with every other right-hand
 * side of its grid in one launch per kernel (a grid with nrhs >= 2 on the
 * default fused schedule); otherwise the right-hand sides ran one after
 * another. */
#define HMG_INFO_BATCHED 2

typedef struct hmg_ctx  hmg_ctx;
typedef struct hmg_grid hmg_grid;

/* ---- context ------------------------------------------------------------ */

/* Fill *o with the defaults above (the paper's constants, Section 5). */
void        hmg_opts_default(hmg_opts *o);
/* Open device `device` (HIP ordinal).  hbm_budget_bytes bounds the device
 * memory admitted by the request server (0 = 90% of free memory). */
hmg_status  hmg_ctx_create(int device, size_t hbm_budget_bytes, hmg_ctx **out);
void        hmg_ctx_destroy(hmg_ctx *ctx);
const char *hmg_last_error(void);

/* ---- grid ----------------------------------------------------------------- */

/* Build the hierarchy for one problem (Section 1 problem statement; Section 5
 * V-cycle components): n >= opts->coarsest_n with n + 1 even on every level
 * above the coarsest (see the grid conventions), h > 0, k per node
 * ((n+2)^2 doubles), f: nrhs right-hand sides of (n+2)^2 complex each (NULL:
 * all zero), nrhs >= 1.  Coarse grids halve the interval count until n <=
 * coarsest_n, take k by injection and rediscretise the 5-point operator; the
 * coarsest operator is factored by dense LU in FP64 on the host.  opts NULL
 * means the defaults.  All inputs are copied. */
hmg_status hmg_grid_create(hmg_ctx *ctx, int n, double h, const double *k,
                           const hmg_c64 *f, int nrhs, const hmg_opts *opts,
                           hmg_grid **out);
void       hmg_grid_destroy(hmg_grid *g);
hmg_status hmg_grid_plan(const hmg_grid *g, hmg_plan *plan);
/* Replace right-hand side `rhs` (host array of (n+2)^2). */
hmg_status hmg_grid_set_rhs(hmg_grid *g, int rhs, const hmg_c64 *f);
/* Device bytes held by the grid. */
size_t     hmg_grid_footprint(const hmg_grid *g);

/* ---- preconditioner: one V-cycle (Section 5) -------------------------------
 * z = B_V r: one V-cycle from a zero initial guess on every level (pre-
 * relaxation, residual, full weighting, recursion, bilinear correction,
 * post-relaxation; dense solve on the coarsest level).  r and z are complex
 * FP64 fields of (n+2)^2; in MIXED precision the cycle runs in complex float
 * between the FP64 input and output. */
hmg_status hmg_vcycle(hmg_grid *g, const hmg_c64 *r, hmg_c64 *z);
hmg_status hmg_vcycle_dev(hmg_grid *g, const void *d_r, void *d_z, void *stream);

/* ---- solve: right-preconditioned Bi-CGSTAB (Section 6) ---------------------
 * Solves L^h x = f for every right-hand side of the grid.  x0: nrhs initial
 * guesses of (n+2)^2 (host, read before any device work), or NULL for the
 * zero initial guess of Section 6.  x: nrhs fields of (n+2)^2, the
 * solutions on exit (x may equal x0).  Stops when ||r|| / ||f|| <= rtol
 * (checked at every half iteration and confirmed with the recomputed FP64
 * residual) or after maxit iterations.  info: nrhs entries (may be NULL).
 * Returns the worst status over the right-hand sides. */
hmg_status hmg_solve(hmg_grid *g, const hmg_c64 *x0, hmg_c64 *x, double rtol, int maxit,
                     hmg_solve_info *info);
/* Device variant for right-hand side `rhs`: d_b (input, may be NULL = the
 * grid's stored f) and d_x (in: initial guess if x0_given, out: solution) are
 * caller-owned complex FP64 device fields.  Synchronises the stream before
 * returning (the iteration count is data dependent). */
hmg_status hmg_solve_dev(hmg_grid *g, int rhs, const void *d_b, void *d_x,
                         int x0_given, double rtol, int maxit,
                         hmg_solve_info *info, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of hmg_solve_dev (same arguments, results and stream behaviour) without
 * any device allocation.  Its reduction partials and residual history live
 * in a fixed device array of HMG_STATIC_SCRATCH_BYTES per GPU, held from the
 * first hmg_ctx_create on that GPU until the process ends; the iteration is
 * enqueued kernel by kernel (no graph is instantiated).  A grid and maxit
 * whose partials (3 doubles per reduction block, at most about 17,000
 * blocks at n = 4095) and history (2 maxit + 2 doubles) exceed the array
 * are rejected with HMG_ERR_TOO_LARGE before any work.  Every call on one
 * GPU shares the array and overwrites it: calls that overlap on one GPU (on
 * different streams or threads) race, so the caller serialises them.
 * hmg_solve_history keeps no record of these solves (it returns 0). */
#define HMG_STATIC_SCRATCH_BYTES (4 << 20)
hmg_status hmg_solve_dev_static(hmg_grid *g, int rhs, const void *d_b, void *d_x,
                                int x0_given, double rtol, int maxit,
                                hmg_solve_info *info, void *stream);

/* The preconditioner as a stationary solver (Section 6.1, the form of its
 * ray-correction table: no Krylov outer iteration):
 *     x <- x + B (f - L x),   B the V-cycle (followed by the ray correction
 *                             when opts.ray_n > 0),
 * for every right-hand side from x0 (host, NULL = 0) until ||f - L x|| <=
 * rtol ||f|| or maxit cycles.  x: nrhs fields (may equal x0); info: nrhs
 * entries, iters = the number of cycles.  HMG_ERR_NOT_CONVERGED when maxit
 * is reached or the residual stops being finite (x holds the last iterate). */
hmg_status hmg_solve_cycles(hmg_grid *g, const hmg_c64 *x0, hmg_c64 *x, double rtol, int maxit,
                            hmg_solve_info *info);

/* Relative residuals ||r|| / ||b|| of the last solve of right-hand side
 * `rhs`, one per half iteration (entry 0 = the initial residual): copies up
 * to cap values into out and returns how many the solve produced (-1 on
 * error). */
int        hmg_solve_history(hmg_grid *g, int rhs, double *out, int cap);

/* ---- batching: many grids and right-hand sides in one launch plan ----------
 * Solves every right-hand side of every grid (zero initial guess); x[q] holds
 * grids[q]'s nrhs solutions, info[q] its nrhs infos (NULL allowed). */
hmg_status hmg_solve_batch(hmg_ctx *ctx, int count, hmg_grid *const *grids,
                           hmg_c64 *const *x, double rtol, int maxit,
                           hmg_solve_info *const *info);

/* ---- serving: continuous batching of solve requests -------------------------
 * A request is copied at submit; the server admits queued requests in arrival
 * order while the sum of admitted device footprints stays within the context
 * budget, advances every admitted solve one Bi-CGSTAB iteration per step
 * (work of different requests overlaps on the device), and retires finished
 * ones.  A retired request's grid stays allocated, idle, for the next
 * request of the same n and options, which is loaded into it in place (no
 * device allocation); idle grids of other sizes are freed, oldest first,
 * only when a request would not fit the budget otherwise.  The server polls
 * its requests' events without blocking, so a finished request is retired
 * while slower ones run on.  poll returns HMG_PENDING until the request is finished, then its
 * final status and (if x_out != NULL) copies the solution; the ticket is
 * released by the first non-pending poll. */
typedef struct {
    int            n;
    double         h;
    const double  *k;
    const hmg_c64 *f;
    hmg_opts       opts;
    double         rtol;
    int            maxit;
} hmg_request;

typedef struct {
    int    status;
    double iters;
    double rel_res_true;
    double t_arrive, t_admit, t_done;   /* seconds on the context's clock     */
    size_t footprint_bytes;
    int    reused;     /* 1: served on the kept grid of an earlier request    */
} hmg_result;

hmg_status hmg_submit(hmg_ctx *ctx, const hmg_request *req, uint64_t *ticket);
hmg_status hmg_poll(hmg_ctx *ctx, uint64_t ticket, hmg_c64 *x_out, hmg_result *res);
hmg_status hmg_cancel(hmg_ctx *ctx, uint64_t ticket);
/* Limit the number of requests in flight at once (0 = limited by the budget
 * only; 1 = serve one request at a time, the serial baseline). */
hmg_status hmg_ctx_set_max_active(hmg_ctx *ctx, int max_active);
/* Seconds since the context was created (the clock of hmg_result). */
double     hmg_ctx_clock(const hmg_ctx *ctx);

/* The ray correction of Section 6.1 on caller-owned FP64 finest-level
 * device fields: z += P (P^H L P)^{-1} P^H (r - L z) (see hmg_opts.ray_n;
 * HMG_ERR_INVALID when the grid has none).  Uses the grid's first right-
 * hand side's scratch, so it must not overlap a solve on the same grid. */
hmg_status hmg_ray_correct_dev(hmg_grid *g, const void *d_r, void *d_z, void *stream);

/* ---- single kernels on one level (parity tests) ----------------------------
 * Each call enqueues one building block of the V-cycle on level `level` of the
 * grid's hierarchy, on caller-owned device fields of (n_l+2)^2 elements in
 * the grid's V-cycle precision (complex double for FP64, complex float for
 * MIXED).  sigma selects L (0) or M (beta).
 *   apply:    out = A_sigma u                       (Section 1 operator)
 *   smooth:   `sweeps` sweeps of red-black Gauss-Seidel (HMG_SM_GS) or
 *             5-colour Kaczmarz (HMG_SM_KACZ) on A_sigma u = f, in place on u;
 *             zero_guess = 1 treats the incoming u as zero (u need not be
 *             initialised)                          (Sections 4 and 5)
 *   restrict: fc = R (f - A_sigma u), full weighting to level+1 (Section 5)
 *   prolong:  u += P ec, bilinear from level+1 to level (Section 5)
 *   coarsest: u = A_c^{-1} f on the last level (dense, FP64)              */
hmg_status hmg_op_apply_dev(hmg_grid *g, int level, double sigma, const void *d_u,
                            void *d_out, void *stream);
hmg_status hmg_op_smooth_dev(hmg_grid *g, int level, int smoother, double sigma,
                             int sweeps, int zero_guess, const void *d_f, void *d_u,
                             void *stream);
/* The same sweeps in lexicographic order (hmg_order LEX; Section 4): Gauss-
 * Seidel (HMG_SM_GS) or Kaczmarz (HMG_SM_KACZ), same arguments and
 * conventions as hmg_op_smooth_dev.  A sweep is a wavefront over tiles of the
 * skewed plane c = i + j, one launch per tile diagonal. */
hmg_status hmg_op_smooth_lex_dev(hmg_grid *g, int level, int smoother, double sigma,
                                 int sweeps, int zero_guess, const void *d_f, void *d_u,
                                 void *stream);
hmg_status hmg_op_restrict_dev(hmg_grid *g, int level, double sigma, const void *d_f,
                               const void *d_u, void *d_fc, void *stream);
hmg_status hmg_op_prolong_dev(hmg_grid *g, int level, const void *d_ec, void *d_u,
                              void *stream);
hmg_status hmg_op_coarsest_dev(hmg_grid *g, const void *d_f, void *d_u, void *stream);

/* Fused kernels of the default schedule (Section 5), same conventions:
 *   gs_down:     u0 = one red-black sweep on A_{sigma_relax} u = f from u = 0,
 *                fc = R (f - A_{sigma_resid} u0)        (pre-smoothing + restriction);
 *                u0 is written to d_u only when d_u != NULL
 *   gs_up:       uo = one red-black sweep on A_{sigma_relax} starting from
 *                u0 + P ec, with u0 read from d_u0 (the field gs_down wrote)
 *                or, when d_u0 == NULL, recomputed from f
 *                                                        (correction + post-smoothing)
 *   kacz_tiled:  uo = S 5-colour Kaczmarz sweeps starting from ui (NULL: zero)
 *                plus P ec (NULL: none); S and the tile side are those of tile
 *                configuration `config` (hmg_kacz_tile_config).
 * Outputs must not alias inputs (tiles read their neighbours' inputs). */
hmg_status hmg_op_gs_down_dev(hmg_grid *g, int level, double sigma_relax, double sigma_resid,
                              const void *d_f, void *d_u, void *d_fc, void *stream);
hmg_status hmg_op_gs_up_dev(hmg_grid *g, int level, double sigma_relax, const void *d_f,
                            const void *d_u0, const void *d_ec, void *d_uo, void *stream);
hmg_status hmg_op_kacz_tiled_dev(hmg_grid *g, int level, double sigma, int config, const void *d_f,
                                 const void *d_ui, const void *d_ec, void *d_uo, void *stream);
/* The up kernel that ends each V-cycle of an FP64 solve on the finest level,
 * with the Bi-CGSTAB product that follows the preconditioner (Section 6:
 * v = A p^ and t = A s^ with A the operator L, sigma = 0): uo as
 * hmg_op_gs_up_dev with d_u0 = NULL, then d_mv = L uo and, in d_sums
 * (device, 3 doubles),
 *   kind 1: Re, Im of sum_p conj(dot_p) mv_p, then 0
 *   kind 2: Re, Im of sum_p conj(mv_p) dot_p, then sum_p |mv_p|^2.
 * d_sums may be NULL: the sums are then left unformed (the kernel alone).
 * d_uo may be NULL: uo is then not stored (as in the solve, which keeps its
 * x update in the preconditioner's input space).
 * FP64 grids only (HMG_ERR_INVALID otherwise).  Uses the grid's reduction
 * scratch, so it must not overlap a solve on the same grid.  Outputs must
 * not alias inputs or each other. */
hmg_status hmg_op_gs_up_product_dev(hmg_grid *g, int level, double sigma_relax, int kind, const void *d_f,
                                    const void *d_ec, void *d_uo, void *d_mv, const void *d_dot,
                                    void *d_sums, void *stream);
/* Kaczmarz pre-smoothing with the restriction (Section 5): uo = S 5-colour
 * Kaczmarz sweeps on A_{sigma_relax} from ui (NULL: zero), then
 * fc = R (f - A_{sigma_resid} uo) on level + 1.  The configuration must be
 * one whose region is staged in LDS (tile side and sweeps as listed by
 * hmg_kacz_tile_config; the kernel works on tiles four nodes smaller with a
 * halo two nodes wider).  Outputs must not alias inputs or each other. */
hmg_status hmg_op_kacz_down_dev(hmg_grid *g, int level, double sigma_relax, double sigma_resid, int config,
                                const void *d_f, const void *d_ui, void *d_uo, void *d_fc, void *stream);
/* A whole Kaczmarz level with n <= 63 in one workgroup (Sections 4-5):
 * uo = `sweeps` 5-colour Kaczmarz sweeps on A_{sigma_relax} starting from
 * ui (NULL: zero) plus P ec (NULL: none); then, when d_fc != NULL,
 * fc = R (f - A_{sigma_resid} uo) on level + 1.  Outputs must not alias
 * inputs or each other. */
hmg_status hmg_op_kacz_level_dev(hmg_grid *g, int level, double sigma_relax, double sigma_resid, int sweeps,
                                 const void *d_f, const void *d_ui, const void *d_ec, void *d_uo, void *d_fc,
                                 void *stream);
/* Tile configuration chosen for a Kaczmarz level of the grid: an index of
 * hmg_kacz_tile_config, the number of configurations when the tuner chose
 * the whole-level kernel (hmg_op_kacz_level_dev), or -1 when the level is
 * not a Kaczmarz level of the fused schedule. */
int        hmg_grid_kacz_config(const hmg_grid *g, int level);
/* Tile width, sweeps per launch and workgroup size of Kaczmarz tile
 * configuration `config` (NULL outputs are skipped); returns the number of
 * configurations, or -1 for an unknown one. */
int        hmg_kacz_tile_config(int config, int *tile, int *sweeps, int *threads);
/* Tile height of configuration `config` (equal to its width except for the
 * rectangular ones), or -1 for an unknown one. */
int        hmg_kacz_tile_height(int config);

#ifdef __cplusplus
}
#endif
#endif /* HMG_H */
