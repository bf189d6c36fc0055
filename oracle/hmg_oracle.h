/*
 * hmg_oracle.h -- FP64 CPU oracle for the shifted-Laplacian / hybrid multigrid
 * preconditioned Bi-CGSTAB Helmholtz solver (Livshits, "Shifted Laplacian based
 * multigrid preconditioners for solving indefinite Helmholtz equations",
 * arXiv:1312.2880).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * Conventions (all functions):
 *   - grid with n interior nodes per side, nodes (i,j), 0 <= i,j <= N = n+1,
 *     node (i,j) at (i*h, j*h); every node is an unknown (Sommerfeld rows are
 *     Robin rows, not Dirichlet);
 *   - arrays are row-major with x fastest: p = j*(n+2) + i, length (n+2)^2;
 *   - complex arrays are C99 double complex (two doubles, re then im);
 *   - k is the (real, positive) wavenumber per node, not k^2;
 *   - sigma selects the operator: 0 gives L (Helmholtz), beta gives M = L + i beta k^2.
 */
#ifndef HMG_ORACLE_H
#define HMG_ORACLE_H

#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef double complex orc_cplx;

/* ---- single-level operations (Section 1 eq:diff, eq:disc, eq:mh) ---- */
void orc_apply(int n, double h, const double *k, double sigma,
               const orc_cplx *u, orc_cplx *out);
void orc_residual(int n, double h, const double *k, double sigma,
                  const orc_cplx *f, const orc_cplx *u, orc_cplx *r);
void orc_dense(int n, double h, const double *k, double sigma, orc_cplx *A);

/* ---- relaxation (Section 4; Section 5 smoothing list) ---- */
void orc_gs_lex(int n, double h, const double *k, double sigma,
                const orc_cplx *f, orc_cplx *u);
void orc_gs_rb(int n, double h, const double *k, double sigma,
               const orc_cplx *f, orc_cplx *u);
void orc_kacz_lex(int n, double h, const double *k, double sigma,
                  const orc_cplx *f, orc_cplx *u);
void orc_kacz_5c(int n, double h, const double *k, double sigma,
                 const orc_cplx *f, orc_cplx *u);

/* ---- transfers (Section 5: bilinear interpolation, full weighting) ---- */
void orc_restrict_fw(int n, const orc_cplx *r, orc_cplx *fc);   /* n -> (n-1)/2 */
void orc_prolong_add(int nc, const orc_cplx *ec, orc_cplx *u);  /* nc -> 2nc+1  */
void orc_inject_k(int n, const double *k, double *kc);

/* ---- dense LU with partial pivoting (coarsest grid) ---- */
int  orc_lu_factor(int m, orc_cplx *A, int *piv);
void orc_lu_solve(int m, const orc_cplx *LU, const int *piv, orc_cplx *b);

/* ---- multigrid hierarchy, level plan, V-cycle (Section 5) ---- */
enum { ORC_SL = 0, ORC_HLM = 1, ORC_HYB = 2 };
enum { ORC_SM_GS = 0, ORC_SM_KACZ = 1, ORC_SM_LU = 2 };
enum { ORC_ORDER_COLOUR = 0, ORC_ORDER_LEX = 1 };

typedef struct {
    int    variant;      /* ORC_SL / ORC_HLM / ORC_HYB                      */
    double beta;         /* shift, 0.5 in the paper                        */
    int    nu_pre, nu_post;      /* GS sweeps, 1 + 1                       */
    int    kacz_pre, kacz_post;  /* normal-equation sweeps, 4 + 4          */
    int    kacz_band;    /* 1: Kaczmarz on kH ~ 1.25 levels; 0: GS there    */
    int    coarsest_n;   /* interior size of the LU level (7)              */
    int    gs_order;     /* ORC_ORDER_COLOUR (red-black) or ORC_ORDER_LEX  */
    int    kacz_order;   /* ORC_ORDER_COLOUR (5 colours) or ORC_ORDER_LEX  */
    int    hyb_mid;      /* HYB only: 1 = M for relaxation on the intermediate
                            scales up to kH ~ 2.5 as well (the motivation of
                            the hybrid in Section 5); 0 = the variant's
                            definition, M only for 0.625 <~ kH <~ 1.25      */
} orc_opts;

#define ORC_MAX_LEVELS 24
typedef struct {
    int    nlev;
    int    n[ORC_MAX_LEVELS];
    double H[ORC_MAX_LEVELS];
    double kHmin[ORC_MAX_LEVELS], kHmax[ORC_MAX_LEVELS];
    int    smoother[ORC_MAX_LEVELS];     /* ORC_SM_*                         */
    double sigma_relax[ORC_MAX_LEVELS];  /* role (A): relaxation operator    */
    double sigma_resid[ORC_MAX_LEVELS];  /* role (B): residual operator      */
    int    pre[ORC_MAX_LEVELS], post[ORC_MAX_LEVELS];
} orc_plan;

typedef struct orc_grid orc_grid;

void      orc_opts_default(orc_opts *o);
orc_grid *orc_grid_create(int n, double h, const double *k, const orc_opts *o);
void      orc_grid_destroy(orc_grid *g);
void      orc_grid_plan(const orc_grid *g, orc_plan *p);
void      orc_vcycle(orc_grid *g, const orc_cplx *f, orc_cplx *u);
int       orc_grid_override_level(orc_grid *g, int l, int smoother, double sigma_relax,
                                  double sigma_resid, int pre, int post);

/* ---- study switches: readings of Section 5 other than the default, for
 * iteration-count studies (the default reading is what every pin fixes).
 * fw_transpose: restriction R = P^T / 4 instead of full weighting with
 * mirror folding at the boundary; coarse_sweeps > 0: the coarsest level runs
 * that many Gauss-Seidel sweeps from zero instead of the dense solve.  The
 * boundary row scale (process-wide; leave it off outside a study) multiplies
 * rows with b boundary faces by 2^-b in every operator of the oracle. ---- */
void      orc_grid_set_study(orc_grid *g, int fw_transpose, int coarse_sweeps);
void      orc_set_boundary_row_scale(int on);

/* ---- precision form (O11): the V-cycle with its fields stored in complex
 * float and its arithmetic in double; mode ORC_MIX_FUSED rounds where the
 * fused kernels store (Kaczmarz iterate every kacz_every sweeps, levels with
 * n <= block_n one double block), ORC_MIX_ONEPASS after every elementary
 * step; round_io rounds the cycle's input and output.  The Bi-CGSTAB of a
 * grid in this mode keeps its own arithmetic and L in double. ---- */
enum { ORC_MIX_OFF = 0, ORC_MIX_FUSED = 1, ORC_MIX_ONEPASS = 2 };
void      orc_grid_set_mixed(orc_grid *g, int mode, int kacz_every, int block_n, int round_io);
/* The same with the finest fp64_levels levels kept in double (fused mode;
 * clamped to the first level of the double block); the first float level
 * then takes and returns double fields. */
void      orc_grid_set_mixed_ex(orc_grid *g, int mode, int kacz_every, int block_n, int round_io,
                                int fp64_levels);

/* ---- ray correction (Section 6.1): a Galerkin correction whose basis is
 * each of the 8 plane waves exp(i k (cos(j pi/4) x + sin(j pi/4) y)) times
 * the bilinear hats of a ray grid with ray_n interior nodes per side; set
 * ray_n = 0 to switch it off.  With it, the grid's preconditioner is the
 * V-cycle followed by the correction of its residual. ---- */
int  orc_grid_set_ray(orc_grid *g, int ray_n);
void orc_ray_correct(orc_grid *g, const orc_cplx *f, orc_cplx *u);   /* u += C_R (f - L u) */
/* stationary iteration x <- x + B (f - L x) (Section 6.1, the solver form of
 * Table 4); returns the number of cycles */
int  orc_cycles(orc_grid *g, const orc_cplx *f, orc_cplx *x, double rtol, int maxit, double *res_hist);

/* ---- Bi-CGSTAB (Section 6) ---- */
enum { ORC_PREC_NONE = 0, ORC_PREC_VCYCLE = 1, ORC_PREC_EXACT = 2 };
enum { ORC_OK = 0, ORC_NOT_CONVERGED = 4, ORC_BREAKDOWN = 5 };
typedef struct {
    int    halfsteps;      /* iterations counted in halves               */
    double rel_res;        /* ||b - A x|| / ||b|| recomputed at exit       */
    int    restarts;
    int    status;
    int    vcycles;        /* preconditioner applications               */
} orc_info;

int orc_bicgstab(orc_grid *g, const orc_cplx *b, orc_cplx *x, double rtol,
                 int maxit, int precond, orc_info *info,
                 double *res_hist, int hist_cap);
/* The same, with force_breakdown_at = K > 0 taking the breakdown branch at
 * the start of iteration K + 1 whatever rho is (tests of the restart path). */
int orc_bicgstab_ex(orc_grid *g, const orc_cplx *b, orc_cplx *x, double rtol,
                    int maxit, int precond, orc_info *info,
                    double *res_hist, int hist_cap, int force_breakdown_at);
/* The same with true_res_every = K > 0 (after every K-th full iteration that
 * misses the tolerance the residual is recomputed as b - A x and the
 * iteration restarts from it, or ends if it meets the tolerance) and nan_at
 * = K > 0 (the residual norm at the end of iteration K is taken as NaN).  A
 * residual norm that is not finite ends the solve with ORC_BREAKDOWN, x
 * holding the last iterate. */
int orc_bicgstab_ex2(orc_grid *g, const orc_cplx *b, orc_cplx *x, double rtol,
                     int maxit, int precond, orc_info *info,
                     double *res_hist, int hist_cap, int force_breakdown_at,
                     int true_res_every, int nan_at);

#ifdef __cplusplus
}
#endif
#endif
