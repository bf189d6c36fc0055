/*
 * hmg_oracle.c -- plain, slow, FP64 reference implementation of the method of
 * Livshits, arXiv:1312.2880.  TEST INFRASTRUCTURE: used only by the tests, the
 * smoke check and the CPU baseline of the benchmark; never by the GPU library.
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off.  OpenMP is used only on
 * loops whose iterations are independent (colour passes, operator apply,
 * transfers, axpy-type updates); every inner product is a sequential loop, so
 * results do not depend on the thread count.
 *
 * Readings of points the paper leaves open are listed with the functions that
 * take them; they are the same readings the design document lists.
 */
#include "hmg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(M, i, j) ((size_t)(j) * (size_t)(M) + (size_t)(i))
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Discrete operator.                                                        */
/*                                                                           */
/* Section 1 (eq:diff with the Sommerfeld condition, eq:disc): the 5-point   */
/* second-order Laplacian plus k^2 on every node (i,j), 0..N.  The paper     */
/* only says "standard discretization"; the reading taken here is the        */
/* ghost-point central difference of du/dn - i k u = 0.  At x = 0 the         */
/* outward normal is -x, so -(u_1 - u_-1)/(2h) - i k u_0 = 0, i.e.           */
/* u_-1 = u_1 + 2 i k h u_0; the same on every side, both at corners.        */
/* Substituting the ghost value gives, for node p with b_p boundary faces:   */
/*   a_pp = (-4 + 2 i k_p h b_p)/h^2 + k_p^2 (1 + i sigma)                  */
/*   a_pq = w_pq / h^2, w_pq = 2 for the inward neighbour across a boundary  */
/*          face of p, 1 for every other in-grid neighbour.                  */
/* eq:mh: M = L + i beta k^2 adds i beta k^2 to every diagonal entry.        */
/* Rows are not rescaled.                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    orc_cplx app;      /* diagonal entry                               */
    double   w[4];     /* neighbour weights / h^2: left, right, down, up */
} orc_row;

/* Study switch (not the default reading): rows with b boundary faces
 * multiplied by 2^-b, which makes the matrix complex symmetric (the doubled
 * inward weight is halved).  The solution of A x = f is that of the scaled
 * system with the scaled right-hand side. */
static int g_row_scale = 0;
void orc_set_boundary_row_scale(int on) { g_row_scale = on ? 1 : 0; }

static orc_row row_of(int N, double h, double kp, double sigma, int i, int j)
{
    orc_row r;
    double  ih2 = 1.0 / (h * h);
    int     b   = (i == 0) + (i == N) + (j == 0) + (j == N);
    r.app = (-4.0 + 2.0 * I * kp * h * (double)b) * ih2 + kp * kp * (1.0 + I * sigma);
    r.w[0] = (i > 0) ? ((i == N) ? 2.0 : 1.0) * ih2 : 0.0;   /* (i-1, j) */
    r.w[1] = (i < N) ? ((i == 0) ? 2.0 : 1.0) * ih2 : 0.0;   /* (i+1, j) */
    r.w[2] = (j > 0) ? ((j == N) ? 2.0 : 1.0) * ih2 : 0.0;   /* (i, j-1) */
    r.w[3] = (j < N) ? ((j == 0) ? 2.0 : 1.0) * ih2 : 0.0;   /* (i, j+1) */
    if (g_row_scale && b) {
        double sc = ldexp(1.0, -b);
        r.app *= sc;
        for (int q = 0; q < 4; ++q) r.w[q] *= sc;
    }
    return r;
}

/* sum over the in-grid neighbours q of p of a_pq u_q */
static orc_cplx offdiag_sum(const orc_row *r, int M, int i, int j, const orc_cplx *u)
{
    orc_cplx s = 0.0;
    if (r->w[0] != 0.0) s += r->w[0] * u[IDX(M, i - 1, j)];
    if (r->w[1] != 0.0) s += r->w[1] * u[IDX(M, i + 1, j)];
    if (r->w[2] != 0.0) s += r->w[2] * u[IDX(M, i, j - 1)];
    if (r->w[3] != 0.0) s += r->w[3] * u[IDX(M, i, j + 1)];
    return s;
}

void orc_apply(int n, double h, const double *k, double sigma,
               const orc_cplx *u, orc_cplx *out)
{
    int M = n + 2, N = n + 1;
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) {
            orc_row r = row_of(N, h, k[IDX(M, i, j)], sigma, i, j);
            out[IDX(M, i, j)] = r.app * u[IDX(M, i, j)] + offdiag_sum(&r, M, i, j, u);
        }
}

void orc_residual(int n, double h, const double *k, double sigma,
                  const orc_cplx *f, const orc_cplx *u, orc_cplx *res)
{
    int M = n + 2, N = n + 1;
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) {
            orc_row r = row_of(N, h, k[IDX(M, i, j)], sigma, i, j);
            res[IDX(M, i, j)] = f[IDX(M, i, j)]
                - (r.app * u[IDX(M, i, j)] + offdiag_sum(&r, M, i, j, u));
        }
}

/* Dense matrix of A_sigma, row-major (M^2 x M^2), assembled column by column
 * by applying the operator to unit vectors. */
void orc_dense(int n, double h, const double *k, double sigma, orc_cplx *A)
{
    int    M = n + 2;
    size_t m = (size_t)M * M;
    orc_cplx *e   = calloc(m, sizeof(orc_cplx));
    orc_cplx *col = malloc(m * sizeof(orc_cplx));
    for (size_t c = 0; c < m; ++c) {
        e[c] = 1.0;
        orc_apply(n, h, k, sigma, e, col);
        for (size_t r = 0; r < m; ++r) A[r * m + c] = col[r];
        e[c] = 0.0;
    }
    free(e);
    free(col);
}

/* ------------------------------------------------------------------------ */
/* Relaxation (Section 4 and the smoothing list of Section 5).               */
/* Gauss-Seidel row update: u_p <- (f_p - sum_{q != p} a_pq u_q) / a_pp.     */
/* Lexicographic order is x fastest (i inner), as analysed in Section 4;     */
/* red-black takes (i+j) even first, then odd.  Relaxation weight 1.         */
/* ------------------------------------------------------------------------ */

static void gs_point(int N, int M, double h, const double *k, double sigma,
                     const orc_cplx *f, orc_cplx *u, int i, int j)
{
    orc_row r = row_of(N, h, k[IDX(M, i, j)], sigma, i, j);
    u[IDX(M, i, j)] = (f[IDX(M, i, j)] - offdiag_sum(&r, M, i, j, u)) / r.app;
}

void orc_gs_lex(int n, double h, const double *k, double sigma,
                const orc_cplx *f, orc_cplx *u)
{
    int M = n + 2, N = n + 1;
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i)
            gs_point(N, M, h, k, sigma, f, u, i, j);
}

void orc_gs_rb(int n, double h, const double *k, double sigma,
               const orc_cplx *f, orc_cplx *u)
{
    int M = n + 2, N = n + 1;
    for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j <= N; ++j)
            for (int i = (colour + j) & 1; i <= N; i += 2)
                gs_point(N, M, h, k, sigma, f, u, i, j);
    }
}

/* Relaxation of the normal equations "in the spirit of Kaczmarz" (Section 4,
 * after the smoothing-rate list).  Reading taken: the row-action method, i.e.
 * Gauss-Seidel on A A^* y = f with u = A^* y.  For row p:
 *   delta = (f_p - (A u)_p) / ||a_p||^2,   u_q <- u_q + conj(a_pq) delta
 * for every q in the stencil of p (p itself included).  ^* is the conjugate
 * transpose, as the paper states for its ^T. */
static void kacz_row(int N, int M, double h, const double *k, double sigma,
                     const orc_cplx *f, orc_cplx *u, int i, int j)
{
    orc_row  r   = row_of(N, h, k[IDX(M, i, j)], sigma, i, j);
    orc_cplx res = f[IDX(M, i, j)] - (r.app * u[IDX(M, i, j)] + offdiag_sum(&r, M, i, j, u));
    double   nrm = creal(r.app) * creal(r.app) + cimag(r.app) * cimag(r.app)
                 + r.w[0] * r.w[0] + r.w[1] * r.w[1] + r.w[2] * r.w[2] + r.w[3] * r.w[3];
    orc_cplx d   = res / nrm;
    u[IDX(M, i, j)] += conj(r.app) * d;
    if (r.w[0] != 0.0) u[IDX(M, i - 1, j)] += r.w[0] * d;
    if (r.w[1] != 0.0) u[IDX(M, i + 1, j)] += r.w[1] * d;
    if (r.w[2] != 0.0) u[IDX(M, i, j - 1)] += r.w[2] * d;
    if (r.w[3] != 0.0) u[IDX(M, i, j + 1)] += r.w[3] * d;
}

void orc_kacz_lex(int n, double h, const double *k, double sigma,
                  const orc_cplx *f, orc_cplx *u)
{
    int M = n + 2, N = n + 1;
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i)
            kacz_row(N, M, h, k, sigma, f, u, i, j);
}

/* Five colours c = (i + 2j) mod 5, taken in order c = 0..4.  Two rows of one
 * colour are at Manhattan distance >= 3, so their 5-point stencils are
 * disjoint and the rows of a colour commute. */
void orc_kacz_5c(int n, double h, const double *k, double sigma,
                 const orc_cplx *f, orc_cplx *u)
{
    int M = n + 2, N = n + 1;
    for (int c = 0; c < 5; ++c) {
#pragma omp parallel for schedule(static)
        for (int j = 0; j <= N; ++j) {
            int i0 = ((c - 2 * j) % 5 + 5) % 5;
            for (int i = i0; i <= N; i += 5)
                kacz_row(N, M, h, k, sigma, f, u, i, j);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Transfers (Section 5: "bilinear interpolation", "full weighting").         */
/* Vertex-centred nesting: coarse node (I,J) sits on fine node (2I,2J);      */
/* fine nodes 0..N, coarse 0..N/2.                                           */
/* ------------------------------------------------------------------------ */

/* Full weighting, weights (1,2,1) x (1,2,1) / 16.  At the boundary the fine
 * residual is mirrored, r(-1) = r(1) and r(N+1) = r(N-1) (reading taken; the
 * paper gives no boundary rule), which keeps every row sum equal to one. */
void orc_restrict_fw(int n, const orc_cplx *r, orc_cplx *fc)
{
    int M = n + 2, N = n + 1, Nc = N / 2, Mc = Nc + 1;
#pragma omp parallel for schedule(static)
    for (int jc = 0; jc <= Nc; ++jc)
        for (int ic = 0; ic <= Nc; ++ic) {
            orc_cplx s = 0.0;
            for (int e = -1; e <= 1; ++e)
                for (int d = -1; d <= 1; ++d) {
                    int i = 2 * ic + d, j = 2 * jc + e;
                    if (i < 0) i = -i;
                    if (i > N) i = 2 * N - i;
                    if (j < 0) j = -j;
                    if (j > N) j = 2 * N - j;
                    double wgt = (double)((2 - abs(d)) * (2 - abs(e)));
                    s += wgt * r[IDX(M, i, j)];
                }
            fc[IDX(Mc, ic, jc)] = s / 16.0;
        }
}

/* Bilinear interpolation of the coarse correction, added to u. */
void orc_prolong_add(int nc, const orc_cplx *ec, orc_cplx *u)
{
    int Nc = nc + 1, Mc = nc + 2, N = 2 * Nc, M = N + 1;
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) {
            int ic = i / 2, jc = j / 2;
            orc_cplx e;
            if (!(i & 1) && !(j & 1))
                e = ec[IDX(Mc, ic, jc)];
            else if ((i & 1) && !(j & 1))
                e = 0.5 * (ec[IDX(Mc, ic, jc)] + ec[IDX(Mc, ic + 1, jc)]);
            else if (!(i & 1) && (j & 1))
                e = 0.5 * (ec[IDX(Mc, ic, jc)] + ec[IDX(Mc, ic, jc + 1)]);
            else
                e = 0.25 * (ec[IDX(Mc, ic, jc)] + ec[IDX(Mc, ic + 1, jc)]
                            + ec[IDX(Mc, ic, jc + 1)] + ec[IDX(Mc, ic + 1, jc + 1)]);
            u[IDX(M, i, j)] += e;
        }
}

/* Coarse-grid wavenumber by injection, k_c(I,J) = k(2I,2J). */
void orc_inject_k(int n, const double *k, double *kc)
{
    int M = n + 2, Nc = (n + 1) / 2, Mc = Nc + 1;
    for (int jc = 0; jc <= Nc; ++jc)
        for (int ic = 0; ic <= Nc; ++ic)
            kc[IDX(Mc, ic, jc)] = k[IDX(M, 2 * ic, 2 * jc)];
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (Doolittle, row-major, in place).          */
/* ------------------------------------------------------------------------ */

int orc_lu_factor(int m, orc_cplx *A, int *piv)
{
    for (int c = 0; c < m; ++c) {
        int    p    = c;
        double best = cabs(A[(size_t)c * m + c]);
        for (int r = c + 1; r < m; ++r) {
            double v = cabs(A[(size_t)r * m + c]);
            if (v > best) { best = v; p = r; }
        }
        piv[c] = p;
        if (best == 0.0) return -1;
        if (p != c)
            for (int q = 0; q < m; ++q) {
                orc_cplx t = A[(size_t)c * m + q];
                A[(size_t)c * m + q] = A[(size_t)p * m + q];
                A[(size_t)p * m + q] = t;
            }
        for (int r = c + 1; r < m; ++r) {
            orc_cplx l = A[(size_t)r * m + c] / A[(size_t)c * m + c];
            A[(size_t)r * m + c] = l;
            for (int q = c + 1; q < m; ++q)
                A[(size_t)r * m + q] -= l * A[(size_t)c * m + q];
        }
    }
    return 0;
}

void orc_lu_solve(int m, const orc_cplx *LU, const int *piv, orc_cplx *b)
{
    for (int c = 0; c < m; ++c)
        if (piv[c] != c) { orc_cplx t = b[c]; b[c] = b[piv[c]]; b[piv[c]] = t; }
    for (int r = 0; r < m; ++r) {
        orc_cplx s = b[r];
        for (int q = 0; q < r; ++q) s -= LU[(size_t)r * m + q] * b[q];
        b[r] = s;
    }
    for (int r = m - 1; r >= 0; --r) {
        orc_cplx s = b[r];
        for (int q = r + 1; q < m; ++q) s -= LU[(size_t)r * m + q] * b[q];
        b[r] = s / LU[(size_t)r * m + r];
    }
}

/* ------------------------------------------------------------------------ */
/* Hierarchy and level plan (Section 5).                                     */
/* ------------------------------------------------------------------------ */

struct orc_grid {
    orc_opts opts;
    orc_plan plan;
    int      n;
    double   h;
    double  *k[ORC_MAX_LEVELS];     /* wavenumber per level (injection)   */
    orc_cplx *f[ORC_MAX_LEVELS];    /* right-hand side per level          */
    orc_cplx *u[ORC_MAX_LEVELS];    /* iterate / correction per level     */
    orc_cplx *r[ORC_MAX_LEVELS];    /* residual scratch per level         */
    orc_cplx *lu;                   /* coarsest factor                    */
    int      *piv;
    orc_cplx *exact_lu;             /* dense factor of L^h (exact preconditioner) */
    int      *exact_piv;
    /* precision form (O11): where the preconditioner rounds to float */
    int       mix_mode;             /* ORC_MIX_OFF / ORC_MIX_FUSED / ORC_MIX_ONEPASS */
    int       mix_kacz_every;       /* fused: Kaczmarz sweeps between stores   */
    int       mix_block_n;          /* fused: levels with n <= this form one FP64 block */
    int       mix_round_io;         /* the cycle's input and output are rounded */
    int       mix_t;                /* first level stored in float (finer ones double) */
    double   *kv[ORC_MAX_LEVELS];   /* k used inside the V-cycle (rounded in the precision form) */
    /* ray correction (Section 6.1): 8 plane waves times bilinear ray functions */
    int       ray_n;                /* interior nodes per side of the ray grid (0: off) */
    orc_cplx *ray_P;                /* basis, dense (n+2)^2 x 8 (ray_n+2)^2, row-major   */
    orc_cplx *ray_A;                /* Galerkin matrix P^H L P, LU-factored              */
    int      *ray_piv;
    /* study switches (readings other than the default; see orc_grid_set_study) */
    int       st_fw_transpose;
    int       st_coarse_sweeps;
};

void orc_opts_default(orc_opts *o)
{
    o->variant    = ORC_HYB;
    o->beta       = 0.5;
    o->nu_pre     = 1;
    o->nu_post    = 1;
    o->kacz_pre   = 4;
    o->kacz_post  = 4;
    o->kacz_band  = 1;
    o->coarsest_n = 7;
    o->gs_order   = ORC_ORDER_COLOUR;
    o->kacz_order = ORC_ORDER_COLOUR;
    o->hyb_mid    = 0;
}

/* Level classification.  The paper states its rules for constant k on
 * grids with kH = 0.3125 * 2^j; the reading for a level whose nodes span
 * [kH_min, kH_max] is (first match wins):
 *   1. last level: dense LU; M for SL, L for HLM and HYB (L on the coarsest
 *      scales, end of Section 5);
 *   2. kacz_band and the span meets [1.25/sqrt2, 1.25*sqrt2): four pre- and
 *      four post-sweeps of the normal-equation relaxation, on M (SL, HYB) or
 *      L (HLM);
 *   3. kacz_band and the span meets [1.25*sqrt2, 2.5): the same relaxation
 *      on the variant's operator (M for SL, L for HLM and HYB): Section 4
 *      finds Gauss-Seidel good only for kH up to about 0.625 and from about
 *      2.5 on, and takes the normal equation where it fails (between them
 *      lie 1.25 and the span up to 2.5; Gauss-Seidel on L also loses its
 *      pivot at kH = 2);
 *   4. HYB only, span meets [0.625/sqrt2, 0.625*sqrt2): Gauss-Seidel on M;
 *   5. otherwise Gauss-Seidel, on M for SL and on L for HLM and HYB.
 * The residual operator (role (B)) is M for SL and L for HLM and HYB.
 * With hyb_mid (HYB only) the relaxation operator is M on every level whose
 * span meets [0.625/sqrt2, 2.5*sqrt2) (rules 3 and 4): Section 5 motivates
 * the hybrid by M's transformation of near-kernel error on the intermediate
 * scales and L's accuracy on the coarsest ones, and Section 3 finds M's
 * approximation at kH = 2.5 wrong "in the right way" for a preconditioner,
 * while the variant's definition keeps M to 0.625 <~ kH <~ 1.25. */
static void classify(orc_grid *g, int l, int last)
{
    const orc_opts *o  = &g->opts;
    orc_plan       *pl = &g->plan;
    int    n = pl->n[l], M = n + 2;
    double H = pl->H[l], lo = 1e300, hi = -1e300, beta = o->beta;
    for (int j = 0; j < M; ++j)
        for (int i = 0; i < M; ++i) {
            double kh = g->k[l][IDX(M, i, j)] * H;
            if (kh < lo) lo = kh;
            if (kh > hi) hi = kh;
        }
    pl->kHmin[l] = lo;
    pl->kHmax[l] = hi;
    pl->sigma_resid[l] = (o->variant == ORC_SL) ? beta : 0.0;
    if (last) {
        pl->smoother[l]    = ORC_SM_LU;
        pl->sigma_relax[l] = (o->variant == ORC_SL) ? beta : 0.0;
        pl->pre[l] = pl->post[l] = 0;
        return;
    }
    double s2 = sqrt(2.0);
    int in_kacz = (hi >= 1.25 / s2) && (lo < 1.25 * s2);
    int in_wide = (hi >= 1.25 * s2) && (lo < 2.5);
    int mid     = (o->variant == ORC_HYB) && o->hyb_mid;
    int in_gsm  = (hi >= 0.625 / s2) && (lo < (mid ? 2.5 : 0.625) * s2);
    double sig = (o->variant == ORC_SL) ? beta : 0.0;
    if (o->kacz_band && (in_kacz || in_wide)) {
        pl->smoother[l]    = ORC_SM_KACZ;
        pl->sigma_relax[l] = in_kacz ? ((o->variant == ORC_HLM) ? 0.0 : beta) : (mid ? beta : sig);
        pl->pre[l] = o->kacz_pre;
        pl->post[l] = o->kacz_post;
        return;
    }
    if (o->variant == ORC_HYB && in_gsm) {
        pl->smoother[l]    = ORC_SM_GS;
        pl->sigma_relax[l] = beta;
        pl->pre[l] = o->nu_pre;
        pl->post[l] = o->nu_post;
        return;
    }
    pl->smoother[l]    = ORC_SM_GS;
    pl->sigma_relax[l] = sig;
    pl->pre[l] = o->nu_pre;
    pl->post[l] = o->nu_post;
}

orc_grid *orc_grid_create(int n, double h, const double *k, const orc_opts *o)
{
    orc_grid *g = calloc(1, sizeof(orc_grid));
    g->opts = *o;
    g->n = n;
    g->h = h;
    int l = 0, nl = n;
    double H = h;
    for (;;) {
        size_t m = (size_t)(nl + 2) * (nl + 2);
        g->plan.n[l] = nl;
        g->plan.H[l] = H;
        g->k[l] = malloc(m * sizeof(double));
        g->f[l] = calloc(m, sizeof(orc_cplx));
        g->u[l] = calloc(m, sizeof(orc_cplx));
        g->r[l] = calloc(m, sizeof(orc_cplx));
        if (l == 0) memcpy(g->k[0], k, m * sizeof(double));
        else        orc_inject_k(g->plan.n[l - 1], g->k[l - 1], g->k[l]);
        g->kv[l] = g->k[l];
        if (nl <= o->coarsest_n || nl < 3 || l == ORC_MAX_LEVELS - 1) break;
        nl = (nl - 1) / 2;
        H *= 2.0;
        ++l;
    }
    g->plan.nlev = l + 1;
    for (int q = 0; q <= l; ++q) classify(g, q, q == l);
    /* coarsest factor */
    int    nc = g->plan.n[l];
    size_t m  = (size_t)(nc + 2) * (nc + 2);
    g->lu  = malloc(m * m * sizeof(orc_cplx));
    g->piv = malloc(m * sizeof(int));
    orc_dense(nc, g->plan.H[l], g->k[l], g->plan.sigma_relax[l], g->lu);
    orc_lu_factor((int)m, g->lu, g->piv);
    return g;
}

void orc_grid_destroy(orc_grid *g)
{
    if (!g) return;
    for (int l = 0; l < g->plan.nlev; ++l) {
        if (g->kv[l] != g->k[l]) free(g->kv[l]);
        free(g->k[l]); free(g->f[l]); free(g->u[l]); free(g->r[l]);
    }
    free(g->lu); free(g->piv); free(g->exact_lu); free(g->exact_piv);
    free(g->ray_P); free(g->ray_A); free(g->ray_piv);
    free(g);
}

void orc_grid_plan(const orc_grid *g, orc_plan *p) { *p = g->plan; }

void orc_grid_set_study(orc_grid *g, int fw_transpose, int coarse_sweeps)
{
    g->st_fw_transpose  = fw_transpose ? 1 : 0;
    g->st_coarse_sweeps = coarse_sweeps > 0 ? coarse_sweeps : 0;
}

/* Replace the classification of one non-coarsest level (tests and studies of
 * other plans); the coarsest factor is rebuilt when its shift changes. */
int orc_grid_override_level(orc_grid *g, int l, int smoother, double sigma_relax,
                            double sigma_resid, int pre, int post)
{
    orc_plan *pl = &g->plan;
    if (l < 0 || l >= pl->nlev) return -1;
    int last = (l == pl->nlev - 1);
    if (last != (smoother == ORC_SM_LU)) return -1;
    pl->smoother[l] = smoother;
    pl->sigma_relax[l] = sigma_relax;
    pl->sigma_resid[l] = sigma_resid;
    pl->pre[l] = pre;
    pl->post[l] = post;
    if (last) {
        int    nc = pl->n[l];
        size_t m  = (size_t)(nc + 2) * (nc + 2);
        orc_dense(nc, pl->H[l], g->k[l], sigma_relax, g->lu);
        return orc_lu_factor((int)m, g->lu, g->piv);
    }
    return 0;
}

static void relax(orc_grid *g, int l, const orc_cplx *f, orc_cplx *u, int sweeps)
{
    const orc_plan *pl = &g->plan;
    int    n = pl->n[l];
    double H = pl->H[l], s = pl->sigma_relax[l];
    for (int it = 0; it < sweeps; ++it) {
        if (pl->smoother[l] == ORC_SM_GS) {
            if (g->opts.gs_order == ORC_ORDER_LEX) orc_gs_lex(n, H, g->kv[l], s, f, u);
            else                                   orc_gs_rb(n, H, g->kv[l], s, f, u);
        } else {
            if (g->opts.kacz_order == ORC_ORDER_LEX) orc_kacz_lex(n, H, g->kv[l], s, f, u);
            else                                     orc_kacz_5c(n, H, g->kv[l], s, f, u);
        }
    }
}

/* V-cycle with zero initial guess on each level:
 *   u = 0; relax (role A); r = f - B u (role B); f_c = R r;
 *   e_c = V(l+1, f_c); u += P e_c; relax (role A). */
/* Study reading of the restriction: R = P^T / 4, the transpose of the
 * bilinear interpolation (weights 4, 2, 1 over 16 around the coarse node),
 * with the weights of fine nodes outside the grid dropped rather than
 * folded back (row sums below one at the boundary). */
static void restrict_transpose(int n, const orc_cplx *r, orc_cplx *fc)
{
    int N = n + 1, M = n + 2, Nc = N / 2, Mc = Nc + 1;
    for (int cj = 0; cj <= Nc; ++cj)
        for (int ci = 0; ci <= Nc; ++ci) {
            orc_cplx s = 0.0;
            for (int e = -1; e <= 1; ++e)
                for (int d = -1; d <= 1; ++d) {
                    int i = 2 * ci + d, j = 2 * cj + e;
                    if (i < 0 || j < 0 || i > N || j > N) continue;
                    s += (double)((2 - abs(d)) * (2 - abs(e))) * r[IDX(M, i, j)];
                }
            fc[IDX(Mc, ci, cj)] = s / 16.0;
        }
}

static void vcycle_level(orc_grid *g, int l, const orc_cplx *f, orc_cplx *u)
{
    const orc_plan *pl = &g->plan;
    int    n = pl->n[l];
    size_t m = (size_t)(n + 2) * (n + 2);
    if (pl->smoother[l] == ORC_SM_LU) {
        if (g->st_coarse_sweeps > 0) {
            /* study reading: a few Gauss-Seidel sweeps from zero on the
             * coarsest operator instead of the direct solve */
            memset(u, 0, m * sizeof(orc_cplx));
            for (int it = 0; it < g->st_coarse_sweeps; ++it) {
                if (g->opts.gs_order == ORC_ORDER_LEX) orc_gs_lex(n, pl->H[l], g->kv[l], pl->sigma_relax[l], f, u);
                else                                   orc_gs_rb(n, pl->H[l], g->kv[l], pl->sigma_relax[l], f, u);
            }
            return;
        }
        memcpy(u, f, m * sizeof(orc_cplx));
        orc_lu_solve((int)m, g->lu, g->piv, u);
        return;
    }
    memset(u, 0, m * sizeof(orc_cplx));
    relax(g, l, f, u, pl->pre[l]);
    orc_residual(n, pl->H[l], g->kv[l], pl->sigma_resid[l], f, u, g->r[l]);
    if (g->st_fw_transpose) restrict_transpose(n, g->r[l], g->f[l + 1]);
    else                    orc_restrict_fw(n, g->r[l], g->f[l + 1]);
    vcycle_level(g, l + 1, g->f[l + 1], g->u[l + 1]);
    orc_prolong_add(pl->n[l + 1], g->u[l + 1], u);
    relax(g, l, f, u, pl->post[l]);
}

/* ------------------------------------------------------------------------ */
/* O11: the V-cycle of the precision form.  The preconditioner keeps its    */
/* fields in complex single precision and computes in double: a value is    */
/* rounded to float (round to nearest even) exactly where the field holding */
/* it is stored, and every arithmetic step takes the float values widened   */
/* to double.  The outer Bi-CGSTAB, the operator L of the outer iteration   */
/* and the coarsest-grid operator (assembled from the unrounded k) stay     */
/* double.  Two schedules of stores are modelled:                           */
/*                                                                           */
/*   ORC_MIX_FUSED: the fields passed between fused kernels.  k on every     */
/*     level; each restricted right-hand side; each correction handed to    */
/*     the finer level; on Kaczmarz levels the iterate after every          */
/*     mix_kacz_every sweeps (the residual for the restriction is formed    */
/*     from the iterate before its last store of the pre-smoothing leg);   */
/*     Gauss-Seidel levels keep their pre-smoothed iterate in double;       */
/*     levels with n <= mix_block_n form one double-precision block whose  */
/*     only stored field is its result.                                     */
/*   ORC_MIX_ONEPASS: every elementary step stores: k, each colour pass of  */
/*     a sweep, each restriction, each prolongation-and-add, the coarsest   */
/*     result.                                                              */
/* With mix_round_io the cycle's input is rounded before the first step and */
/* its output after the last (otherwise both stay double).  With            */
/* fp64_levels = t > 0 (fused schedule) the finest t levels keep double     */
/* fields and k, and level t, the first in float, takes its right-hand side */
/* and returns its correction in double (t is clamped to the first level of */
/* the double block).  Only the coloured orders are modelled.               */
/* ------------------------------------------------------------------------ */

static double rnd32(double x) { return (double)(float)x; }

static void round_field(size_t m, orc_cplx *a)
{
    double *d = (double *)a;           /* C99: a complex is an array of two reals */
    for (size_t i = 0; i < 2 * m; ++i) d[i] = rnd32(d[i]);
}

/* one colour pass of red-black Gauss-Seidel (colour = (i + j) mod 2) */
static void gs_colour_pass(int n, double h, const double *k, double sigma,
                           const orc_cplx *f, orc_cplx *u, int colour)
{
    int M = n + 2, N = n + 1;
    for (int j = 0; j <= N; ++j)
        for (int i = (colour + j) & 1; i <= N; i += 2)
            gs_point(N, M, h, k, sigma, f, u, i, j);
}

/* one colour pass of the 5-colour Kaczmarz sweep (colour = (i + 2j) mod 5) */
static void kacz_colour_pass(int n, double h, const double *k, double sigma,
                             const orc_cplx *f, orc_cplx *u, int colour)
{
    int M = n + 2, N = n + 1;
    for (int j = 0; j <= N; ++j) {
        int i0 = ((colour - 2 * j) % 5 + 5) % 5;
        for (int i = i0; i <= N; i += 5)
            kacz_row(N, M, h, k, sigma, f, u, i, j);
    }
}

/* A relaxation leg of level l in the precision form.  last_store: round the
 * iterate after the leg's final sweep group (the pre-smoothing leg of a
 * fused Kaczmarz level stores it only after its residual has been formed). */
static void relax_mixed(orc_grid *g, int l, const orc_cplx *f, orc_cplx *u, int sweeps, int last_store)
{
    const orc_plan *pl = &g->plan;
    int    n = pl->n[l];
    size_t m = (size_t)(n + 2) * (n + 2);
    double H = pl->H[l], s = pl->sigma_relax[l];
    const double *k = g->kv[l];
    int onepass = g->mix_mode == ORC_MIX_ONEPASS;
    int kacz = pl->smoother[l] == ORC_SM_KACZ;
    int every = g->mix_kacz_every > 0 ? g->mix_kacz_every : sweeps;
    int stores = l >= g->mix_t;          /* the level's fields are float */
    for (int it = 0; it < sweeps; ++it) {
        int ncol = kacz ? 5 : 2;
        for (int c = 0; c < ncol; ++c) {
            if (kacz) kacz_colour_pass(n, H, k, s, f, u, c);
            else      gs_colour_pass(n, H, k, s, f, u, c);
            if (onepass && stores) round_field(m, u);
        }
        if (!onepass && stores && kacz && ((it + 1) % every == 0) && (it + 1 < sweeps || last_store))
            round_field(m, u);
    }
}

/* Level l of the mixed cycle; u is left unrounded where the caller stores
 * it (the caller rounds the level's result). */
static void vcycle_mixed(orc_grid *g, int l, const orc_cplx *f, orc_cplx *u)
{
    const orc_plan *pl = &g->plan;
    int    n = pl->n[l], nc;
    size_t m = (size_t)(n + 2) * (n + 2), mc;
    int    onepass = g->mix_mode == ORC_MIX_ONEPASS;
    if (pl->smoother[l] == ORC_SM_LU) {
        memcpy(u, f, m * sizeof(orc_cplx));
        orc_lu_solve((int)m, g->lu, g->piv, u);
        return;
    }
    if (!onepass && n <= g->mix_block_n) {   /* the double-precision block */
        vcycle_level(g, l, f, u);
        return;
    }
    int kacz = pl->smoother[l] == ORC_SM_KACZ;
    int stores = l >= g->mix_t;                 /* this level's fields are float    */
    int cstores = l + 1 > g->mix_t;             /* the coarse fields handed over are */
    nc = pl->n[l + 1];
    mc = (size_t)(nc + 2) * (nc + 2);
    memset(u, 0, m * sizeof(orc_cplx));
    relax_mixed(g, l, f, u, pl->pre[l], 0);
    orc_residual(n, pl->H[l], g->kv[l], pl->sigma_resid[l], f, u, g->r[l]);
    if (stores && kacz && !onepass && pl->pre[l] > 0) round_field(m, u);
    orc_restrict_fw(n, g->r[l], g->f[l + 1]);
    if (cstores) round_field(mc, g->f[l + 1]);
    vcycle_mixed(g, l + 1, g->f[l + 1], g->u[l + 1]);
    if (cstores) round_field(mc, g->u[l + 1]);
    orc_prolong_add(nc, g->u[l + 1], u);
    if (onepass && stores) round_field(m, u);
    relax_mixed(g, l, f, u, pl->post[l], 1);
}

void orc_grid_set_mixed(orc_grid *g, int mode, int kacz_every, int block_n, int round_io)
{
    orc_grid_set_mixed_ex(g, mode, kacz_every, block_n, round_io, 0);
}

void orc_grid_set_mixed_ex(orc_grid *g, int mode, int kacz_every, int block_n, int round_io,
                           int fp64_levels)
{
    g->mix_mode = mode;
    g->mix_kacz_every = kacz_every;
    g->mix_block_n = block_n;
    g->mix_round_io = round_io;
    g->mix_t = (mode == ORC_MIX_FUSED) ? fp64_levels : 0;
    for (int l = 0; l < g->plan.nlev && l < g->mix_t; ++l)
        if (g->plan.n[l] <= block_n || g->plan.smoother[l] == ORC_SM_LU) { g->mix_t = l; break; }
    for (int l = 0; l < g->plan.nlev; ++l) {
        size_t m = (size_t)(g->plan.n[l] + 2) * (g->plan.n[l] + 2);
        if (g->kv[l] != g->k[l]) free(g->kv[l]);
        g->kv[l] = g->k[l];
        if (mode == ORC_MIX_OFF || l < g->mix_t) continue;
        g->kv[l] = malloc(m * sizeof(double));
        for (size_t q = 0; q < m; ++q) g->kv[l][q] = rnd32(g->k[l][q]);
    }
}

void orc_vcycle(orc_grid *g, const orc_cplx *f, orc_cplx *u)
{
    if (g->mix_mode == ORC_MIX_OFF) {
        vcycle_level(g, 0, f, u);
        return;
    }
    size_t m = (size_t)(g->n + 2) * (g->n + 2);
    orc_cplx *fin = malloc(m * sizeof(orc_cplx));
    memcpy(fin, f, m * sizeof(orc_cplx));
    int rio = g->mix_round_io && g->mix_t == 0;
    if (rio) round_field(m, fin);
    vcycle_mixed(g, 0, fin, u);
    if (rio) round_field(m, u);
    free(fin);
}

/* ------------------------------------------------------------------------ */
/* Ray correction (Section 6.1).  Near-kernel error is written as a sum of  */
/* the 8 plane waves exp(i kappa_j . x), kappa_j = k (cos(j pi/4),          */
/* sin(j pi/4)), j = 1..8, times smooth ray functions a_j.  Reading taken   */
/* (the construction of the cited wave-ray papers is not available): each   */
/* a_j is bilinear on a vertex-centred ray grid of ray_n interior nodes per */
/* side over the same square, so the correction space is spanned by the     */
/* fine-grid vectors                                                        */
/*     P e_(j,a) (x) = exp(i kappa_j . x) phi_a(x),                         */
/* phi_a the bilinear hat of ray-grid node a, and the correction of a        */
/* residual w is the Galerkin one, P (P^H L P)^{-1} P^H w.  The ray         */
/* wavenumber is the mean of k over the nodes (k itself for the constant-k  */
/* problems of the paper).  The basis is stored as a dense matrix here: the */
/* oracle is for small grids.                                               */
/* ------------------------------------------------------------------------ */

static double nrm2_plain(size_t m, const orc_cplx *a)
{
    double s = 0.0;
    for (size_t i = 0; i < m; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return sqrt(s);
}

/* value of the bilinear hat of ray-grid node (ia, ja) at the point (x, y);
 * the ray grid spans the same square [0, len]^2 as the fine grid */
static double ray_hat(int nr, double len, int ia, int ja, double x, double y)
{
    double Hr = len / (nr + 1);
    double wx = 1.0 - fabs(x / Hr - ia), wy = 1.0 - fabs(y / Hr - ja);
    return (wx > 0.0 && wy > 0.0) ? wx * wy : 0.0;
}

int orc_grid_set_ray(orc_grid *g, int ray_n)
{
    free(g->ray_P); free(g->ray_A); free(g->ray_piv);
    g->ray_P = NULL; g->ray_A = NULL; g->ray_piv = NULL;
    g->ray_n = 0;
    if (ray_n <= 0) return 0;
    int    n = g->n, M = n + 2, Mr = ray_n + 2;
    size_t m = (size_t)M * M, K = (size_t)8 * Mr * Mr;
    double h = g->h;
    g->ray_P   = malloc(m * K * sizeof(orc_cplx));
    g->ray_A   = malloc(K * K * sizeof(orc_cplx));
    g->ray_piv = malloc(K * sizeof(int));
    double kr = 0.0;
    for (size_t p = 0; p < m; ++p) kr += g->k[0][p];
    kr /= (double)m;
    /* the basis, column (j, a) with j = 1..8 stored as 0..7 */
    for (size_t p = 0; p < m; ++p) {
        int    i = (int)(p % M), jj = (int)(p / M);
        double x = i * h, y = jj * h, kp = kr;
        for (int d = 0; d < 8; ++d) {
            double   th = (d + 1) * ORC_PI / 4.0;
            orc_cplx wave = cexp(I * kp * (cos(th) * x + sin(th) * y));
            for (int a = 0; a < Mr * Mr; ++a)
                g->ray_P[p * K + (size_t)d * Mr * Mr + a] =
                    wave * ray_hat(ray_n, (n + 1) * h, a % Mr, a / Mr, x, y);
        }
    }
    /* P^H L P, column by column */
    orc_cplx *col = malloc(m * sizeof(orc_cplx)), *lcol = malloc(m * sizeof(orc_cplx));
    for (size_t c = 0; c < K; ++c) {
        for (size_t p = 0; p < m; ++p) col[p] = g->ray_P[p * K + c];
        orc_apply(n, h, g->k[0], 0.0, col, lcol);
        for (size_t r = 0; r < K; ++r) {
            orc_cplx acc = 0.0;
            for (size_t p = 0; p < m; ++p) acc += conj(g->ray_P[p * K + r]) * lcol[p];
            g->ray_A[r * K + c] = acc;
        }
    }
    free(col); free(lcol);
    if (orc_lu_factor((int)K, g->ray_A, g->ray_piv) != 0) return -1;
    g->ray_n = ray_n;
    return 0;
}

/* u += P (P^H L P)^{-1} P^H (f - L u) */
void orc_ray_correct(orc_grid *g, const orc_cplx *f, orc_cplx *u)
{
    if (!g->ray_n) return;
    int    n = g->n, Mr = g->ray_n + 2;
    size_t m = (size_t)(n + 2) * (n + 2), K = (size_t)8 * Mr * Mr;
    orc_cplx *w = malloc(m * sizeof(orc_cplx)), *b = malloc(K * sizeof(orc_cplx));
    orc_residual(n, g->h, g->k[0], 0.0, f, u, w);
    for (size_t r = 0; r < K; ++r) {
        orc_cplx acc = 0.0;
        for (size_t p = 0; p < m; ++p) acc += conj(g->ray_P[p * K + r]) * w[p];
        b[r] = acc;
    }
    orc_lu_solve((int)K, g->ray_A, g->ray_piv, b);
    for (size_t p = 0; p < m; ++p) {
        orc_cplx acc = 0.0;
        for (size_t c = 0; c < K; ++c) acc += g->ray_P[p * K + c] * b[c];
        u[p] += acc;
    }
    free(w); free(b);
}

/* The preconditioner with the ray correction after the V-cycle:
 * z = B_V r, then z += C_R (r - L z), i.e. B = B_V + C_R (I - L B_V). */
static void vcycle_ray(orc_grid *g, const orc_cplx *r, orc_cplx *z)
{
    orc_vcycle(g, r, z);
    orc_ray_correct(g, r, z);
}

/* Stationary iteration with the (ray-corrected) V-cycle as the solver
 * (Section 6.1, Table 4): x <- x + B (f - L x) until ||f - L x|| <= rtol
 * ||f||; returns the number of cycles (maxit if not reached). */
int orc_cycles(orc_grid *g, const orc_cplx *f, orc_cplx *x, double rtol, int maxit, double *res_hist)
{
    int    n = g->n;
    size_t m = (size_t)(n + 2) * (n + 2);
    orc_cplx *r = malloc(m * sizeof(orc_cplx)), *z = malloc(m * sizeof(orc_cplx));
    double bn = nrm2_plain(m, f);
    if (bn == 0.0) bn = 1.0;
    int it = 0;
    for (;; ++it) {
        orc_residual(n, g->h, g->k[0], 0.0, f, x, r);
        double rel = nrm2_plain(m, r) / bn;
        if (res_hist) res_hist[it] = rel;
        if (rel <= rtol || it >= maxit || !isfinite(rel)) break;
        vcycle_ray(g, r, z);
        for (size_t p = 0; p < m; ++p) x[p] += z[p];
    }
    free(r); free(z);
    return it;
}

/* ------------------------------------------------------------------------ */
/* Bi-CGSTAB (Section 6): x^0 = 0, right preconditioning (so r is the true  */
/* residual of the unpreconditioned system), preconditioner applied twice   */
/* per iteration, iterations counted in halves.  Stop when ||r||/||b|| <=   */
/* rtol; on that signal the residual is recomputed as b - A x and accepted  */
/* only if it also meets rtol (otherwise the iteration restarts from it).   */
/* Breakdown |rho| <= 1e-14 ||rhat|| ||r|| restarts with rhat = r.          */
/* Inner products are (a,b) = sum conj(a_i) b_i.                            */
/* ------------------------------------------------------------------------ */

static orc_cplx dotc(size_t m, const orc_cplx *a, const orc_cplx *b)
{
    orc_cplx s = 0.0;
    for (size_t i = 0; i < m; ++i) s += conj(a[i]) * b[i];
    return s;
}

static double nrm2(size_t m, const orc_cplx *a)
{
    double s = 0.0;
    for (size_t i = 0; i < m; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return sqrt(s);
}

static void precondition(orc_grid *g, int precond, const orc_cplx *in, orc_cplx *out, size_t m)
{
    if (precond == ORC_PREC_VCYCLE) {
        vcycle_ray(g, in, out);
    } else if (precond == ORC_PREC_EXACT) {
        if (!g->exact_lu) {
            g->exact_lu  = malloc(m * m * sizeof(orc_cplx));
            g->exact_piv = malloc(m * sizeof(int));
            orc_dense(g->n, g->h, g->k[0], 0.0, g->exact_lu);
            orc_lu_factor((int)m, g->exact_lu, g->exact_piv);
        }
        memcpy(out, in, m * sizeof(orc_cplx));
        orc_lu_solve((int)m, g->exact_lu, g->exact_piv, out);
    } else {
        memcpy(out, in, m * sizeof(orc_cplx));
    }
}

int orc_bicgstab(orc_grid *g, const orc_cplx *b, orc_cplx *x, double rtol,
                 int maxit, int precond, orc_info *info,
                 double *res_hist, int hist_cap)
{
    return orc_bicgstab_ex(g, b, x, rtol, maxit, precond, info, res_hist, hist_cap, 0);
}

int orc_bicgstab_ex(orc_grid *g, const orc_cplx *b, orc_cplx *x, double rtol,
                    int maxit, int precond, orc_info *info,
                    double *res_hist, int hist_cap, int force_breakdown_at)
{
    return orc_bicgstab_ex2(g, b, x, rtol, maxit, precond, info, res_hist, hist_cap,
                            force_breakdown_at, 0, 0);
}

/* true_res_every = K > 0: after every K-th full iteration (counted among the
 * full iterations that miss the tolerance) the residual is recomputed as b - A x; if that meets the
 * tolerance the solve ends, otherwise it restarts from it (rhat = r, p = v =
 * 0), as after a failed convergence check.  A residual norm that is not
 * finite ends the solve with ORC_BREAKDOWN; nan_at = K > 0 treats the norm
 * at the end of iteration K as not finite (tests of that path). */
int orc_bicgstab_ex2(orc_grid *g, const orc_cplx *b, orc_cplx *x, double rtol,
                     int maxit, int precond, orc_info *info,
                     double *res_hist, int hist_cap, int force_breakdown_at,
                     int true_res_every, int nan_at)
{
    int    n = g->n;
    double h = g->h;
    size_t m = (size_t)(n + 2) * (n + 2);
    orc_cplx *r  = malloc(m * sizeof(orc_cplx)), *rh = malloc(m * sizeof(orc_cplx));
    orc_cplx *p  = calloc(m, sizeof(orc_cplx)),  *v  = calloc(m, sizeof(orc_cplx));
    orc_cplx *ph = malloc(m * sizeof(orc_cplx)), *s  = malloc(m * sizeof(orc_cplx));
    orc_cplx *sh = malloc(m * sizeof(orc_cplx)), *t  = malloc(m * sizeof(orc_cplx));
    double bn = nrm2(m, b);
    int    half = 0, nhist = 0, status = ORC_NOT_CONVERGED, fulls = 0;
    info->restarts = 0;
    info->vcycles  = 0;
    if (bn == 0.0) bn = 1.0;

    orc_residual(n, h, g->k[0], 0.0, b, x, r);     /* r = b - L x */
    memcpy(rh, r, m * sizeof(orc_cplx));
    orc_cplx rho_old = 1.0, alpha = 1.0, omega = 1.0;
    double   rn = nrm2(m, r);
    if (res_hist && nhist < hist_cap) res_hist[nhist++] = rn / bn;
    int converged = (rn / bn <= rtol);

    for (;;) {
        if (converged) {
            /* true residual check; on failure restart from it (rhat = r) */
            orc_residual(n, h, g->k[0], 0.0, b, x, r);
            rn = nrm2(m, r);
            if (rn / bn <= rtol) { status = ORC_OK; break; }
            converged = 0;
            memcpy(rh, r, m * sizeof(orc_cplx));
            memset(p, 0, m * sizeof(orc_cplx));
            memset(v, 0, m * sizeof(orc_cplx));
            rho_old = alpha = omega = 1.0;
            info->restarts++;
        }
        if (half >= 2 * maxit) break;
        orc_cplx rho = dotc(m, rh, r);
        int forced = force_breakdown_at > 0 && half == 2 * force_breakdown_at;
        if (cabs(rho) <= 1e-14 * nrm2(m, rh) * rn || forced) {
            memcpy(rh, r, m * sizeof(orc_cplx));
            memset(p, 0, m * sizeof(orc_cplx));
            memset(v, 0, m * sizeof(orc_cplx));
            rho_old = alpha = omega = 1.0;
            rho = dotc(m, rh, r);
            info->restarts++;
        }
        orc_cplx beta = (rho / rho_old) * (alpha / omega);
        for (size_t i = 0; i < m; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        precondition(g, precond, p, ph, m);
        info->vcycles++;
        orc_apply(n, h, g->k[0], 0.0, ph, v);
        alpha = rho / dotc(m, rh, v);
        for (size_t i = 0; i < m; ++i) s[i] = r[i] - alpha * v[i];
        half++;
        double sn = nrm2(m, s);
        if (res_hist && nhist < hist_cap) res_hist[nhist++] = sn / bn;
        if (!isfinite(sn)) { status = ORC_BREAKDOWN; break; }
        if (sn / bn <= rtol) {
            for (size_t i = 0; i < m; ++i) x[i] += alpha * ph[i];
            converged = 1;
            continue;
        }
        precondition(g, precond, s, sh, m);
        info->vcycles++;
        orc_apply(n, h, g->k[0], 0.0, sh, t);
        omega = dotc(m, t, s) / dotc(m, t, t);
        for (size_t i = 0; i < m; ++i) {
            x[i] += alpha * ph[i] + omega * sh[i];
            r[i] = s[i] - omega * t[i];
        }
        half++;
        rho_old = rho;
        rn = nrm2(m, r);
        if (nan_at > 0 && half == 2 * nan_at) rn = NAN;
        if (res_hist && nhist < hist_cap) res_hist[nhist++] = rn / bn;
        if (!isfinite(rn)) { status = ORC_BREAKDOWN; break; }
        if (rn / bn <= rtol) {
            converged = 1;
        } else if (true_res_every > 0 && ++fulls % true_res_every == 0 && half < 2 * maxit) {
            orc_residual(n, h, g->k[0], 0.0, b, x, r);
            rn = nrm2(m, r);
            if (rn / bn <= rtol) {
                converged = 1;
            } else {
                memcpy(rh, r, m * sizeof(orc_cplx));
                memset(p, 0, m * sizeof(orc_cplx));
                memset(v, 0, m * sizeof(orc_cplx));
                rho_old = alpha = omega = 1.0;
                info->restarts++;
            }
        }
    }
    /* final true relative residual */
    orc_residual(n, h, g->k[0], 0.0, b, x, r);
    info->rel_res   = nrm2(m, r) / bn;
    info->halfsteps = half;
    info->status    = status;
    free(r); free(rh); free(p); free(v); free(ph); free(s); free(sh); free(t);
    return status;
}
