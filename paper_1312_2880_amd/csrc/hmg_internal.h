// hmg_internal.h -- declarations shared by the kernel and host translation
// units of libhmg.  Not part of the public C-ABI (include/hmg.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hmgk {

enum Prec { P64 = 0, P32 = 1 };

// Geometry of one level: n interior nodes per side, M = n + 2 nodes per
// side, N = n + 1 intervals, spacing H.  Fields are dense M x M, x fastest.
struct Geo {
    int    n, M, N;
    double H;
};

inline Geo make_geo(int n, double H) { return Geo{n, n + 2, n + 1, H}; }

// Scalars of one Bi-CGSTAB solve, resident in device memory.  Complex
// numbers are stored as (re, im) pairs.
struct KState {
    double rho[2], rho_old[2], alpha[2], omega[2], beta[2];
    double bnorm;        // ||b|| (1 if b = 0)
    double rnorm2;       // ||r||^2 of the current residual
    double snorm2;       // ||s||^2 of the current half step
    double rhat_norm2;   // ||rhat||^2
    double rtol;
    double true_rel;     // ||b - L x|| / ||b|| from the last true-residual check
    int    halfsteps;
    int    maxhalf;
    int    done;         // 0 running, 1 recursive residual met rtol, 2 maxit,
                         // 3 a residual norm was not finite
    int    half_exit;    // converged at the half step of this iteration
    int    restart;      // next p-update restarts with rhat = p = r
    int    stop;         // done || half_exit: later kernels of the iteration skip
    int    restarts;
    int    hist_cap;
    int    force_bd;     // > 0: iteration after which a breakdown is forced
    int    true_every;   // > 0: true-residual check after every true_every-th full iteration
    int    nan_at;       // > 0: the norm after iteration nan_at is taken as NaN (test hook)
    int    fullits;      // full iterations that missed rtol (the true_every counter)
    int    check;        // a true-residual check is due after this iteration
};

// A batched launch runs one kernel on nz right-hand sides of a grid at once
// (blockIdx.z): every per-right-hand-side buffer of slot z lies zs bytes
// after the same buffer of slot z - 1 (the slots of a grid are carved with
// one layout), so a kernel offsets those pointers by blockIdx.z * zs and
// leaves the shared ones (k, row tables, the bottom matrix) alone.
struct Bz {
    long zs = 0;
    int  nz = 1;
};

// Device pointers of one solve slot (finest-level Krylov vectors).
struct Krylov {
    double *b, *x, *r, *rh, *p, *v, *s, *t, *ph, *sh;   // complex interleaved
    double *partials;    // reduction scratch: 3 x pcap doubles
    int     pcap;        // partial sums per quantity the scratch holds (>= nblocks)
    double *hist;        // relative residual per half step
    KState *st;
    int    *done_host;   // pinned host copy of st->done, written by the device
    int     nblocks;
};

// ---- multigrid building blocks (templated on precision via Prec) --------
// k: real field of the level in the level precision; complex fields likewise.
void launch_apply(Prec p, hipStream_t s, const Geo &g, const void *k, double sigma,
                  const void *u, void *out);
void launch_gs_colour(Prec p, hipStream_t s, const Geo &g, const void *k, double sigma,
                      const void *f, void *u, int colour, int zero_guess, const int *skip);
void launch_kacz_colour(Prec p, hipStream_t s, const Geo &g, const void *k, double sigma,
                        const void *f, void *u, int colour, const int *skip);
void launch_fill_zero(Prec p, hipStream_t s, void *u, size_t count, const int *skip, Bz bz = {});
void launch_residual_fw(Prec p, hipStream_t s, const Geo &g, const void *k, double sigma,
                        const void *f, const void *u, void *fc, const int *skip, Bz bz = {});
void launch_prolong_add(Prec p, hipStream_t s, const Geo &gfine, const void *ec, void *u,
                        const int *skip, Bz bz = {});
void launch_coarsest(Prec p, hipStream_t s, int m, const double *ainv_t, const void *f,
                     void *u, const int *skip);
void launch_convert(hipStream_t s, int to_float, const void *src, void *dst, size_t count,
                    const int *skip, Bz bz = {});

// ---- lexicographic sweeps (hmg_lex.hip) -------------------------------------
// One sweep in lexicographic order (x fastest) of Gauss-Seidel (kacz = 0) or
// Kaczmarz (kacz = 1) on A_sigma u = f, in place on u; launches one kernel
// per tile diagonal of the wavefront.
void launch_lex_sweep(Prec p, int kacz, hipStream_t s, const Geo &g, const void *k, double sigma,
                      const void *f, void *u, const int *skip);

// ---- fused LDS-tiled kernels (hmg_fused.hip) --------------------------------
constexpr int HMG_SM_GS_DEV = 0, HMG_SM_KACZ_DEV = 1;
constexpr int BOT_MAXL = 6;

struct BottomLevelDesc {
    int         n;
    double      H, sa, sb;
    const void *k;
    int         sm, pre, post;
    int         uoff, foff;     // complex-slot offsets of u and f in the LDS arena
    int         koff;           // real-slot offset of k
};
struct BottomDesc {
    int             nlev;
    BottomLevelDesc L[BOT_MAXL];
    const double   *ainv_t;
};
struct KaczCfg {
    int ts, sweeps, threads;    // tile width, sweeps per launch, workgroup size
    int ty, rty;                // tile height; that of the RESID form before its shrink by 4
};
constexpr int KACZ_NCFG = 8;
constexpr int KACZ_DEFAULT = 7;   // the LDS-staged 16 x 8 tile, 2 sweeps per launch
extern const KaczCfg kKaczCfgs[KACZ_NCFG];
bool   kacz_cfg_fits(Prec p, int cfg);
int    bottom_complex_slots();   // LDS capacity of the bottom solver
int    bottom_real_slots();

// f64in / io64: the level-0 input (and output) are FP64 while the level
// computes in float (mixed precision).
void launch_gs_down(Prec p, bool f64in, hipStream_t s, const Geo &g, const void *k, double sa, double sb,
                    const void *f, void *uo, void *fc, const int *skip, bool uo_black = false, Bz bz = {});
// uo may be null in launch_gs_down (the smoothed iterate is not stored);
// uo_black: store it on the black nodes only (all that launch_gs_up reads);
// launch_gs_up recomputes it from f.
// u0: the pre-smoothed iterate stored by launch_gs_down, or null (recomputed
// from f)
void launch_gs_up(Prec p, bool io64, hipStream_t s, const Geo &g, const void *k, double sa, const void *f,
                  const void *u0, const void *ec, void *uo, const int *skip, Bz bz = {});
// The finest up kernel of an FP64 solve fused with the Bi-CGSTAB product
// (kind 1: v = L uo with the partials of (dot, v); kind 2: t = L uo with the
// partials of (t, dot) and (t, t)); partials laid out for gs_up_mv_blocks(g)
// blocks; uo may be null (the iterate is not stored).  Only where gs_up_mv_ok
// (FP64 level without a stored iterate, big tiles).
bool gs_up_mv_ok(Prec p, const Geo &g);
int  gs_up_mv_blocks(const Geo &g);
void launch_gs_up_mv(hipStream_t s, int kind, const Geo &g, const void *k, double sa, const void *f,
                     const void *ec, void *uo, void *mvo, const void *dot, double *partials, const int *skip,
                     Bz bz = {});
// tab: (k_p, 1 / ||a_p||^2) for sigma from launch_kacz_table, or null (the
// kernel forms them)
void launch_kacz_tb(Prec p, int cfg, hipStream_t s, const Geo &g, const void *k, const double *tab, double sig,
                    const void *f, const void *ui, const void *ec, void *uo, const int *skip, Bz bz = {});
void launch_kacz_table(Prec p, hipStream_t s, const Geo &g, const void *k, double sig, double *tab);
// a whole level (n <= 63) in one workgroup: `sweeps` sweeps from ui (null:
// zero) + P ec (null: none) into uo, then fc = R (f - A_{sigb} uo) if fc
bool kacz_level_fits(const Geo &g);
void launch_kacz_level(Prec p, hipStream_t s, const Geo &g, const void *k, const double *tab, double sig,
                       double sigb, int sweeps, const void *f, const void *ui, const void *ec, void *uo, void *fc,
                       const int *skip);
bool kacz_cfg_resid(int cfg);   // configuration has the fused residual form
// S sweeps (configuration cfg) from ui (null: zero), then fc = R (f - A_{sigb} u)
void launch_kacz_tb_resid(Prec p, int cfg, hipStream_t s, const Geo &g, const void *k, const double *tab,
                          double sig, double sigb, const void *f, const void *ui, void *uo, void *fc,
                          const int *skip, Bz bz = {});
void launch_bottom(Prec p, bool io64, hipStream_t s, const BottomDesc &d, const void *f, void *uo,
                   const int *skip);
int  bottom_matrix_size(const BottomDesc &d);
void launch_bottom_basis(Prec p, hipStream_t s, const BottomDesc &d, double *B);
void launch_dense_apply(Prec p, bool io64, hipStream_t s, const double *B, int m, const void *f, void *u,
                        const int *skip, Bz bz = {});

// ---- ray correction (hmg_ray.hip) -------------------------------------------
// Geometry of the ray grid over the finest level: fine N = n + 1 intervals and
// M = n + 2 nodes per side; ray grid nr interior nodes, Mr = nr + 2 nodes and
// Nr = nr + 1 cells of c fine intervals per side; the restriction works on
// patches of P x P fine nodes (P divides c), np per side.
struct RayGeo {
    int N, M;
    int nr, Mr, Nr;
    int c;
    int P;
    int np;
};
// z += P A^{-1} P^H (r - L z) on FP64 finest-level fields (k: FP64 finest k;
// ex, ey: the wave tables; part, b, a: the correction's scratch)
void launch_ray_correct(hipStream_t s, const RayGeo &R, double H, const double *k, const void *ex, const void *ey,
                        const double *Ainv, const void *r, void *z, double *part, void *b, void *a,
                        const int *skip, Bz bz = {});
// column col of A = P^H L P (row-major K x K) into A; zfine: a scratch FP64
// finest-level field
void launch_ray_column(hipStream_t s, const RayGeo &R, double H, const double *k, const void *ex, const void *ey,
                       void *zfine, double *part, void *b, void *a, void *A, int col);

// ---- Bi-CGSTAB (FP64, finest level, L = A_0) -------------------------------
// Every launcher runs on one slot K, or batched (kb.nz > 1) on the kb.nz
// slots from K on: their vectors, partial sums and scalars kb.zs bytes apart,
// their residual histories kb.hz bytes apart.
struct Kz {
    long zs = 0, hz = 0;
    int  nz = 1;
};
int  krylov_nblocks(const Geo &g);
void kry_init(hipStream_t s, const Geo &g, const double *k, const Krylov &K, int x0_given,
              double rtol, int maxhalf, int force_bd, int true_every = 0, int nan_at = 0,
              Kz kb = {});
// The periodic true-residual check (when due): r = b - L x; the solve ends
// if it meets rtol, else restarts from it (rhat = p = r).
void kry_checkpoint(hipStream_t s, const Geo &g, const double *k, const Krylov &K, Kz kb = {});
void kry_update_p(hipStream_t s, const Geo &g, const Krylov &K, Kz kb = {});
void kry_matvec_alpha(hipStream_t s, const Geo &g, const double *k, const Krylov &K, Kz kb = {});
// the single-block finalisations after a fused product (nb partial blocks)
void kry_alpha_fin(hipStream_t s, const Krylov &K, int nb, Kz kb = {});
// out[0..2] = the totals of nv (2 or 3) block partials, zero-padded
void launch_sum_partials(hipStream_t s, const double *partials, int nb, int nv, double *out);
void kry_omega_fin(hipStream_t s, const Krylov &K, int nb, Kz kb = {});
void kry_update_s(hipStream_t s, const Geo &g, const Krylov &K, Kz kb = {});
void kry_matvec_omega(hipStream_t s, const Geo &g, const double *k, const Krylov &K, Kz kb = {});
void kry_update_xr(hipStream_t s, const Geo &g, const Krylov &K, Kz kb = {});
// The x update kept in the preconditioner's input space (y in K.ph):
// y += alpha p + omega s with r and its sums as kry_update_xr; kry_fold
// adds z = B y (in K.sh) to x and clears y.
void kry_update_yr(hipStream_t s, const Geo &g, const Krylov &K, Kz kb = {});
void kry_fold(hipStream_t s, const Geo &g, const Krylov &K);
void kry_true_residual(hipStream_t s, const Geo &g, const double *k, const Krylov &K);
void kry_restart_from_true(hipStream_t s, const Krylov &K);

}  // namespace hmgk
