// hmg_api.hip -- host side of libhmg: the C-ABI of include/hmg.h, the level
// plan, the hierarchy, the coarsest-grid factorisation, the V-cycle schedule
// and the Bi-CGSTAB driver (Livshits, arXiv:1312.2880, Sections 1, 5, 6).

#include "hmg.h"
#include "hmg_internal.h"
#include "hmg_host.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace hmgk;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

hmg_status hmg_fail(hmg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

extern "C" const char *hmg_last_error(void) { return g_last_error.c_str(); }

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return hmg_fail(HMG_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

double hmg_now() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// options and plan
// ---------------------------------------------------------------------------
extern "C" void hmg_opts_default(hmg_opts *o) {
    std::memset(o, 0, sizeof *o);
    o->variant = HMG_HYB;
    o->precision = HMG_FP64;
    o->beta = 0.5;
    o->nu_pre = 1;
    o->nu_post = 1;
    o->kacz_pre = 4;
    o->kacz_post = 4;
    o->kacz_band = 1;
    o->coarsest_n = 7;
    o->use_graph = 1;
    o->one_pass_kernels = 0;
    o->autotune = 1;
    o->bottom_dense = 1;
}

// Level classification (Section 5).  The paper states its rules on grids
// with kH = 0.3125 * 2^j and constant k; for a level whose nodes span
// [kH_min, kH_max] the first matching rule applies:
//   last level                       -> dense LU on M (SL) or L (HLM, HYB);
//   kacz_band, span meets [1.25/sqrt2, 1.25 sqrt2)
//                                    -> Kaczmarz 4+4 on M (SL, HYB) or L (HLM);
//   kacz_band, span meets [1.25 sqrt2, 2.5)
//                                    -> Kaczmarz 4+4 on M (SL) or L (HLM, HYB)
//                                       (Section 4: Gauss-Seidel is good only
//                                       up to kH ~ 0.625 and from ~ 2.5 on;
//                                       where it fails, the normal equation);
//   HYB, span meets [0.625/sqrt2, 0.625 sqrt2)
//                                    -> Gauss-Seidel on M;
//   otherwise                        -> Gauss-Seidel on M (SL) or L (HLM, HYB).
// With opts.hyb_mid (HYB only) M is the relaxation operator on every level
// whose span meets [0.625/sqrt2, 2.5 sqrt2) (the intermediate scales of the
// hybrid's motivation in Section 5), the Kaczmarz levels of that span included.
// Residuals (role (B)) use M for SL and L for HLM and HYB.
static void classify_level(const hmg_opts &o, hmg_plan &pl, int l, bool last, const double *k) {
    int n = pl.n[l], M = n + 2;
    double H = pl.H[l], lo = 1e300, hi = -1e300, beta = o.beta;
    for (int j = 0; j < M; ++j)
        for (int i = 0; i < M; ++i) {
            double kh = k[(size_t)j * M + i] * H;
            lo = std::min(lo, kh);
            hi = std::max(hi, kh);
        }
    pl.kHmin[l] = lo;
    pl.kHmax[l] = hi;
    bool sl = (o.variant == HMG_SL);
    pl.sigma_resid[l] = sl ? beta : 0.0;
    if (last) {
        pl.smoother[l] = HMG_SM_LU;
        pl.sigma_relax[l] = sl ? beta : 0.0;
        pl.pre[l] = pl.post[l] = 0;
        return;
    }
    const double r2 = std::sqrt(2.0);
    const double sig = sl ? beta : 0.0;
    bool band_k = hi >= 1.25 / r2 && lo < 1.25 * r2;
    bool band_w = hi >= 1.25 * r2 && lo < 2.5;
    const bool mid = o.variant == HMG_HYB && o.hyb_mid;
    bool band_m = hi >= 0.625 / r2 && lo < (mid ? 2.5 : 0.625) * r2;
    if (o.kacz_band && (band_k || band_w)) {
        pl.smoother[l] = HMG_SM_KACZ;
        pl.sigma_relax[l] = band_k ? ((o.variant == HMG_HLM) ? 0.0 : beta) : (mid ? beta : sig);
        pl.pre[l] = o.kacz_pre;
        pl.post[l] = o.kacz_post;
        return;
    }
    if (o.variant == HMG_HYB && band_m) {
        pl.smoother[l] = HMG_SM_GS;
        pl.sigma_relax[l] = beta;
        pl.pre[l] = o.nu_pre;
        pl.post[l] = o.nu_post;
        return;
    }
    pl.smoother[l] = HMG_SM_GS;
    pl.sigma_relax[l] = sig;
    pl.pre[l] = o.nu_pre;
    pl.post[l] = o.nu_post;
}

// ---------------------------------------------------------------------------
// coarsest level: dense A_sigma, LU with partial pivoting, explicit inverse
// ---------------------------------------------------------------------------
typedef std::complex<double> cd;

static void dense_operator(int n, double H, const double *k, double sigma, std::vector<cd> &A) {
    int M = n + 2, N = n + 1;
    size_t m = (size_t)M * M;
    A.assign(m * m, cd(0.0, 0.0));
    double ih2 = 1.0 / (H * H);
    for (int j = 0; j <= N; ++j)
        for (int i = 0; i <= N; ++i) {
            size_t p = (size_t)j * M + i;
            double kp = k[p];
            int b = (i == 0) + (i == N) + (j == 0) + (j == N);
            A[p * m + p] = cd(-4.0 * ih2 + kp * kp, 2.0 * kp * H * b * ih2 + kp * kp * sigma);
            if (i > 0) A[p * m + p - 1] += ((i == N) ? 2.0 : 1.0) * ih2;
            if (i < N) A[p * m + p + 1] += ((i == 0) ? 2.0 : 1.0) * ih2;
            if (j > 0) A[p * m + p - M] += ((j == N) ? 2.0 : 1.0) * ih2;
            if (j < N) A[p * m + p + M] += ((j == 0) ? 2.0 : 1.0) * ih2;
        }
}

// Inverse of A (m x m, row-major) via LU with partial pivoting; returns it
// column-major (out[c*m + r] = inv(r, c)).  false if singular.
static bool invert_dense(size_t m, std::vector<cd> A, std::vector<cd> &out) {
    std::vector<size_t> piv(m);
    for (size_t c = 0; c < m; ++c) {
        size_t p = c;
        double best = std::abs(A[c * m + c]);
        for (size_t r = c + 1; r < m; ++r)
            if (std::abs(A[r * m + c]) > best) { best = std::abs(A[r * m + c]); p = r; }
        if (best == 0.0) return false;
        piv[c] = p;
        if (p != c)
            for (size_t q = 0; q < m; ++q) std::swap(A[c * m + q], A[p * m + q]);
        for (size_t r = c + 1; r < m; ++r) {
            cd l = A[r * m + c] / A[c * m + c];
            A[r * m + c] = l;
            for (size_t q = c + 1; q < m; ++q) A[r * m + q] -= l * A[c * m + q];
        }
    }
    out.assign(m * m, cd(0.0, 0.0));
    std::vector<cd> x(m);
    for (size_t c = 0; c < m; ++c) {
        std::fill(x.begin(), x.end(), cd(0.0, 0.0));
        x[c] = 1.0;
        for (size_t q = 0; q < m; ++q)
            if (piv[q] != q) std::swap(x[q], x[piv[q]]);
        for (size_t r = 0; r < m; ++r)
            for (size_t q = 0; q < r; ++q) x[r] -= A[r * m + q] * x[q];
        for (size_t r = m; r-- > 0;) {
            for (size_t q = r + 1; q < m; ++q) x[r] -= A[r * m + q] * x[q];
            x[r] /= A[r * m + r];
        }
        for (size_t r = 0; r < m; ++r) out[c * m + r] = x[r];
    }
    return true;
}

// ---------------------------------------------------------------------------
// device memory: one allocation per grid, carved into 256-byte aligned parts
// ---------------------------------------------------------------------------
struct Carver {
    size_t off = 0;
    char  *base = nullptr;
    void  *take(size_t bytes) {
        off = (off + 255) & ~size_t(255);
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

// Ray grid over the finest level (Section 6.1 ray correction): returns the
// number of ray unknowns 8 (nr + 2)^2, or 0 when ray_n is 0; -1 when n and
// ray_n do not fit (ray_n <= 7, n + 1 a multiple of ray_n + 1 with cells of
// at least 8 fine intervals, a multiple of 8).
static int ray_geometry(int n, int ray_n, RayGeo &R) {
    if (ray_n == 0) return 0;
    if (ray_n < 1 || ray_n > 7 || (n + 1) % (ray_n + 1) != 0) return -1;
    R.N = n + 1;
    R.M = n + 2;
    R.nr = ray_n;
    R.Mr = ray_n + 2;
    R.Nr = ray_n + 1;
    R.c = (n + 1) / (ray_n + 1);
    if (R.c < 8 || R.c % 8 != 0) return -1;
    R.P = (R.c % 16 == 0) ? 16 : 8;
    R.np = R.Nr * R.c / R.P + 1;
    return 8 * R.Mr * R.Mr;
}

// Lay out (or size, when c.base is null) every device buffer of the grid.
static void layout(hmg_grid *g, Carver &c) {
    for (int l = 0; l < g->nlev; ++l) {
        Level &L = g->lev[l];
        size_t m = (size_t)L.geo.M * L.geo.M;
        L.k = c.take(m * (L.prec == P64 ? 8 : 4));
        // a row table on every level, so that the layout depends on n and
        // the options only (a request server reuses the memory of a grid
        // for the next problem of the same size, whose plan may differ)
        L.ktab = (double *)c.take(m * 16);
    }
    g->k0 = (double *)c.take((size_t)g->lev[0].geo.M * g->lev[0].geo.M * 8);
    int mc = g->lev[g->nlev - 1].geo.M;
    g->ainv_t = (double *)c.take((size_t)mc * mc * (size_t)mc * mc * 16);
    g->bop = nullptr;
    g->bop_m = 0;
    if (g->lb >= 0 && g->opts.bottom_dense) {
        g->bop_m = g->lev[g->lb].geo.M * g->lev[g->lb].geo.M;
        g->bop = (double *)c.take((size_t)g->bop_m * g->bop_m * 16);
    }
    const size_t K = (size_t)g->ray_K;
    if (K) {
        g->ray_ex = c.take((size_t)8 * g->ray.M * 16);
        g->ray_ey = c.take((size_t)8 * g->ray.M * 16);
        g->ray_Ainv = (double *)c.take(K * K * 16);
    }
    size_t m0 = (size_t)g->lev[0].geo.M * g->lev[0].geo.M;
    int nb = krylov_nblocks(g->lev[0].geo);
    for (int s = 0; s < g->nrhs; ++s) {
        Slot &S = g->slot[s];
        for (int l = 0; l < g->nlev; ++l) {
            const Level &L = g->lev[l];
            size_t m = (size_t)L.geo.M * L.geo.M;
            // the first complex-float level below double levels takes its
            // right-hand side and returns its result in double
            size_t csz = (L.prec == P64 || L.io64) ? 16 : 8;
            S.f[l] = c.take(m * csz);
            S.u[l] = c.take(m * csz);
            S.u2[l] = c.take(m * csz);
        }
        Krylov &K = S.K;
        double **vecs[] = {&K.b, &K.x, &K.r, &K.rh, &K.p, &K.v, &K.s, &K.t, &K.ph, &K.sh};
        for (double **v : vecs) *v = (double *)c.take(m0 * 16);
        K.nblocks = nb;
        // room for the partial sums of the Krylov kernels and of the fused
        // finest up kernel, whichever launches more blocks
        K.pcap = std::max(nb, gs_up_mv_blocks(g->lev[0].geo));
        K.partials = (double *)c.take((size_t)3 * K.pcap * 8);
        S.hist_cap = 0;
        K.hist = nullptr;
        K.st = (KState *)c.take(sizeof(KState));
        if (g->ray_K) {
            S.ray_part = (double *)c.take((size_t)g->ray.np * g->ray.np * 64 * 8);
            S.ray_b = c.take((size_t)g->ray_K * 16);
            S.ray_a = c.take((size_t)g->ray_K * 16);
        }
    }
}

// Kernel schedule per level.  The bottom solver takes the deepest levels
// whose fields (u on every level, f below its first level) fit in the LDS of
// one workgroup; above it, Gauss-Seidel levels with one pre- and one post-
// sweep use the fused down/up kernels and Kaczmarz levels the tiled kernel.
// First level of the bottom solver (-1: none); depends on the level sizes
// and the options only.  The bottom solver keeps u, f and k of each of its
// levels in LDS and is used for levels with n <= 31.
static bool one_pass(const hmg_grid *g) {
    // the lexicographic sweeps exist only as separate kernels
    return g->opts.one_pass_kernels || g->opts.relax_order == HMG_ORDER_LEX;
}

static int find_bottom(const hmg_grid *g) {
    if (one_pass(g)) return -1;
    for (int l = 0; l < g->nlev; ++l) {
        if (g->nlev - l > BOT_MAXL || g->lev[l].geo.n > 31) continue;
        int cs = 0, rs = 0;
        for (int q = l; q < g->nlev; ++q) {
            int M = g->lev[q].geo.M, m = M * M;
            cs += (M + 2) * (M + 2) + m;   // u with a ring of zero cells, f
            rs += 2 * m;                   // k and a reciprocal per node
        }
        if (cs <= bottom_complex_slots() && rs <= bottom_real_slots()) return l;
    }
    return -1;
}

// The configuration whose RESID form ends the pre-smoothing of a level run
// with cfg: cfg itself, or else one with the same sweeps per launch (the
// default first), whose sweeps give the same values as cfg's, so that the
// residual is always restricted from the iterate before its last rounding
// to the level's storage; -1 if there is none.
static int kacz_resid_config(int cfg) {
    if (kacz_cfg_resid(cfg)) return cfg;
    const int sw = kKaczCfgs[cfg].sweeps;
    if (kKaczCfgs[KACZ_DEFAULT].sweeps == sw && kacz_cfg_resid(KACZ_DEFAULT)) return KACZ_DEFAULT;
    for (int c = 0; c < KACZ_NCFG; ++c)
        if (kKaczCfgs[c].sweeps == sw && kacz_cfg_resid(c)) return c;
    return -1;
}

static void plan_paths(hmg_grid *g) {
    for (int l = 0; l < g->nlev; ++l) {
        g->lev[l].mode = LM_SIMPLE;
        g->lev[l].kacz_cfg = 0;
    }
    g->lb = find_bottom(g);
    if (one_pass(g)) return;
    int top = (g->lb < 0) ? g->nlev - 1 : g->lb;
    for (int l = 0; l < top; ++l) {
        const hmg_plan &pl = g->plan;
        if (pl.smoother[l] == HMG_SM_GS && pl.pre[l] == 1 && pl.post[l] == 1) {
            g->lev[l].mode = LM_GS_FUSED;
        } else if (pl.smoother[l] == HMG_SM_KACZ) {
            g->lev[l].mode = LM_KACZ_TILED;
            // default before tuning: the LDS-staged 16 x 8 tile with 2
            // sweeps per launch (1024 threads) if 2 divides both sweep
            // counts, else one sweep per launch on 16 x 16 tiles
            int best = (pl.pre[l] % 2 == 0 && pl.post[l] % 2 == 0) ? KACZ_DEFAULT : 5;
            g->lev[l].kacz_cfg = best;
        }
    }
}

// Storage precision per level.  FP64 grids keep every level in double.
// MIXED grids keep the finest t = min(fp64_levels, levels above the bottom
// solver) levels in double and the rest in complex float; level t then
// takes its right-hand side and returns its correction in double, which the
// fused Gauss-Seidel kernels and the bottom solver do (the other schedules
// are rejected).
static hmg_status assign_precision(hmg_grid *g) {
    const int top = (g->lb < 0) ? g->nlev : g->lb;
    const int t = (g->prec == P64) ? g->nlev : std::min(g->opts.fp64_levels, top);
    for (int l = 0; l < g->nlev; ++l) {
        g->lev[l].prec = (l < t) ? P64 : g->prec;
        g->lev[l].io64 = (g->prec == P32 && t > 0 && l == t);
    }
    if (g->prec == P32 && t > 0 && t < g->nlev && t != g->lb && g->lev[t].mode != LM_GS_FUSED)
        return hmg_fail(HMG_ERR_INVALID,
                        "fp64_levels = %d: the first complex-float level (n = %d) must be a Gauss-Seidel level "
                        "of the fused schedule or the first bottom level", g->opts.fp64_levels, g->lev[t].geo.n);
    return HMG_OK;
}

static void bottom_desc(hmg_grid *g) {
    if (g->lb < 0) return;
    BottomDesc &d = g->bottom;
    d.nlev = g->nlev - g->lb;
    d.ainv_t = g->ainv_t;
    int off = 0;
    for (int q = 0; q < d.nlev; ++q) {
        int l = g->lb + q;
        BottomLevelDesc &D = d.L[q];
        D.n = g->lev[l].geo.n;
        D.H = g->lev[l].geo.H;
        D.sa = g->plan.sigma_relax[l];
        D.sb = g->plan.sigma_resid[l];
        D.k = g->lev[l].k;
        D.sm = (g->plan.smoother[l] == HMG_SM_KACZ) ? HMG_SM_KACZ_DEV : HMG_SM_GS_DEV;
        D.pre = g->plan.pre[l];
        D.post = g->plan.post[l];
        D.uoff = off;
        off += (D.n + 4) * (D.n + 4);   // u is stored with a ring of zero cells
    }
    for (int q = 0; q < d.nlev; ++q) {
        BottomLevelDesc &D = d.L[q];
        D.foff = off;
        off += (D.n + 2) * (D.n + 2);
    }
    int koff = 0;
    for (int q = 0; q < d.nlev; ++q) {
        BottomLevelDesc &D = d.L[q];
        D.koff = koff;
        koff += 2 * (D.n + 2) * (D.n + 2);   // k, then the reciprocals
    }
}

// ---------------------------------------------------------------------------
// Tile-configuration tuner for the tiled Kaczmarz kernel: every feasible
// configuration runs one relaxation leg (pre sweeps, ping-ponging between the
// level's two buffers) on the level's own shape; the fastest is kept.  The
// choice is cached per (device, n, precision, sweep counts) for the process.
// ---------------------------------------------------------------------------
#include <map>
#include <mutex>
#include <tuple>

static std::mutex g_tune_mu;
// (device, n, precision, pre, post) -> (configuration, level mode)
static std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> g_tune_cache;

static hmg_status tune_kacz_level(hmg_grid *g, int l) {
    const hmg_plan &pl = g->plan;
    auto key = std::make_tuple(g->ctx->device, g->lev[l].geo.n, (int)g->lev[l].prec, pl.pre[l], pl.post[l]);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            g->lev[l].kacz_cfg = it->second.first;
            g->lev[l].mode = it->second.second;
            return HMG_OK;
        }
    }
    // On complex-float levels the sweeps per launch decide where the iterate
    // is rounded to float, so the candidates keep the default's count, and
    // the pre-smoothing always ends with a fused residual (kacz_resid_config),
    // which restricts the iterate before its rounding; tile shape and size
    // change no value (each node sees the same row updates in the same
    // order), so the results do not depend on timing.
    const bool float_level = g->lev[l].prec == P32;
    const int sw_default = kKaczCfgs[g->lev[l].kacz_cfg].sweeps;
    std::vector<int> cand;
    for (int cfg = 0; cfg < KACZ_NCFG; ++cfg) {
        int sw = kKaczCfgs[cfg].sweeps;
        if (float_level && (sw != sw_default || kacz_resid_config(cfg) < 0)) continue;
        if (kacz_cfg_fits(g->lev[l].prec, cfg) && pl.pre[l] % sw == 0 && pl.post[l] % sw == 0) cand.push_back(cfg);
    }
    if (cand.size() > 1 && pl.pre[l] > 0) {
        const Level &L = g->lev[l];
        Slot &S = g->slot[0];
        const Level &Lc = g->lev[l + 1];
        size_t bytes = (size_t)L.geo.M * L.geo.M * (L.prec == P64 ? 16 : 8);
        size_t cbytes = (size_t)Lc.geo.M * Lc.geo.M * ((Lc.prec == P64 || Lc.io64) ? 16 : 8);
        HIPCHK(hipMemsetAsync(S.f[l], 0, bytes, g->stream));
        HIPCHK(hipMemsetAsync(S.u[l], 0, bytes, g->stream));
        HIPCHK(hipMemsetAsync(S.u2[l], 0, bytes, g->stream));
        HIPCHK(hipMemsetAsync(S.u[l + 1], 0, cbytes, g->stream));
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        float best_ms = 1e30f;
        int best = g->lev[l].kacz_cfg;
        for (int cfg : cand) {
            int sw = kKaczCfgs[cfg].sweeps;
            // the level's two legs as the V-cycle runs them: pre sweeps from
            // zero, post sweeps from u + P e
            auto legs = [&]() {
                const void *cur = nullptr;
                void *bufs[2] = {S.u[l], S.u2[l]};
                int w = 0;
                const int rcfg = kacz_resid_config(cfg);
                for (int q = 0; q < pl.pre[l]; q += sw) {
                    if (rcfg >= 0 && q + sw >= pl.pre[l])
                        launch_kacz_tb_resid(L.prec, rcfg, g->stream, L.geo, L.k, L.ktab, pl.sigma_relax[l],
                                             pl.sigma_resid[l], S.f[l], cur, bufs[w], S.f[l + 1], nullptr);
                    else
                        launch_kacz_tb(L.prec, cfg, g->stream, L.geo, L.k, L.ktab, pl.sigma_relax[l], S.f[l],
                                       cur, nullptr, bufs[w], nullptr);
                    cur = bufs[w];
                    w ^= 1;
                }
                // without a fused residual the separate residual and
                // restriction kernel runs, as in the V-cycle
                if (rcfg < 0 && cur)
                    launch_residual_fw(L.prec, g->stream, L.geo, L.k, pl.sigma_resid[l], S.f[l], cur, S.f[l + 1],
                                       nullptr);
                for (int q = 0; q < pl.post[l] && cur; q += sw) {
                    launch_kacz_tb(L.prec, cfg, g->stream, L.geo, L.k, L.ktab, pl.sigma_relax[l], S.f[l], cur,
                                   q == 0 ? S.u[l + 1] : nullptr, bufs[w], nullptr);
                    cur = bufs[w];
                    w ^= 1;
                }
            };
            // timed as a graph replay, the way the solver launches them
            hipGraph_t gr = nullptr;
            hipGraphExec_t ge = nullptr;
            HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
            for (int r = 0; r < 4; ++r) legs();
            HIPCHK(hipStreamEndCapture(g->stream, &gr));
            hipError_t ie = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                (void)hipGraphDestroy(gr);
                return hmg_fail(HMG_ERR_DEVICE, "tuner graph: %s", hipGetErrorString(ie));
            }
            float ms = 1e30f;
            hipError_t le = hipGraphLaunch(ge, g->stream);   // warm-up
            for (int r = 0; r < 3 && le == hipSuccess; ++r) {
                le = hipEventRecord(e0, g->stream);
                if (le == hipSuccess) le = hipGraphLaunch(ge, g->stream);
                if (le == hipSuccess) le = hipEventRecord(e1, g->stream);
                if (le == hipSuccess) le = hipEventSynchronize(e1);
                float t = 0.f;
                if (le == hipSuccess) le = hipEventElapsedTime(&t, e0, e1);
                if (le == hipSuccess) ms = std::min(ms, t);
            }
            (void)hipGraphExecDestroy(ge);
            (void)hipGraphDestroy(gr);
            if (le != hipSuccess) return hmg_fail(HMG_ERR_DEVICE, "tuner: %s", hipGetErrorString(le));
            if (std::getenv("HMG_TUNE_LOG"))
                std::fprintf(stderr, "hmg tune: n=%d config %d (tile %d, %d sweeps, %d threads): %.4f ms\n",
                             L.geo.n, cfg, kKaczCfgs[cfg].ts, sw, kKaczCfgs[cfg].threads, ms);
            // the default keeps its place unless another configuration is
            // clearly faster (runs then agree on the choice)
            if (cfg == g->lev[l].kacz_cfg) ms *= 0.95f;
            if (ms < best_ms) {
                best_ms = ms;
                best = cfg;
            }
        }
        // a level small enough for one workgroup may run whole (no halo
        // work, but one CU): same two legs, kept only if faster
        // (with several right-hand sides the tiles are kept: only they run
        // every right-hand side in one launch)
        bool whole = false;
        if (kacz_level_fits(L.geo) && !float_level && g->nrhs == 1) {
            auto legs = [&]() {
                launch_kacz_level(L.prec, g->stream, L.geo, L.k, L.ktab, pl.sigma_relax[l], pl.sigma_resid[l],
                                  pl.pre[l], S.f[l], nullptr, nullptr, S.u[l], S.f[l + 1], nullptr);
                launch_kacz_level(L.prec, g->stream, L.geo, L.k, L.ktab, pl.sigma_relax[l], 0.0, pl.post[l],
                                  S.f[l], S.u[l], S.u[l + 1], S.u2[l], nullptr, nullptr);
            };
            hipGraph_t gr = nullptr;
            hipGraphExec_t ge = nullptr;
            HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
            for (int r = 0; r < 4; ++r) legs();
            HIPCHK(hipStreamEndCapture(g->stream, &gr));
            hipError_t le = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
            float ms = 1e30f;
            if (le == hipSuccess) le = hipGraphLaunch(ge, g->stream);
            for (int r = 0; r < 3 && le == hipSuccess; ++r) {
                le = hipEventRecord(e0, g->stream);
                if (le == hipSuccess) le = hipGraphLaunch(ge, g->stream);
                if (le == hipSuccess) le = hipEventRecord(e1, g->stream);
                if (le == hipSuccess) le = hipEventSynchronize(e1);
                float t = 0.f;
                if (le == hipSuccess) le = hipEventElapsedTime(&t, e0, e1);
                if (le == hipSuccess) ms = std::min(ms, t);
            }
            if (ge) (void)hipGraphExecDestroy(ge);
            (void)hipGraphDestroy(gr);
            if (le != hipSuccess) return hmg_fail(HMG_ERR_DEVICE, "tuner: %s", hipGetErrorString(le));
            if (std::getenv("HMG_TUNE_LOG"))
                std::fprintf(stderr, "hmg tune: n=%d whole level in one workgroup: %.4f ms\n", L.geo.n, ms);
            whole = ms < 0.95f * best_ms;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        g->lev[l].kacz_cfg = best;
        if (whole) g->lev[l].mode = LM_KACZ_LEVEL;
    } else if (cand.size() == 1) {
        g->lev[l].kacz_cfg = cand[0];
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = std::make_pair(g->lev[l].kacz_cfg, g->lev[l].mode);
    return HMG_OK;
}

// The byte distance between the buffers of consecutive slots when it is the
// same for every per-slot buffer (the carver lays the slots out alike), else 0.
static long slot_stride(const hmg_grid *g) {
    if (g->nrhs < 2) return 0;
    auto ptrs = [&](const Slot &S) {
        std::vector<const char *> v;
        for (int l = 0; l < g->nlev; ++l) {
            v.push_back((const char *)S.f[l]);
            v.push_back((const char *)S.u[l]);
            v.push_back((const char *)S.u2[l]);
        }
        const Krylov &K = S.K;
        const void *kv[] = {K.b, K.x, K.r, K.rh, K.p, K.v, K.s, K.t, K.ph, K.sh, K.partials, K.st,
                            S.ray_part, S.ray_b, S.ray_a};
        for (const void *q : kv) v.push_back((const char *)q);
        return v;
    };
    const std::vector<const char *> p0 = ptrs(g->slot[0]), p1 = ptrs(g->slot[1]);
    const long zs = (long)(p1[0] - p0[0]);
    for (int r = 1; r < g->nrhs; ++r) {
        const std::vector<const char *> pr = ptrs(g->slot[r]);
        for (size_t q = 0; q < p0.size(); ++q) {
            if (!p0[q] || !pr[q]) {   // a part the grid does not use (the ray fields): absent in every slot
                if (p0[q] != pr[q]) return 0;
                continue;
            }
            if (pr[q] - p0[q] != (long)r * zs) return 0;
        }
    }
    return zs;
}

bool grid_batchable(const hmg_grid *g) {
    if (g->nrhs < 2 || g->zs == 0 || one_pass(g) || g->lb < 0 || !g->bop) return false;
    for (int l = 0; l < g->lb; ++l)
        if (g->lev[l].mode != LM_GS_FUSED && g->lev[l].mode != LM_KACZ_TILED) return false;
    return true;
}

static hmg_status tune_levels(hmg_grid *g) {
    MarkRange mark_("hmg tuner");
    if (!g->opts.autotune) return HMG_OK;
    for (int l = 0; l < g->nlev; ++l)
        if (g->lev[l].mode == LM_KACZ_TILED) {
            hmg_status st = tune_kacz_level(g, l);
            if (st) return st;
        }
    return HMG_OK;
}

extern "C" int hmg_grid_kacz_config(const hmg_grid *g, int level) {
    if (!g || level < 0 || level >= g->nlev) return -1;
    if (g->lev[level].mode == LM_KACZ_LEVEL) return KACZ_NCFG;
    if (g->lev[level].mode != LM_KACZ_TILED) return -1;
    return g->lev[level].kacz_cfg;
}

// Device bytes of a grid of size n with options o (sizes do not depend on k).
size_t estimate_footprint(int n, const hmg_opts &o) {
    hmg_grid g;
    g.nrhs = 1;
    g.prec = (o.precision == HMG_MIXED) ? P32 : P64;
    int nl = n, l = 0;
    double H = 1.0;
    for (;; ++l) {
        g.lev[l].geo = make_geo(nl, H);
        if (nl <= o.coarsest_n || l == HMG_MAX_LEVELS - 1) break;
        nl = (nl - 1) / 2;
        H *= 2.0;
    }
    g.nlev = l + 1;
    g.opts = o;
    g.ray_K = std::max(0, ray_geometry(n, o.ray_n, g.ray));
    g.lb = find_bottom(&g);
    {
        const int top = (g.lb < 0) ? g.nlev : g.lb;
        const int t = (g.prec == P64) ? g.nlev : std::min(o.fp64_levels, top);
        for (int q = 0; q < g.nlev; ++q) {
            g.lev[q].prec = (q < t) ? P64 : g.prec;
            g.lev[q].io64 = (g.prec == P32 && t > 0 && q == t);
        }
    }
    // the Kaczmarz levels depend on k: count a row table on every level
    // below the finest
    for (int q = 1; q < g.nlev; ++q) g.lev[q].mode = LM_KACZ_TILED;
    g.slot.resize(1);
    Carver c;
    layout(&g, c);
    return c.off + 256;
}

// The ray correction's tables and Galerkin matrix (Section 6.1): the wave
// factors exp(i kr cos(theta_d) x) and exp(i kr sin(theta_d) y) per
// direction theta_d = (d + 1) pi / 4 and fine line, kr the mean of k; A =
// P^H L P built on the device column by column with the correction's own
// kernels (prolong a unit vector, apply L, restrict), inverted on the host
// (LU with partial pivoting) and stored row-major for the solve kernel.
static hmg_status ray_setup(hmg_grid *g) {
    const RayGeo &R = g->ray;
    const int K = g->ray_K, M = R.M;
    const size_t m0 = (size_t)M * M;
    std::vector<double> k0(m0);
    HIPCHK(hipMemcpy(k0.data(), g->k0, m0 * 8, hipMemcpyDeviceToHost));
    double kr = 0.0;
    for (double v : k0) kr += v;
    kr /= (double)m0;
    std::vector<cd> ex((size_t)8 * M), ey((size_t)8 * M);
    for (int d = 0; d < 8; ++d) {
        const double th = (d + 1) * M_PI / 4.0, cx = std::cos(th), sy = std::sin(th);
        for (int i = 0; i < M; ++i) {
            const double x = i * g->h;
            ex[(size_t)d * M + i] = std::exp(cd(0.0, kr * cx * x));
            ey[(size_t)d * M + i] = std::exp(cd(0.0, kr * sy * x));
        }
    }
    HIPCHK(hipMemcpy(g->ray_ex, ex.data(), ex.size() * 16, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->ray_ey, ey.data(), ey.size() * 16, hipMemcpyHostToDevice));
    Slot &S = g->slot[0];
    for (int col = 0; col < K; ++col)
        launch_ray_column(g->stream, R, g->lev[0].geo.H, g->k0, g->ray_ex, g->ray_ey, S.K.t, S.ray_part, S.ray_b,
                          S.ray_a, g->ray_Ainv, col);
    HIPCHK(hipGetLastError());
    std::vector<cd> A((size_t)K * K), inv;
    HIPCHK(hipMemcpyAsync(A.data(), g->ray_Ainv, A.size() * 16, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    if (!invert_dense((size_t)K, A, inv)) return hmg_fail(HMG_ERR_INVALID, "the ray Galerkin matrix is singular");
    // invert_dense returns the inverse column-major; the solve kernel reads rows
    for (int r = 0; r < K; ++r)
        for (int c = 0; c < K; ++c) A[(size_t)r * K + c] = inv[(size_t)c * K + r];
    HIPCHK(hipMemcpy(g->ray_Ainv, A.data(), A.size() * 16, hipMemcpyHostToDevice));
    return HMG_OK;
}

extern "C" hmg_status hmg_ray_correct_dev(hmg_grid *g, const void *d_r, void *d_z, void *stream) {
    if (!g || !d_r || !d_z) return hmg_fail(HMG_ERR_INVALID, "null argument");
    if (!g->ray_K) return hmg_fail(HMG_ERR_INVALID, "the grid has no ray correction (ray_n = 0)");
    if (d_r == d_z) return hmg_fail(HMG_ERR_INVALID, "r and z must not alias");
    HIPCHK(hipSetDevice(g->ctx->device));
    Slot &S = g->slot[0];
    launch_ray_correct(stream ? (hipStream_t)stream : g->stream, g->ray, g->lev[0].geo.H, g->k0, g->ray_ex,
                       g->ray_ey, g->ray_Ainv, d_r, d_z, S.ray_part, S.ray_b, S.ray_a, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

// Checks of the problem and options (the conventions of hmg_grid_create).
static hmg_status check_problem(const hmg_opts &o, int n, double h, const double *k, const hmg_c64 *f, int nrhs) {
    if (o.coarsest_n < 1 || o.coarsest_n > 31)
        return hmg_fail(HMG_ERR_INVALID, "coarsest_n must be in [1, 31], got %d", o.coarsest_n);
    if (!valid_hierarchy(n, o.coarsest_n))
        return hmg_fail(HMG_ERR_INVALID,
                        "n must be >= coarsest_n (%d) and halve exactly (n + 1 even) down to it, got %d",
                        o.coarsest_n, n);
    if (!(h > 0.0) || !std::isfinite(h)) return hmg_fail(HMG_ERR_INVALID, "h must be finite and > 0");
    if (!k) return hmg_fail(HMG_ERR_INVALID, "k is required");
    if (nrhs < 1 || nrhs > 4096) return hmg_fail(HMG_ERR_INVALID, "nrhs must be in [1, 4096]");
    if (o.variant < 0 || o.variant > 2) return hmg_fail(HMG_ERR_INVALID, "bad variant");
    if (o.precision != HMG_FP64 && o.precision != HMG_MIXED) return hmg_fail(HMG_ERR_INVALID, "bad precision");
    if (o.relax_order != HMG_ORDER_COLOUR && o.relax_order != HMG_ORDER_LEX)
        return hmg_fail(HMG_ERR_INVALID, "bad relax_order");
    if (o.breakdown_at < 0) return hmg_fail(HMG_ERR_INVALID, "breakdown_at must be >= 0");
    if (o.true_res_every < 0) return hmg_fail(HMG_ERR_INVALID, "true_res_every must be >= 0");
    if (o.nan_at < 0) return hmg_fail(HMG_ERR_INVALID, "nan_at must be >= 0");
    if (o.fp64_levels < 0) return hmg_fail(HMG_ERR_INVALID, "fp64_levels must be >= 0");
    if (o.hyb_mid != 0 && o.hyb_mid != 1) return hmg_fail(HMG_ERR_INVALID, "hyb_mid must be 0 or 1");
    {
        RayGeo rg{};
        if (ray_geometry(n, o.ray_n, rg) < 0)
            return hmg_fail(HMG_ERR_INVALID,
                            "ray_n = %d: needs 1 <= ray_n <= 7 with n + 1 = %d a multiple of ray_n + 1 and ray cells "
                            "of a multiple of 8 fine intervals", o.ray_n, n + 1);
    }
    if (o.fp64_levels > 0 && o.precision == HMG_MIXED && (o.one_pass_kernels || o.relax_order == HMG_ORDER_LEX))
        return hmg_fail(HMG_ERR_INVALID, "fp64_levels needs the fused schedule with coloured sweeps");
    if (!std::isfinite(o.beta) || o.nu_pre < 0 || o.nu_post < 0 || o.kacz_pre < 0 || o.kacz_post < 0 ||
        o.nu_pre > 64 || o.nu_post > 64 || o.kacz_pre > 64 || o.kacz_post > 64)
        return hmg_fail(HMG_ERR_INVALID, "bad sweep counts or beta");
    size_t m0 = (size_t)(n + 2) * (n + 2);
    for (size_t q = 0; q < m0; ++q)
        if (!(k[q] > 0.0) || !std::isfinite(k[q])) return hmg_fail(HMG_ERR_INVALID, "k must be finite and > 0");
    if (f)
        for (size_t q = 0; q < m0 * (size_t)nrhs; ++q)
            if (!std::isfinite(f[q].re) || !std::isfinite(f[q].im))
                return hmg_fail(HMG_ERR_INVALID, "f must be finite");
    return HMG_OK;
}

// The host side of a problem on a grid whose n, nrhs and options are set:
// the hierarchy of k (injection), the level plan (Section 5), the level
// schedule and precisions, and the coarsest inverse.
static hmg_status plan_problem(hmg_grid *g, double h, const double *k, std::vector<std::vector<double>> &kl,
                               std::vector<cd> &inv) {
    const hmg_opts &o = g->opts;
    const int n = g->n;
    const size_t m0 = (size_t)(n + 2) * (n + 2);
    g->h = h;
    g->plan = hmg_plan{};
    kl.clear();
    kl.emplace_back(k, k + m0);
    int nl = n;
    double H = h;
    for (int l = 0;; ++l) {
        g->plan.n[l] = nl;
        g->plan.H[l] = H;
        if (nl <= o.coarsest_n || l == HMG_MAX_LEVELS - 1) {
            g->nlev = l + 1;
            break;
        }
        int nc = (nl - 1) / 2, Mc = nc + 2, M = nl + 2;
        std::vector<double> kc((size_t)Mc * Mc);
        for (int J = 0; J < Mc; ++J)
            for (int I = 0; I < Mc; ++I) kc[(size_t)J * Mc + I] = kl.back()[(size_t)(2 * J) * M + 2 * I];
        kl.push_back(std::move(kc));
        nl = nc;
        H *= 2.0;
    }
    g->plan.nlev = g->nlev;
    for (int l = 0; l < g->nlev; ++l) {
        classify_level(o, g->plan, l, l == g->nlev - 1, kl[l].data());
        g->lev[l].geo = make_geo(g->plan.n[l], g->plan.H[l]);
    }
    int lc = g->nlev - 1;
    std::vector<cd> A;
    dense_operator(g->plan.n[lc], g->plan.H[lc], kl[lc].data(), g->plan.sigma_relax[lc], A);
    size_t mc = (size_t)(g->plan.n[lc] + 2) * (g->plan.n[lc] + 2);
    if (!invert_dense(mc, A, inv)) return hmg_fail(HMG_ERR_INVALID, "coarsest operator is singular");
    plan_paths(g);
    g->ray_K = ray_geometry(n, o.ray_n, g->ray);
    return assign_precision(g);
}

// The device side of a problem on an allocated grid: k on every level, the
// coarsest inverse, the right-hand sides, the Kaczmarz row tables, the
// bottom-cycle matrix, the tuned tile configurations and the ray correction.
static hmg_status load_problem(hmg_grid *g, const std::vector<std::vector<double>> &kl, const std::vector<cd> &inv,
                               const hmg_c64 *f) {
    bottom_desc(g);
    hmg_status st = grid_upload(g, kl, inv, f);
    if (st == HMG_OK) {
        for (int l = 0; l < g->nlev; ++l)
            if (g->lev[l].mode == LM_KACZ_TILED || g->lev[l].mode == LM_KACZ_LEVEL)
                launch_kacz_table(g->lev[l].prec, g->stream, g->lev[l].geo, g->lev[l].k, g->plan.sigma_relax[l],
                                  g->lev[l].ktab);
        hipError_t le = hipGetLastError();
        if (le != hipSuccess) st = hmg_fail(HMG_ERR_DEVICE, "Kaczmarz tables: %s", hipGetErrorString(le));
    }
    if (st == HMG_OK && g->bop) {
        // the bottom cycle on every unit vector: its matrix, column by column
        launch_bottom_basis(g->lev[g->lb].prec, g->stream, g->bottom, g->bop);
        hipError_t le = hipGetLastError();
        if (le == hipSuccess) le = hipStreamSynchronize(g->stream);
        if (le != hipSuccess) st = hmg_fail(HMG_ERR_DEVICE, "bottom matrix: %s", hipGetErrorString(le));
    }
    if (st == HMG_OK) st = tune_levels(g);
    if (st == HMG_OK && g->ray_K) st = ray_setup(g);
    return st;
}

extern "C" hmg_status hmg_grid_create(hmg_ctx *ctx, int n, double h, const double *k, const hmg_c64 *f, int nrhs,
                                      const hmg_opts *opts, hmg_grid **out) {
    MarkRange mark_("hmg_grid_create");
    if (!ctx || !out) return hmg_fail(HMG_ERR_INVALID, "null context or output handle");
    *out = nullptr;
    hmg_opts o;
    if (opts) o = *opts;
    else hmg_opts_default(&o);
    hmg_status st = check_problem(o, n, h, k, f, nrhs);
    if (st) return st;

    hmg_grid *g = new hmg_grid();
    g->ctx = ctx;
    g->opts = o;
    g->n = n;
    g->nrhs = nrhs;
    g->prec = (o.precision == HMG_MIXED) ? P32 : P64;
    std::vector<std::vector<double>> kl;
    std::vector<cd> inv;
    st = plan_problem(g, h, k, kl, inv);
    if (st) {
        delete g;
        return st;
    }
    g->slot.resize(nrhs);
    Carver sizer;
    layout(g, sizer);
    g->bytes = sizer.off + 256;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMalloc((void **)&g->mem, g->bytes);
    if (e != hipSuccess) {
        delete g;
        return hmg_fail(HMG_ERR_NOMEM, "hipMalloc of %zu bytes failed: %s", sizer.off, hipGetErrorString(e));
    }
    Carver c;
    c.base = g->mem;
    layout(g, c);
    g->zs = slot_stride(g);
    st = grid_init_device(g);
    if (st == HMG_OK) st = load_problem(g, kl, inv, f);
    if (st != HMG_OK) {
        hmg_grid_destroy(g);
        return st;
    }
    *out = g;
    return HMG_OK;
}

// Whether grid g can take a problem of size n with options o in place.
bool grid_reusable(const hmg_grid *g, int n, int nrhs, const hmg_opts &o) {
    return g && g->n == n && g->nrhs == nrhs && std::memcmp(&g->opts, &o, sizeof o) == 0;
}

// Put a new problem (spacing h, wavenumber k, right-hand sides f) on a grid
// of the same size and options, in its memory: no device allocation (the
// layout depends on n and the options only).  The level plan, tables,
// coarsest inverse and bottom matrix are rebuilt and captured graphs dropped.
hmg_status grid_reload(hmg_grid *g, double h, const double *k, const hmg_c64 *f) {
    MarkRange mark_("hmg grid reload");
    hmg_status st = check_problem(g->opts, g->n, h, k, f, g->nrhs);
    if (st) return st;
    HIPCHK(hipSetDevice(g->ctx->device));
    HIPCHK(hipStreamSynchronize(g->stream));
    for (Slot &S : g->slot) {
        if (S.iter_graph) (void)hipGraphExecDestroy(S.iter_graph);
        S.iter_graph = nullptr;
        S.last_halfsteps = -1;
    }
    if (g->batch_graph) (void)hipGraphExecDestroy(g->batch_graph);
    g->batch_graph = nullptr;
    // the buffers stay where they are: the layout is a function of n and
    // the options (level precisions included), which match
    std::vector<std::vector<double>> kl;
    std::vector<cd> inv;
    st = plan_problem(g, h, k, kl, inv);
    if (st) return st;
    return load_problem(g, kl, inv, f);
}

// Per-grid runtime objects: the stream, pinned status records and events.
hmg_status grid_init_device(hmg_grid *g) {
    HIPCHK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    HIPCHK(hipHostMalloc((void **)&g->host_state, 4 * sizeof(KState), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&g->done_host, (size_t)g->nrhs * sizeof(int), hipHostMallocDefault));
    for (int s = 0; s < g->nrhs; ++s) {
        g->done_host[s] = 0;
        g->slot[s].K.done_host = &g->done_host[s];
    }
    for (int q = 0; q < 4; ++q) HIPCHK(hipEventCreateWithFlags(&g->ev[q], hipEventDisableTiming));
    return HMG_OK;
}

// k of every level in its precision, the FP64 finest k, the coarsest inverse
// and the right-hand sides (zero where f is null).
hmg_status grid_upload(hmg_grid *g, const std::vector<std::vector<double>> &kl, const std::vector<cd> &inv,
                       const hmg_c64 *f) {
    for (int l = 0; l < g->nlev; ++l) {
        size_t m = kl[l].size();
        if (g->lev[l].prec == P64) {
            HIPCHK(hipMemcpy(g->lev[l].k, kl[l].data(), m * 8, hipMemcpyHostToDevice));
        } else {
            std::vector<float> kf(m);
            for (size_t q = 0; q < m; ++q) kf[q] = (float)kl[l][q];
            HIPCHK(hipMemcpy(g->lev[l].k, kf.data(), m * 4, hipMemcpyHostToDevice));
        }
    }
    HIPCHK(hipMemcpy(g->k0, kl[0].data(), kl[0].size() * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->ainv_t, inv.data(), inv.size() * 16, hipMemcpyHostToDevice));
    size_t m0 = kl[0].size();
    for (int s = 0; s < g->nrhs; ++s) {
        if (f) HIPCHK(hipMemcpy(g->slot[s].K.b, f + m0 * s, m0 * 16, hipMemcpyHostToDevice));
        else HIPCHK(hipMemsetAsync(g->slot[s].K.b, 0, m0 * 16, g->stream));
    }
    HIPCHK(hipStreamSynchronize(g->stream));
    return HMG_OK;
}

extern "C" void hmg_grid_destroy(hmg_grid *g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (Slot &S : g->slot)
        if (S.iter_graph) (void)hipGraphExecDestroy(S.iter_graph);
    if (g->hist_all) (void)hipFree(g->hist_all);
    if (g->batch_graph) (void)hipGraphExecDestroy(g->batch_graph);
    if (g->mem) (void)hipFree(g->mem);
    for (int q = 0; q < 4; ++q)
        if (g->ev[q]) (void)hipEventDestroy(g->ev[q]);
    if (g->host_state) (void)hipHostFree(g->host_state);
    if (g->done_host) (void)hipHostFree(g->done_host);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

extern "C" hmg_status hmg_grid_plan(const hmg_grid *g, hmg_plan *plan) {
    if (!g || !plan) return hmg_fail(HMG_ERR_INVALID, "null argument");
    *plan = g->plan;
    return HMG_OK;
}

extern "C" size_t hmg_grid_footprint(const hmg_grid *g) { return g ? g->bytes : 0; }

extern "C" hmg_status hmg_grid_set_rhs(hmg_grid *g, int rhs, const hmg_c64 *f) {
    if (!g || !f || rhs < 0 || rhs >= g->nrhs) return hmg_fail(HMG_ERR_INVALID, "bad argument");
    size_t m0 = (size_t)g->lev[0].geo.M * g->lev[0].geo.M;
    for (size_t q = 0; q < m0; ++q)
        if (!std::isfinite(f[q].re) || !std::isfinite(f[q].im)) return hmg_fail(HMG_ERR_INVALID, "f must be finite");
    HIPCHK(hipSetDevice(g->ctx->device));
    HIPCHK(hipMemcpy(g->slot[rhs].K.b, f, m0 * 16, hipMemcpyHostToDevice));
    return HMG_OK;
}

// ---------------------------------------------------------------------------
// V-cycle schedule (Section 5): zero initial guess on every level,
//   pre-relax (role A) -> residual (role B) + full weighting -> recurse ->
//   bilinear correction -> post-relax (role A); dense solve on the coarsest.
// ---------------------------------------------------------------------------
// `sweeps` sweeps of smoother sm (HMG_SM_GS / HMG_SM_KACZ) in order `order` on
// A_sig u = f, in place; zero_guess: the incoming u counts as zero.
static void sweep(Prec p, int sm, int order, hipStream_t s, const Geo &geo, const void *k, double sig,
                  const void *f, void *u, int sweeps, bool zero_guess, const int *skip) {
    const size_t m = (size_t)geo.M * geo.M;
    if (order == HMG_ORDER_LEX) {
        if (zero_guess) launch_fill_zero(p, s, u, m, skip);
        for (int q = 0; q < sweeps; ++q) launch_lex_sweep(p, sm == HMG_SM_KACZ, s, geo, k, sig, f, u, skip);
    } else if (sm == HMG_SM_GS) {
        if (sweeps == 0 && zero_guess) launch_fill_zero(p, s, u, m, skip);
        for (int q = 0; q < sweeps; ++q) {
            launch_gs_colour(p, s, geo, k, sig, f, u, 0, (zero_guess && q == 0) ? 1 : 0, skip);
            launch_gs_colour(p, s, geo, k, sig, f, u, 1, 0, skip);
        }
    } else {
        if (zero_guess) launch_fill_zero(p, s, u, m, skip);
        for (int q = 0; q < sweeps; ++q)
            for (int c = 0; c < 5; ++c) launch_kacz_colour(p, s, geo, k, sig, f, u, c, skip);
    }
}

static void relax(hmg_grid *g, int l, const void *f, void *u, int sweeps, bool zero_guess, hipStream_t s,
                  const int *skip) {
    const Level &L = g->lev[l];
    sweep(L.prec, g->plan.smoother[l], g->opts.relax_order, s, L.geo, L.k, g->plan.sigma_relax[l], f, u, sweeps,
          zero_guess, skip);
}

static void vcycle_level(hmg_grid *g, Slot &S, int l, const void *f, void *u, hipStream_t s, const int *skip) {
    const Level &L = g->lev[l];
    if (g->plan.smoother[l] == HMG_SM_LU) {
        launch_coarsest(L.prec, s, L.geo.M * L.geo.M, g->ainv_t, f, u, skip);
        return;
    }
    relax(g, l, f, u, g->plan.pre[l], true, s, skip);
    launch_residual_fw(L.prec, s, L.geo, L.k, g->plan.sigma_resid[l], f, u, S.f[l + 1], skip);
    vcycle_level(g, S, l + 1, S.f[l + 1], S.u[l + 1], s, skip);
    launch_prolong_add(L.prec, s, L.geo, S.u[l + 1], u, skip);
    relax(g, l, f, u, g->plan.post[l], false, s, skip);
}

// Fused schedule of levels l.. on right-hand side f.  The result goes to
// `out` when given (else to a level buffer, whose pointer is returned).  f64
// marks the FP64 level-0 input / output of the mixed precision.
static const void *vc_fast(hmg_grid *g, Slot &S, int l, const void *f, bool f64, void *out, hipStream_t s,
                           const int *skip, MvFuse *mv = nullptr, Bz bz = {}) {
    const Level &L = g->lev[l];
    const hmg_plan &pl = g->plan;
    if (l == g->lb) {
        void *dst = out ? out : S.u[l];
        if (g->bop) launch_dense_apply(L.prec, f64, s, g->bop, g->bop_m, f, dst, skip, bz);
        else launch_bottom(L.prec, f64, s, g->bottom, f, dst, skip);   // single right-hand side only
        return dst;
    }
    if (L.mode == LM_GS_FUSED) {
        // The up kernel needs the pre-smoothed iterate u0 (on the black
        // nodes: red values are overwritten unread).  On FP64 levels small
        // enough for their fields to stay in cache (n <= 511) the down kernel
        // stores it there and the up kernel reads it (one dependent phase
        // fewer); on larger levels the extra HBM traffic costs as much as the
        // phase saves, and complex-float levels must not round it: both
        // recompute it from f.
        void *u0 = (L.prec == P64 && L.geo.n <= 511) ? S.u[l] : nullptr;
        launch_gs_down(L.prec, f64, s, L.geo, L.k, pl.sigma_relax[l], pl.sigma_resid[l], f, u0, S.f[l + 1],
                       skip, true, bz);
        const void *e = vc_fast(g, S, l + 1, S.f[l + 1], g->lev[l + 1].io64, nullptr, s, skip, nullptr, bz);
        void *dst = out ? out : S.u2[l];
        // the finest up kernel of an FP64 solve also forms the Krylov product
        // of its result when the caller asks for it
        if (mv && l == 0 && !u0 && !f64 && gs_up_mv_ok(L.prec, L.geo) &&
            gs_up_mv_blocks(L.geo) <= S.K.pcap) {
            launch_gs_up_mv(s, mv->kind, L.geo, L.k, pl.sigma_relax[l], f, e, mv->no_z ? nullptr : dst, mv->out,
                            mv->dot, mv->partials, skip, bz);
            mv->blocks = gs_up_mv_blocks(L.geo);
            mv->fused = true;
            return dst;
        }
        launch_gs_up(L.prec, f64, s, L.geo, L.k, pl.sigma_relax[l], f, u0, e, dst, skip, bz);
        return dst;
    }
    size_t m = (size_t)L.geo.M * L.geo.M;
    if (L.mode == LM_KACZ_LEVEL) {
        // pre-smoothing + restriction, coarser levels, correction + post-smoothing
        double sig = pl.sigma_relax[l];
        launch_kacz_level(L.prec, s, L.geo, L.k, L.ktab, sig, pl.sigma_resid[l], pl.pre[l], f, nullptr, nullptr,
                          S.u[l], S.f[l + 1], skip);
        const void *e = vc_fast(g, S, l + 1, S.f[l + 1], g->lev[l + 1].io64, nullptr, s, skip, nullptr, bz);
        void *dst = out ? out : S.u2[l];
        launch_kacz_level(L.prec, s, L.geo, L.k, L.ktab, sig, 0.0, pl.post[l], f, S.u[l], e, dst, nullptr, skip);
        return dst;
    }
    if (L.mode == LM_KACZ_TILED) {
        int cfg = L.kacz_cfg, sw = kKaczCfgs[cfg].sweeps;
        double sig = pl.sigma_relax[l];
        void *bufs[2] = {S.u[l], S.u2[l]};
        const void *cur = nullptr;
        int w = 0;
        // the last pre-smoothing launch also restricts the residual (in the
        // RESID form of cfg, or of a configuration with cfg's sweeps per
        // launch when cfg's region is too large for it)
        const int rcfg = pl.pre[l] > 0 ? kacz_resid_config(cfg) : -1;
        const bool fuse = rcfg >= 0;
        for (int q = 0; q < pl.pre[l]; q += sw) {
            if (fuse && q + sw >= pl.pre[l])
                launch_kacz_tb_resid(L.prec, rcfg, s, L.geo, L.k, L.ktab, sig, pl.sigma_resid[l], f, cur, bufs[w],
                                     S.f[l + 1], skip, bz);
            else
                launch_kacz_tb(L.prec, cfg, s, L.geo, L.k, L.ktab, sig, f, cur, nullptr, bufs[w], skip, bz);
            cur = bufs[w];
            w ^= 1;
        }
        if (!cur) {
            launch_fill_zero(L.prec, s, bufs[w], m, skip, bz);
            cur = bufs[w];
            w ^= 1;
        }
        if (!fuse) launch_residual_fw(L.prec, s, L.geo, L.k, pl.sigma_resid[l], f, cur, S.f[l + 1], skip, bz);
        const void *e = vc_fast(g, S, l + 1, S.f[l + 1], g->lev[l + 1].io64, nullptr, s, skip, nullptr, bz);
        if (pl.post[l] == 0) {
            launch_prolong_add(L.prec, s, L.geo, e, (void *)cur, skip, bz);
        }
        for (int q = 0; q < pl.post[l]; q += sw) {
            launch_kacz_tb(L.prec, cfg, s, L.geo, L.k, L.ktab, sig, f, cur, q == 0 ? e : nullptr, bufs[w], skip,
                           bz);
            cur = bufs[w];
            w ^= 1;
        }
        if (out) {
            for (int z = 0; z < bz.nz; ++z)
                (void)hipMemcpyAsync((char *)out + z * bz.zs, (const char *)cur + z * bz.zs,
                                     m * (L.prec == P64 ? 16 : 8), hipMemcpyDeviceToDevice, s);
            return out;
        }
        return cur;
    }
    // one-pass kernels, in place
    void *u = out ? out : S.u[l];
    relax(g, l, f, u, pl.pre[l], true, s, skip);
    launch_residual_fw(L.prec, s, L.geo, L.k, pl.sigma_resid[l], f, u, S.f[l + 1], skip);
    const void *e = vc_fast(g, S, l + 1, S.f[l + 1], g->lev[l + 1].io64, nullptr, s, skip);   // single only
    launch_prolong_add(L.prec, s, L.geo, e, u, skip);
    relax(g, l, f, u, pl.post[l], false, s, skip);
    return u;
}

// The conditions under which vc_fast hands level 0's up kernel to
// launch_gs_up_mv for an FP64 solve.
bool vcycle_forms_products(const hmg_grid *g, const Slot &S) {
    const Geo &g0 = g->lev[0].geo;
    return !one_pass(g) && g->lev[0].prec == P64 && g->lb != 0 && g->lev[0].mode == LM_GS_FUSED && g0.n > 511 &&
           gs_up_mv_ok(P64, g0) && gs_up_mv_blocks(g0) <= S.K.pcap;
}

// z = B_V r on FP64 device fields r, z (finest level); batched (bz.nz > 1)
// on the right-hand sides of S and the slots after it.
void enqueue_vcycle(hmg_grid *g, Slot &S, const double *r, double *z, hipStream_t s, const int *skip,
                    MvFuse *mv, Bz bz) {
    if (!one_pass(g)) {
        bool mixed = g->lev[0].prec == P32;
        if (!mixed || g->lb == 0 || g->lev[0].mode == LM_GS_FUSED) {
            vc_fast(g, S, 0, r, mixed, z, s, skip, mv, bz);
        } else {
            size_t m0 = (size_t)g->lev[0].geo.M * g->lev[0].geo.M;
            launch_convert(s, 1, r, S.f[0], m0, skip, bz);
            const void *res = vc_fast(g, S, 0, S.f[0], false, nullptr, s, skip, nullptr, bz);
            launch_convert(s, 0, res, z, m0, skip, bz);
        }
        return;
    }
    if (g->lev[0].prec == P64) {
        vcycle_level(g, S, 0, r, z, s, skip);
    } else {
        size_t m0 = (size_t)g->lev[0].geo.M * g->lev[0].geo.M;
        launch_convert(s, 1, r, S.f[0], m0, skip);
        vcycle_level(g, S, 0, S.f[0], S.u[0], s, skip);
        launch_convert(s, 0, S.u[0], z, m0, skip);
    }
}

static hipStream_t pick_stream(hmg_grid *g, void *stream) { return stream ? (hipStream_t)stream : g->stream; }

extern "C" hmg_status hmg_vcycle_dev(hmg_grid *g, const void *d_r, void *d_z, void *stream) {
    if (!g || !d_r || !d_z) return hmg_fail(HMG_ERR_INVALID, "null argument");
    if (d_r == d_z) return hmg_fail(HMG_ERR_INVALID, "r and z must not alias");
    HIPCHK(hipSetDevice(g->ctx->device));
    hipStream_t s = pick_stream(g, stream);
    enqueue_vcycle(g, g->slot[0], (const double *)d_r, (double *)d_z, s, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_vcycle(hmg_grid *g, const hmg_c64 *r, hmg_c64 *z) {
    if (!g || !r || !z) return hmg_fail(HMG_ERR_INVALID, "null argument");
    HIPCHK(hipSetDevice(g->ctx->device));
    size_t m0 = (size_t)g->lev[0].geo.M * g->lev[0].geo.M;
    Slot &S = g->slot[0];
    HIPCHK(hipMemcpyAsync(S.K.p, r, m0 * 16, hipMemcpyHostToDevice, g->stream));
    enqueue_vcycle(g, S, S.K.p, S.K.ph, g->stream, nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(z, S.K.ph, m0 * 16, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    return HMG_OK;
}

// ---------------------------------------------------------------------------
// single building blocks (parity tests)
// ---------------------------------------------------------------------------
static hmg_status check_level(hmg_grid *g, int level, bool need_coarser) {
    if (!g) return hmg_fail(HMG_ERR_INVALID, "null grid");
    if (level < 0 || level >= g->nlev || (need_coarser && level >= g->nlev - 1))
        return hmg_fail(HMG_ERR_INVALID, "level %d out of range", level);
    HIPCHK(hipSetDevice(g->ctx->device));
    return HMG_OK;
}

extern "C" hmg_status hmg_op_apply_dev(hmg_grid *g, int level, double sigma, const void *d_u, void *d_out,
                                       void *stream) {
    hmg_status st = check_level(g, level, false);
    if (st) return st;
    if (!d_u || !d_out) return hmg_fail(HMG_ERR_INVALID, "null field");
    const Level &L = g->lev[level];
    launch_apply(L.prec, pick_stream(g, stream), L.geo, L.k, sigma, d_u, d_out);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_smooth_dev(hmg_grid *g, int level, int smoother, double sigma, int sweeps,
                                        int zero_guess, const void *d_f, void *d_u, void *stream) {
    hmg_status st = check_level(g, level, false);
    if (st) return st;
    if (!d_f || !d_u || sweeps < 0) return hmg_fail(HMG_ERR_INVALID, "bad argument");
    if (smoother != HMG_SM_GS && smoother != HMG_SM_KACZ) return hmg_fail(HMG_ERR_INVALID, "bad smoother");
    const Level &L = g->lev[level];
    sweep(L.prec, smoother, HMG_ORDER_COLOUR, pick_stream(g, stream), L.geo, L.k, sigma, d_f, d_u, sweeps,
          zero_guess != 0, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_smooth_lex_dev(hmg_grid *g, int level, int smoother, double sigma, int sweeps,
                                            int zero_guess, const void *d_f, void *d_u, void *stream) {
    hmg_status st = check_level(g, level, false);
    if (st) return st;
    if (!d_f || !d_u || sweeps < 0) return hmg_fail(HMG_ERR_INVALID, "bad argument");
    if (smoother != HMG_SM_GS && smoother != HMG_SM_KACZ) return hmg_fail(HMG_ERR_INVALID, "bad smoother");
    const Level &L = g->lev[level];
    sweep(L.prec, smoother, HMG_ORDER_LEX, pick_stream(g, stream), L.geo, L.k, sigma, d_f, d_u, sweeps,
          zero_guess != 0, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_restrict_dev(hmg_grid *g, int level, double sigma, const void *d_f, const void *d_u,
                                          void *d_fc, void *stream) {
    hmg_status st = check_level(g, level, true);
    if (st) return st;
    if (!d_f || !d_u || !d_fc) return hmg_fail(HMG_ERR_INVALID, "null field");
    const Level &L = g->lev[level];
    launch_residual_fw(L.prec, pick_stream(g, stream), L.geo, L.k, sigma, d_f, d_u, d_fc, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_prolong_dev(hmg_grid *g, int level, const void *d_ec, void *d_u, void *stream) {
    hmg_status st = check_level(g, level, true);
    if (st) return st;
    if (!d_ec || !d_u) return hmg_fail(HMG_ERR_INVALID, "null field");
    launch_prolong_add(g->lev[level].prec, pick_stream(g, stream), g->lev[level].geo, d_ec, d_u, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_coarsest_dev(hmg_grid *g, const void *d_f, void *d_u, void *stream) {
    if (!g || !d_f || !d_u) return hmg_fail(HMG_ERR_INVALID, "null argument");
    HIPCHK(hipSetDevice(g->ctx->device));
    const Level &L = g->lev[g->nlev - 1];
    launch_coarsest(L.prec, pick_stream(g, stream), L.geo.M * L.geo.M, g->ainv_t, d_f, d_u, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_gs_down_dev(hmg_grid *g, int level, double sigma_relax, double sigma_resid,
                                         const void *d_f, void *d_u, void *d_fc, void *stream) {
    hmg_status st = check_level(g, level, true);
    if (st) return st;
    if (!d_f || !d_fc || d_u == d_f || d_fc == d_f) return hmg_fail(HMG_ERR_INVALID, "bad fields");
    const Level &L = g->lev[level];
    launch_gs_down(L.prec, false, pick_stream(g, stream), L.geo, L.k, sigma_relax, sigma_resid, d_f, d_u, d_fc,
                   nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_gs_up_dev(hmg_grid *g, int level, double sigma_relax, const void *d_f,
                                       const void *d_u0, const void *d_ec, void *d_uo, void *stream) {
    hmg_status st = check_level(g, level, true);
    if (st) return st;
    if (!d_f || !d_ec || !d_uo || d_uo == d_f || d_uo == d_ec || d_uo == d_u0)
        return hmg_fail(HMG_ERR_INVALID, "bad fields (the output must not alias an input)");
    const Level &L = g->lev[level];
    launch_gs_up(L.prec, false, pick_stream(g, stream), L.geo, L.k, sigma_relax, d_f, d_u0, d_ec, d_uo, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_gs_up_product_dev(hmg_grid *g, int level, double sigma_relax, int kind,
                                               const void *d_f, const void *d_ec, void *d_uo, void *d_mv,
                                               const void *d_dot, void *d_sums, void *stream) {
    hmg_status st = check_level(g, level, true);
    if (st) return st;
    if (g->lev[level].prec != P64) return hmg_fail(HMG_ERR_INVALID, "the fused product runs on FP64 levels only");
    if (kind != 1 && kind != 2) return hmg_fail(HMG_ERR_INVALID, "kind must be 1 or 2");
    if (!d_f || !d_ec || !d_mv || !d_dot) return hmg_fail(HMG_ERR_INVALID, "null field");
    const void *ins[] = {d_f, d_ec, d_dot};
    for (const void *in : ins)
        if ((d_uo && in == d_uo) || in == d_mv || (d_sums && in == d_sums))
            return hmg_fail(HMG_ERR_INVALID, "bad fields (outputs must not alias inputs)");
    if ((d_uo && (d_uo == d_mv || d_uo == d_sums)) || (d_sums && d_mv == d_sums))
        return hmg_fail(HMG_ERR_INVALID, "bad fields (outputs must not alias each other)");
    const Level &L = g->lev[level];
    Krylov &K = g->slot[0].K;
    const int nb = gs_up_mv_blocks(L.geo);
    if (nb > K.pcap) return hmg_fail(HMG_ERR_INVALID, "level %d too large for the reduction scratch", level);
    hipStream_t s = pick_stream(g, stream);
    launch_gs_up_mv(s, kind, L.geo, L.k, sigma_relax, d_f, d_ec, d_uo, d_mv, d_dot, K.partials, nullptr);
    if (d_sums) launch_sum_partials(s, K.partials, nb, kind == 1 ? 2 : 3, (double *)d_sums);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_kacz_tiled_dev(hmg_grid *g, int level, double sigma, int config, const void *d_f,
                                            const void *d_ui, const void *d_ec, void *d_uo, void *stream) {
    hmg_status st = check_level(g, level, false);
    if (st) return st;
    if (config < 0 || config >= KACZ_NCFG || !kacz_cfg_fits(g->lev[level].prec, config))
        return hmg_fail(HMG_ERR_INVALID, "tile configuration %d not available", config);
    if (!d_f || !d_uo || d_uo == d_ui || d_uo == d_f || d_uo == d_ec)
        return hmg_fail(HMG_ERR_INVALID, "bad fields (the output must not alias an input)");
    if (d_ec && level >= g->nlev - 1) return hmg_fail(HMG_ERR_INVALID, "no coarser level");
    const Level &L = g->lev[level];
    launch_kacz_tb(L.prec, config, pick_stream(g, stream), L.geo, L.k, nullptr, sigma, d_f, d_ui, d_ec, d_uo,
                   nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_kacz_down_dev(hmg_grid *g, int level, double sigma_relax, double sigma_resid,
                                           int config, const void *d_f, const void *d_ui, void *d_uo, void *d_fc,
                                           void *stream) {
    hmg_status st = check_level(g, level, false);
    if (st) return st;
    if (level >= g->nlev - 1) return hmg_fail(HMG_ERR_INVALID, "no coarser level");
    if (config < 0 || config >= KACZ_NCFG || !kacz_cfg_resid(config))
        return hmg_fail(HMG_ERR_INVALID, "tile configuration %d has no fused residual form", config);
    if (!d_f || !d_uo || !d_fc || d_uo == d_ui || d_uo == d_f || d_fc == d_f || d_fc == d_ui || d_fc == d_uo)
        return hmg_fail(HMG_ERR_INVALID, "bad fields (outputs must not alias inputs or each other)");
    const Level &L = g->lev[level];
    launch_kacz_tb_resid(L.prec, config, pick_stream(g, stream), L.geo, L.k, nullptr, sigma_relax, sigma_resid,
                         d_f, d_ui, d_uo, d_fc, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" hmg_status hmg_op_kacz_level_dev(hmg_grid *g, int level, double sigma_relax, double sigma_resid,
                                            int sweeps, const void *d_f, const void *d_ui, const void *d_ec,
                                            void *d_uo, void *d_fc, void *stream) {
    hmg_status st = check_level(g, level, false);
    if (st) return st;
    if (!kacz_level_fits(g->lev[level].geo))
        return hmg_fail(HMG_ERR_INVALID, "level %d is larger than n = 63", level);
    if (sweeps < 0 || sweeps > 64) return hmg_fail(HMG_ERR_INVALID, "sweeps must be in [0, 64]");
    if ((d_ec || d_fc) && level >= g->nlev - 1) return hmg_fail(HMG_ERR_INVALID, "no coarser level");
    if (!d_f || !d_uo || d_uo == d_f || d_uo == d_ui || d_uo == d_ec || (d_fc && (d_fc == d_f || d_fc == d_uo)))
        return hmg_fail(HMG_ERR_INVALID, "bad fields (outputs must not alias inputs or each other)");
    const Level &L = g->lev[level];
    launch_kacz_level(L.prec, pick_stream(g, stream), L.geo, L.k, nullptr, sigma_relax, sigma_resid, sweeps, d_f,
                      d_ui, d_ec, d_uo, d_fc, nullptr);
    HIPCHK(hipGetLastError());
    return HMG_OK;
}

extern "C" int hmg_kacz_tile_config(int config, int *tile, int *sweeps, int *threads) {
    if (config < 0 || config >= KACZ_NCFG) return -1;
    if (tile) *tile = kKaczCfgs[config].ts;
    if (sweeps) *sweeps = kKaczCfgs[config].sweeps;
    if (threads) *threads = kKaczCfgs[config].threads;
    return KACZ_NCFG;
}

extern "C" int hmg_kacz_tile_height(int config) {
    if (config < 0 || config >= KACZ_NCFG) return -1;
    return kKaczCfgs[config].ty;
}
