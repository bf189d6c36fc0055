// hmg_host.h -- host-side objects of libhmg (context, grid, solve slots).
// Internal to the library; the public interface is include/hmg.h.
#pragma once

#include "hmg.h"
#include "hmg_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <complex>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

// A named host-side range for rocprofv3 --marker-trace (grid set-up, the
// tuner, solves, batches, the server's admissions and retirements); a
// function call when no tool is attached.
struct MarkRange {
    explicit MarkRange(const char *name) { roctxRangePushA(name); }
    ~MarkRange() { roctxRangePop(); }
    MarkRange(const MarkRange &) = delete;
    MarkRange &operator=(const MarkRange &) = delete;
};

struct ServerState;

// Grid sizes the hierarchy accepts.  Each coarser level halves the interval
// count of the one above (vertex-centred nesting), so every level with
// n > nc must have an even interval count n + 1; the walk stops at the first
// level with n <= nc, the coarsest.  n = 2^m - 1 halves down to nc exactly;
// h = 1/80 (n = 79) gives the levels 79, 39, 19, 9, 4.
inline bool valid_hierarchy(int n, int nc) {
    if (n < 1 || nc < 1 || n < nc) return false;
    for (int l = 0; n > nc; ++l) {
        if (n % 2 == 0 || l >= HMG_MAX_LEVELS - 1) return false;
        n = (n - 1) / 2;
    }
    return true;
}

struct hmg_ctx {
    int    device = 0;
    size_t budget = 0;      // bytes of device memory the server may admit
    double t0 = 0.0;        // clock origin
    double *scratch = nullptr;   // device address of this GPU's static solve scratch
    std::unique_ptr<ServerState> server;
};

// How a level above the bottom solver runs its part of the V-cycle.
enum LevelMode { LM_SIMPLE = 0, LM_GS_FUSED = 1, LM_KACZ_TILED = 2, LM_BOTTOM = 3, LM_KACZ_LEVEL = 4 };

struct Level {
    hmgk::Geo geo;
    hmgk::Prec prec = hmgk::P64;  // storage precision of the level's fields and k
    bool      io64 = false;  // first complex-float level below double levels: its right-hand
                             // side and result are double
    void     *k = nullptr;  // wavenumber in the level's precision
    int       mode = LM_SIMPLE;
    int       kacz_cfg = 1; // index into hmgk::kKaczCfgs
    double   *ktab = nullptr;  // Kaczmarz levels: (k_p, 1 / ||a_p||^2), complex-interleaved FP64
};

// Per right-hand side: level fields of one V-cycle in flight and the
// finest-level Krylov vectors and scalars.
struct Slot {
    void        *f[HMG_MAX_LEVELS] = {};
    void        *u[HMG_MAX_LEVELS] = {};
    void        *u2[HMG_MAX_LEVELS] = {};  // second buffer (tiled kernels never update in place)
    double      *ray_part = nullptr;       // ray correction: patch records, then b and a (K each)
    void        *ray_b = nullptr, *ray_a = nullptr;
    hmgk::Krylov K{};
    int          hist_cap = 0;
    int          last_halfsteps = -1;   // of the last finished solve
    hipGraphExec_t iter_graph = nullptr;
};

struct hmg_grid {
    hmg_ctx   *ctx = nullptr;
    hmg_opts   opts{};
    int        n = 0, nrhs = 0, nlev = 0;
    double     h = 0.0;
    hmgk::Prec prec = hmgk::P64;
    hmg_plan   plan{};
    Level      lev[HMG_MAX_LEVELS];
    double    *k0 = nullptr;      // finest k in FP64 (outer operator)
    int        lb = -1;           // first level of the bottom solver (-1: none)
    hmgk::BottomDesc bottom{};    // per-level parameters of the bottom solver
    double    *ainv_t = nullptr;  // coarsest inverse, column-major complex FP64
    double    *bop = nullptr;     // matrix of the bottom cycle, row-major complex FP64
    int        bop_m = 0;         // its order (nodes of the first bottom level)
    std::vector<Slot> slot;
    char      *mem = nullptr;
    size_t     bytes = 0;
    hipStream_t stream = nullptr;
    long       zs = 0;            // bytes between the buffers of consecutive slots (0: not uniform)
    int        ray_K = 0;         // ray correction: unknowns 8 (nr + 2)^2 (0: off)
    hmgk::RayGeo ray{};
    void      *ray_ex = nullptr, *ray_ey = nullptr;   // wave tables, 8 x M complex each
    double    *ray_Ainv = nullptr;                    // (P^H L P)^{-1}, row-major K x K complex
    double    *hist_all = nullptr;  // residual histories of every slot, hist_cap doubles each
    int        hist_cap = 0;
    hipGraphExec_t batch_graph = nullptr;  // one iteration of every right-hand side, batched
    hmgk::KState *host_state = nullptr;   // pinned, 4 entries
    int          *done_host = nullptr;    // pinned, one done flag per right-hand side
    hipEvent_t ev[4] = {};
};

hmg_status hmg_fail(hmg_status st, const char *fmt, ...);
double     hmg_now();
hmg_status grid_init_device(hmg_grid *g);
hmg_status grid_upload(hmg_grid *g, const std::vector<std::vector<double>> &kl,
                       const std::vector<std::complex<double>> &inv, const hmg_c64 *f);
// Whether grid g can take a problem of size n with nrhs right-hand sides and
// options o in its memory, and the call that puts one there (no device
// allocation; plans, tables, coarsest inverse and bottom matrix rebuilt).
bool       grid_reusable(const hmg_grid *g, int n, int nrhs, const hmg_opts &o);
hmg_status grid_reload(hmg_grid *g, double h, const double *k, const hmg_c64 *f);
size_t     estimate_footprint(int n, const hmg_opts &o);
// A Bi-CGSTAB product the finest up kernel may take over: out = L z with the
// partial sums of kind 1 ((dot, out)) or kind 2 ((out, dot), (out, out)) in
// partials, laid out for `blocks` blocks.  fused reports whether it did; with
// no_z the fused kernel does not store z itself.
struct MvFuse {
    int         kind = 0;
    void       *out = nullptr;
    const void *dot = nullptr;
    double     *partials = nullptr;
    int         blocks = 0;
    bool        fused = false;
    bool        no_z = false;
};
// Whether the finest up kernel of S's V-cycles forms the Krylov products
// (then the solve keeps its x update in the preconditioner's input space:
// kry_update_yr / kry_fold, and the V-cycle outputs are not stored).
bool       vcycle_forms_products(const hmg_grid *g, const Slot &S);
void       enqueue_vcycle(hmg_grid *g, Slot &S, const double *r, double *z, hipStream_t s,
                          const int *skip, MvFuse *mv = nullptr, hmgk::Bz bz = {});
// Whether every right-hand side of the grid can run in one batched launch
// per kernel (fused schedule with the dense bottom matrix, no whole-level
// Kaczmarz kernel, slots at one stride); then g->zs is that stride.
bool       grid_batchable(const hmg_grid *g);
