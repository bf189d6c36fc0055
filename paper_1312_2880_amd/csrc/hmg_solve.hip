// hmg_solve.hip -- context, Bi-CGSTAB driver, batched solves and the request
// server of libhmg (Livshits, arXiv:1312.2880, Section 6).
//
// One Bi-CGSTAB iteration is a fixed sequence of kernels whose scalars stay
// in device memory; the host only reads back a small status record once per
// iteration, one iteration behind the device, so the device never waits for
// the host.  Kernels queued after convergence see the device-side stop flag
// and return at once.  With opts.use_graph the sequence of one iteration is
// captured once per right-hand side and replayed as a hipGraph.

#include "hmg_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>

using namespace hmgk;

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return hmg_fail(HMG_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Request;
// An idle grid kept by the request server for the next request of its size
// and options, with the device bytes it holds.
struct PoolEntry {
    hmg_grid *grid = nullptr;
    size_t    bytes = 0;
};
struct ServerState {
    std::mutex              mu;
    std::condition_variable cv;
    std::thread             worker;
    bool                    running = false;
    bool                    quit = false;
    uint64_t                next_ticket = 1;
    size_t                  used = 0;       // footprints of the admitted requests
    size_t                  pooled = 0;     // bytes of the idle grids in pool
    int                     max_active = 0;
    std::deque<Request *>   queue;
    std::vector<Request *>  active;
    std::vector<PoolEntry>  pool;           // oldest first
    std::map<uint64_t, Request *> all;
};

static void server_stop(hmg_ctx *ctx);

// Device memory of the allocation-free solve (hmg_solve_dev_static): the
// reduction partials and the residual history of one solve at a time per
// GPU.  In host code `scratch` only names the symbol; its device address on
// each GPU comes from hipGetSymbolAddress (below), taken once per device
// with that device current, and only that address is passed to kernels.
static __device__ __align__(256) double scratch[HMG_STATIC_SCRATCH_BYTES / sizeof(double)];
static std::mutex g_scratch_mu;
static std::map<int, double *> g_scratch_addr;   // device -> address of its copy of scratch

static hmg_status scratch_address(int device, double **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it == g_scratch_addr.end()) {
        double *p = nullptr;
        HIPCHK(hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch)));
        if (!p) return hmg_fail(HMG_ERR_DEVICE, "no device address for the static scratch");
        it = g_scratch_addr.emplace(device, p).first;
    }
    *out = it->second;
    return HMG_OK;
}

extern "C" hmg_status hmg_ctx_create(int device, size_t hbm_budget_bytes, hmg_ctx **out) {
    if (!out) return hmg_fail(HMG_ERR_INVALID, "null output handle");
    *out = nullptr;
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return hmg_fail(HMG_ERR_INVALID, "device %d not present", device);
    HIPCHK(hipSetDevice(device));
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    double *scr = nullptr;
    hmg_status sst = scratch_address(device, &scr);   // with `device` current
    if (sst != HMG_OK) return sst;
    hmg_ctx *c = new hmg_ctx();
    c->device = device;
    c->scratch = scr;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
    c->t0 = hmg_now();
    c->server.reset(new ServerState());
    *out = c;
    return HMG_OK;
}

extern "C" void hmg_ctx_destroy(hmg_ctx *ctx) {
    if (!ctx) return;
    server_stop(ctx);
    delete ctx;
}

extern "C" double hmg_ctx_clock(const hmg_ctx *ctx) { return ctx ? hmg_now() - ctx->t0 : 0.0; }

// ---------------------------------------------------------------------------
// one Bi-CGSTAB iteration
// ---------------------------------------------------------------------------
// Whether the solve keeps its x update in the preconditioner's input space
// (y += alpha p + omega s, x += B y when the solve ends): where the finest
// up kernel forms the Krylov products, unless periodic true-residual checks
// need the current x every iteration.
static bool y_space(const hmg_grid *g, const Slot &S) {
    return vcycle_forms_products(g, S) && g->opts.true_res_every == 0 && g->ray_K == 0;
}

// The Section 6.1 ray correction of the preconditioner's result z for the
// input r (when the grid has one): z += C_R (r - L z).
static void ray_after(hmg_grid *g, Slot &S, const double *r, double *z, hipStream_t s, const int *skip, Bz bz) {
    if (!g->ray_K) return;
    launch_ray_correct(s, g->ray, g->lev[0].geo.H, g->k0, g->ray_ex, g->ray_ey, g->ray_Ainv, r, z, S.ray_part,
                       S.ray_b, S.ray_a, skip, bz);
}

// One iteration of slot S, or batched (bz.nz > 1) of slots S .. S + nz - 1:
// each kernel then runs once for all of them with blockIdx.z selecting the
// right-hand side, and a right-hand side whose solve has ended sees its own
// stop flags and returns.
static void enqueue_iteration(hmg_grid *g, Slot &S, hipStream_t s, Bz bz = {}) {
    const Geo &g0 = g->lev[0].geo;
    const int *stop = &S.K.st->stop;
    const Kz kb{bz.zs, (long)g->hist_cap * 8, bz.nz};
    kry_update_p(s, g0, S.K, kb);
    // v = L p^ and t = L s^ come from the V-cycle's last kernel where it can
    // form them, else from kernels of their own.  Where it can, p^ and s^
    // are not stored either: x advances as x + B y with y += alpha p +
    // omega s (B is linear and fixed), folded in when the solve ends.
    const bool ym = y_space(g, S);
    MvFuse mv;
    mv.kind = 1;
    mv.out = S.K.v;
    mv.dot = S.K.rh;
    mv.partials = S.K.partials;
    mv.no_z = ym;
    // with the ray correction the V-cycle's result changes after it, so the
    // products come from kernels of their own
    enqueue_vcycle(g, S, S.K.p, S.K.ph, s, stop, g->ray_K ? nullptr : &mv, bz);
    ray_after(g, S, S.K.p, S.K.ph, s, stop, bz);
    if (mv.fused) kry_alpha_fin(s, S.K, mv.blocks, kb);
    else kry_matvec_alpha(s, g0, g->k0, S.K, kb);
    kry_update_s(s, g0, S.K, kb);
    mv = MvFuse();
    mv.kind = 2;
    mv.out = S.K.t;
    mv.dot = S.K.s;
    mv.partials = S.K.partials;
    mv.no_z = ym;
    enqueue_vcycle(g, S, S.K.s, S.K.sh, s, stop, g->ray_K ? nullptr : &mv, bz);
    ray_after(g, S, S.K.s, S.K.sh, s, stop, bz);
    if (mv.fused) kry_omega_fin(s, S.K, mv.blocks, kb);
    else kry_matvec_omega(s, g0, g->k0, S.K, kb);
    if (ym) kry_update_yr(s, g0, S.K, kb);
    else kry_update_xr(s, g0, S.K, kb);
    if (g->opts.true_res_every > 0) kry_checkpoint(s, g0, g->k0, S.K, kb);
}

static hmg_status iteration_graph(hmg_grid *g, Slot &S) {
    if (S.iter_graph) return HMG_OK;
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
    enqueue_iteration(g, S, g->stream);
    hipError_t e = hipStreamEndCapture(g->stream, &graph);
    if (e != hipSuccess) return hmg_fail(HMG_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&S.iter_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        S.iter_graph = nullptr;
        return hmg_fail(HMG_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    return HMG_OK;
}

static hmg_status launch_iteration(hmg_grid *g, Slot &S, hipStream_t s) {
    if (g->opts.use_graph) {
        hmg_status st = iteration_graph(g, S);
        if (st != HMG_OK) return st;
        HIPCHK(hipGraphLaunch(S.iter_graph, s));
    } else {
        enqueue_iteration(g, S, s);
        HIPCHK(hipGetLastError());
    }
    return HMG_OK;
}

// The residual histories of all right-hand sides of a grid: one allocation,
// the same capacity per slot (so batched kernels find slot z's history at a
// fixed stride), grown when a solve asks for more iterations.
static hmg_status ensure_hist(hmg_grid *g, int maxit) {
    int cap = 2 * maxit + 2;
    if (g->hist_cap >= cap) return HMG_OK;
    if (g->hist_all) (void)hipFree(g->hist_all);
    g->hist_all = nullptr;
    g->hist_cap = 0;
    for (Slot &S : g->slot) {
        S.K.hist = nullptr;
        S.hist_cap = 0;
    }
    HIPCHK(hipMalloc((void **)&g->hist_all, (size_t)cap * 8 * g->nrhs));
    g->hist_cap = cap;
    for (int r = 0; r < g->nrhs; ++r) {
        Slot &S = g->slot[r];
        S.K.hist = g->hist_all + (size_t)r * cap;
        S.hist_cap = cap;
        if (S.iter_graph) {  // the graphs captured the old pointers
            (void)hipGraphExecDestroy(S.iter_graph);
            S.iter_graph = nullptr;
        }
    }
    if (g->batch_graph) {
        (void)hipGraphExecDestroy(g->batch_graph);
        g->batch_graph = nullptr;
    }
    return HMG_OK;
}

// Solve state machine of one slot, usable both blocking (run_solve) and
// stepped by the request server.
struct SolveRun {
    hmg_grid   *g = nullptr;
    Slot       *S = nullptr;
    hipStream_t s = nullptr;
    double      rtol = 1e-6;
    int         maxit = 100;
    int         inflight = 0;      // iterations queued but not yet observed
    int         issued = 0;
    KState     *hs = nullptr;      // pinned, 2 records
    hipEvent_t  ev[2] = {};
    double      t_start = 0.0;
    bool        direct = false;    // enqueue kernel by kernel (no graph, no history allocation)
};

static hmg_status run_begin(SolveRun &R, int x0_given) {
    hmg_grid *g = R.g;
    if (!R.direct) {
        hmg_status st = ensure_hist(g, R.maxit);
        if (st) return st;
    }
    kry_init(R.s, g->lev[0].geo, g->k0, R.S->K, x0_given, R.rtol, 2 * R.maxit, g->opts.breakdown_at,
             g->opts.true_res_every, g->opts.nan_at);
    if (y_space(g, *R.S))   // y = 0 (the x update in the preconditioner's input space)
        launch_fill_zero(P64, R.s, R.S->K.ph, (size_t)g->lev[0].geo.M * g->lev[0].geo.M, nullptr);
    HIPCHK(hipGetLastError());
    R.inflight = 0;
    R.issued = 0;
    R.t_start = hmg_now();
    return HMG_OK;
}

// Queue one iteration and an event behind it; the iteration's kernels write
// the done flag to pinned host memory (run_done).
static hmg_status run_issue(SolveRun &R) {
    if (R.direct) {
        enqueue_iteration(R.g, *R.S, R.s);
        HIPCHK(hipGetLastError());
    } else {
        hmg_status st = launch_iteration(R.g, *R.S, R.s);
        if (st) return st;
    }
    int q = R.issued & 1;
    HIPCHK(hipEventRecord(R.ev[q], R.s));
    R.issued++;
    R.inflight++;
    return HMG_OK;
}

// The device's done flag as of the last finished event (or later).
static bool run_done(const SolveRun &R) { return __atomic_load_n(R.S->K.done_host, __ATOMIC_ACQUIRE) != 0; }

// Finish after the device reported done: confirm with the FP64 true
// residual.  Returns HMG_PENDING if the iteration must go on (restart).
static hmg_status run_finish(SolveRun &R, hmg_solve_info *info) {
    HIPCHK(hipStreamSynchronize(R.s));
    Slot &S = *R.S;
    if (y_space(R.g, S)) {
        // x += B y, y = 0
        enqueue_vcycle(R.g, S, S.K.ph, S.K.sh, R.s, nullptr);
        kry_fold(R.s, R.g->lev[0].geo, S.K);
    }
    kry_true_residual(R.s, R.g->lev[0].geo, R.g->k0, S.K);
    HIPCHK(hipMemcpyAsync(&R.hs[0], S.K.st, sizeof(KState), hipMemcpyDeviceToHost, R.s));
    HIPCHK(hipStreamSynchronize(R.s));
    const KState &k = R.hs[0];
    hmg_status res;
    if (k.done == 1 && k.true_rel <= R.rtol) {
        res = HMG_OK;
    } else if (k.done == 3 || !std::isfinite(k.true_rel)) {
        res = HMG_ERR_BREAKDOWN;   // a residual norm was not finite
    } else if (k.done == 1 && k.halfsteps < 2 * R.maxit) {
        kry_restart_from_true(R.s, S.K);
        HIPCHK(hipGetLastError());
        R.inflight = 0;
        return HMG_PENDING;
    } else {
        res = HMG_ERR_NOT_CONVERGED;
    }
    S.last_halfsteps = k.halfsteps;
    if (info) {
        info->halfsteps = k.halfsteps;
        info->iters = 0.5 * k.halfsteps;
        info->rel_res_true = k.true_rel;
        info->status = res;
        info->levels = R.g->nlev;
        info->restarts = k.restarts;
        info->seconds = hmg_now() - R.t_start;
        info->flags = (R.g->plan.kHmax[0] > 0.2 * M_PI) ? HMG_INFO_KH_ABOVE_GUIDE : 0;
    }
    return res;
}

static hmg_status run_solve(SolveRun &R, int x0_given, hmg_solve_info *info) {
    hmg_status st = run_begin(R, x0_given);
    if (st) return st;
    for (;;) {
        st = run_issue(R);
        if (st) return st;
        if (R.inflight < 2) continue;
        int q = (R.issued - 2) & 1;   // the older of the two in flight
        HIPCHK(hipEventSynchronize(R.ev[q]));
        R.inflight--;
        if (run_done(R)) {
            st = run_finish(R, info);
            if (st == HMG_PENDING) continue;
            return st;
        }
        if (R.issued > R.maxit + 4) {   // the device stops at maxit; guard only
            st = run_finish(R, info);
            return st == HMG_PENDING ? HMG_ERR_NOT_CONVERGED : st;
        }
    }
}

static void run_init(SolveRun &R, hmg_grid *g, Slot *S, hipStream_t s, double rtol, int maxit);

// ---------------------------------------------------------------------------
// Every right-hand side of a grid in one batched iteration (grid_batchable):
// the slots are started one by one, then advance together, one launch per
// kernel for all of them; a slot whose done flag appears is finished alone
// (FP64 true-residual check, a restart or its result) while the others go on.
// ---------------------------------------------------------------------------
struct BatchRun {
    hmg_grid              *g = nullptr;
    std::vector<SolveRun>  runs;
    std::vector<int>       live;      // 1 while the slot's solve runs
    std::vector<hmg_status> status;
    hmg_solve_info        *info = nullptr;   // nrhs entries or null
    int                    inflight = 0, issued = 0, left = 0;
};

static hmg_status batch_graph(hmg_grid *g) {
    if (g->batch_graph) return HMG_OK;
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
    enqueue_iteration(g, g->slot[0], g->stream, Bz{g->zs, g->nrhs});
    hipError_t e = hipStreamEndCapture(g->stream, &graph);
    if (e != hipSuccess) return hmg_fail(HMG_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&g->batch_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g->batch_graph = nullptr;
        return hmg_fail(HMG_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    return HMG_OK;
}

static hmg_status run_begin(SolveRun &R, int x0_given);
static hmg_status run_finish(SolveRun &R, hmg_solve_info *info);
static bool run_done(const SolveRun &R);

static hmg_status batch_begin(BatchRun &B, hmg_grid *g, double rtol, int maxit, int x0_given,
                              hmg_solve_info *info) {
    B.g = g;
    B.info = info;
    B.runs.assign(g->nrhs, SolveRun());
    B.live.assign(g->nrhs, 1);
    B.status.assign(g->nrhs, HMG_OK);
    B.inflight = B.issued = 0;
    B.left = g->nrhs;
    for (int r = 0; r < g->nrhs; ++r) {
        run_init(B.runs[r], g, &g->slot[r], g->stream, rtol, maxit);
        hmg_status st = run_begin(B.runs[r], x0_given);
        if (st) return st;
    }
    if (g->opts.use_graph) return batch_graph(g);
    return HMG_OK;
}

static hmg_status batch_issue(BatchRun &B) {
    hmg_grid *g = B.g;
    if (g->opts.use_graph) {
        HIPCHK(hipGraphLaunch(g->batch_graph, g->stream));
    } else {
        enqueue_iteration(g, g->slot[0], g->stream, Bz{g->zs, g->nrhs});
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipEventRecord(g->ev[2 + (B.issued & 1)], g->stream));
    B.issued++;
    B.inflight++;
    return HMG_OK;
}

// Wait for the older iteration in flight, then finish every slot whose done
// flag is up (finishing drains the stream).
static hmg_status batch_observe(BatchRun &B) {
    hmg_grid *g = B.g;
    HIPCHK(hipEventSynchronize(g->ev[2 + ((B.issued - B.inflight) & 1)]));
    B.inflight--;
    const bool over = B.issued > B.runs[0].maxit + 4;   // the device stops each slot at maxit; guard only
    for (int r = 0; r < g->nrhs; ++r) {
        if (!B.live[r] || !(run_done(B.runs[r]) || over)) continue;
        hmg_status st = run_finish(B.runs[r], B.info ? &B.info[r] : nullptr);
        B.inflight = 0;   // run_finish synchronised the stream
        if (st == HMG_PENDING && !over) continue;   // restarted from the true residual
        if (st == HMG_PENDING) st = HMG_ERR_NOT_CONVERGED;
        if (st != HMG_OK && st != HMG_ERR_NOT_CONVERGED && st != HMG_ERR_BREAKDOWN) return st;
        B.status[r] = st;
        B.live[r] = 0;
        B.left--;
    }
    return HMG_OK;
}

static hmg_status batch_run(BatchRun &B) {
    while (B.left > 0) {
        while (B.inflight < 2) {
            hmg_status st = batch_issue(B);
            if (st) return st;
        }
        hmg_status st = batch_observe(B);
        if (st) return st;
    }
    HIPCHK(hipStreamSynchronize(B.g->stream));
    return HMG_OK;
}

static void run_init(SolveRun &R, hmg_grid *g, Slot *S, hipStream_t s, double rtol, int maxit) {
    R.g = g;
    R.S = S;
    R.s = s;
    R.rtol = rtol;
    R.maxit = maxit;
    R.hs = g->host_state;
    R.ev[0] = g->ev[0];
    R.ev[1] = g->ev[1];
}

static hmg_status check_solve_args(double rtol, int maxit) {
    if (!(rtol > 0.0) || !std::isfinite(rtol)) return hmg_fail(HMG_ERR_INVALID, "rtol must be > 0");
    if (maxit < 1 || maxit > 1000000) return hmg_fail(HMG_ERR_INVALID, "maxit must be in [1, 1e6]");
    return HMG_OK;
}

extern "C" hmg_status hmg_solve(hmg_grid *g, const hmg_c64 *x0, hmg_c64 *x, double rtol, int maxit,
                                hmg_solve_info *info) {
    MarkRange mark_("hmg_solve");
    if (!g || !x) return hmg_fail(HMG_ERR_INVALID, "null argument");
    hmg_status st = check_solve_args(rtol, maxit);
    if (st) return st;
    size_t m0 = (size_t)g->lev[0].geo.M * g->lev[0].geo.M;
    if (x0)
        for (size_t q = 0; q < m0 * (size_t)g->nrhs; ++q)
            if (!std::isfinite(x0[q].re) || !std::isfinite(x0[q].im))
                return hmg_fail(HMG_ERR_INVALID, "x0 must be finite");
    HIPCHK(hipSetDevice(g->ctx->device));
    // every initial guess is on the device before x (which may alias x0) is
    // written
    if (x0)
        for (int r = 0; r < g->nrhs; ++r)
            HIPCHK(hipMemcpy(g->slot[r].K.x, x0 + m0 * r, m0 * 16, hipMemcpyHostToDevice));
    hmg_status worst = HMG_OK;
    if (grid_batchable(g)) {
        // every right-hand side in one batched iteration
        BatchRun B;
        hmg_status st2 = batch_begin(B, g, rtol, maxit, x0 ? 1 : 0, info);
        if (st2 == HMG_OK) st2 = batch_run(B);
        if (st2 != HMG_OK) return st2;
        for (int r = 0; r < g->nrhs; ++r) {
            HIPCHK(hipMemcpy(x + m0 * r, g->slot[r].K.x, m0 * 16, hipMemcpyDeviceToHost));
            if (B.status[r] != HMG_OK && worst == HMG_OK) worst = B.status[r];
            if (info) info[r].flags |= HMG_INFO_BATCHED;
        }
        return worst;
    }
    for (int r = 0; r < g->nrhs; ++r) {
        SolveRun R;
        run_init(R, g, &g->slot[r], g->stream, rtol, maxit);
        hmg_status sr = run_solve(R, x0 ? 1 : 0, info ? &info[r] : nullptr);
        if (sr != HMG_OK && sr != HMG_ERR_NOT_CONVERGED && sr != HMG_ERR_BREAKDOWN) return sr;
        HIPCHK(hipMemcpy(x + m0 * r, g->slot[r].K.x, m0 * 16, hipMemcpyDeviceToHost));
        if (sr != HMG_OK && worst == HMG_OK) worst = sr;
    }
    return worst;
}

extern "C" hmg_status hmg_solve_dev(hmg_grid *g, int rhs, const void *d_b, void *d_x, int x0_given, double rtol,
                                    int maxit, hmg_solve_info *info, void *stream) {
    MarkRange mark_("hmg_solve_dev");
    if (!g || !d_x || rhs < 0 || rhs >= g->nrhs) return hmg_fail(HMG_ERR_INVALID, "bad argument");
    hmg_status st = check_solve_args(rtol, maxit);
    if (st) return st;
    HIPCHK(hipSetDevice(g->ctx->device));
    hipStream_t s = stream ? (hipStream_t)stream : g->stream;
    Slot &S = g->slot[rhs];
    size_t bytes = (size_t)g->lev[0].geo.M * g->lev[0].geo.M * 16;
    if (d_b) HIPCHK(hipMemcpyAsync(S.K.b, d_b, bytes, hipMemcpyDeviceToDevice, s));
    if (x0_given) HIPCHK(hipMemcpyAsync(S.K.x, d_x, bytes, hipMemcpyDeviceToDevice, s));
    SolveRun R;
    run_init(R, g, &S, s, rtol, maxit);
    hmg_status sr = run_solve(R, x0_given, info);
    if (sr != HMG_OK && sr != HMG_ERR_NOT_CONVERGED && sr != HMG_ERR_BREAKDOWN) return sr;
    HIPCHK(hipMemcpyAsync(d_x, S.K.x, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return sr;
}

// The allocation-free form of hmg_solve_dev: the solve runs on a copy of the
// slot whose reduction partials and residual history point into this GPU's
// static scratch, and its iterations are enqueued kernel by kernel.
extern "C" hmg_status hmg_solve_dev_static(hmg_grid *g, int rhs, const void *d_b, void *d_x, int x0_given,
                                           double rtol, int maxit, hmg_solve_info *info, void *stream) {
    if (!g || !d_x || rhs < 0 || rhs >= g->nrhs) return hmg_fail(HMG_ERR_INVALID, "bad argument");
    hmg_status st = check_solve_args(rtol, maxit);
    if (st) return st;
    Slot &S = g->slot[rhs];
    const size_t part_bytes = ((size_t)3 * S.K.pcap * sizeof(double) + 255) & ~size_t(255);
    const size_t hist_n = 2 * (size_t)maxit + 2;
    if (part_bytes + hist_n * sizeof(double) > HMG_STATIC_SCRATCH_BYTES)
        return hmg_fail(HMG_ERR_TOO_LARGE,
                        "the static scratch (%d bytes) holds %zu bytes of partial sums and %zu of history; "
                        "this grid and maxit need %zu",
                        (int)HMG_STATIC_SCRATCH_BYTES, part_bytes, hist_n * sizeof(double),
                        part_bytes + hist_n * sizeof(double));
    if (!g->ctx->scratch) return hmg_fail(HMG_ERR_DEVICE, "the context has no static scratch");
    HIPCHK(hipSetDevice(g->ctx->device));
    hipStream_t s = stream ? (hipStream_t)stream : g->stream;
    size_t bytes = (size_t)g->lev[0].geo.M * g->lev[0].geo.M * 16;
    if (d_b) HIPCHK(hipMemcpyAsync(S.K.b, d_b, bytes, hipMemcpyDeviceToDevice, s));
    if (x0_given) HIPCHK(hipMemcpyAsync(S.K.x, d_x, bytes, hipMemcpyDeviceToDevice, s));
    Slot T = S;                       // same fields and state, other scratch
    T.iter_graph = nullptr;
    T.K.partials = g->ctx->scratch;
    T.K.hist = (double *)((char *)g->ctx->scratch + part_bytes);
    T.hist_cap = (int)hist_n;
    SolveRun R;
    run_init(R, g, &T, s, rtol, maxit);
    R.direct = true;
    hmg_status sr = run_solve(R, x0_given, info);
    S.last_halfsteps = -1;            // the history lived in the static scratch
    if (sr != HMG_OK && sr != HMG_ERR_NOT_CONVERGED && sr != HMG_ERR_BREAKDOWN) return sr;
    HIPCHK(hipMemcpyAsync(d_x, S.K.x, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return sr;
}

// ---------------------------------------------------------------------------
// stationary cycles: x <- x + B (f - L x)
// ---------------------------------------------------------------------------
extern "C" hmg_status hmg_solve_cycles(hmg_grid *g, const hmg_c64 *x0, hmg_c64 *x, double rtol, int maxit,
                                       hmg_solve_info *info) {
    MarkRange mark_("hmg_solve_cycles");
    if (!g || !x) return hmg_fail(HMG_ERR_INVALID, "null argument");
    hmg_status st = check_solve_args(rtol, maxit);
    if (st) return st;
    HIPCHK(hipSetDevice(g->ctx->device));
    st = ensure_hist(g, maxit);
    if (st) return st;
    const Geo &g0 = g->lev[0].geo;
    const size_t m0 = (size_t)g0.M * g0.M;
    hipStream_t s = g->stream;
    hmg_status worst = HMG_OK;
    for (int r = 0; r < g->nrhs; ++r) {
        Slot &S = g->slot[r];
        const double t0 = hmg_now();
        if (x0) HIPCHK(hipMemcpy(S.K.x, x0 + m0 * r, m0 * 16, hipMemcpyHostToDevice));
        kry_init(s, g0, g->k0, S.K, x0 ? 1 : 0, rtol, 2 * maxit, 0);   // ||b||, x (0 unless x0)
        std::vector<double> hist;
        int cyc = 0;
        hmg_status res = HMG_ERR_NOT_CONVERGED;
        double rel = -1.0;
        for (;; ++cyc) {
            kry_true_residual(s, g0, g->k0, S.K);   // r = b - L x and ||r|| / ||b||
            HIPCHK(hipMemcpyAsync(g->host_state, S.K.st, sizeof(KState), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            rel = g->host_state->true_rel;
            hist.push_back(rel);
            if (rel <= rtol) {
                res = HMG_OK;
                break;
            }
            if (cyc >= maxit || !std::isfinite(rel)) break;
            enqueue_vcycle(g, S, S.K.r, S.K.sh, s, nullptr);
            ray_after(g, S, S.K.r, S.K.sh, s, nullptr, Bz{});
            kry_fold(s, g0, S.K);   // x += z
            HIPCHK(hipGetLastError());
        }
        if (S.K.hist && !hist.empty())
            HIPCHK(hipMemcpy(S.K.hist, hist.data(), std::min(hist.size(), (size_t)S.hist_cap) * 8,
                             hipMemcpyHostToDevice));
        S.last_halfsteps = (int)hist.size() - 1;
        if (info) {
            hmg_solve_info &I = info[r];
            I = hmg_solve_info{};
            I.iters = cyc;
            I.halfsteps = cyc;
            I.rel_res_true = rel;
            I.status = res;
            I.levels = g->nlev;
            I.seconds = hmg_now() - t0;
            I.flags = (g->plan.kHmax[0] > 0.2 * M_PI) ? HMG_INFO_KH_ABOVE_GUIDE : 0;
        }
        HIPCHK(hipMemcpy(x + m0 * r, S.K.x, m0 * 16, hipMemcpyDeviceToHost));
        if (res != HMG_OK && worst == HMG_OK) worst = res;
    }
    return worst;
}

// ---------------------------------------------------------------------------
// batched solves of many grids: each grid advances every right-hand side one
// iteration per round on its own stream (one batched launch per kernel where
// the grid allows it, else its right-hand sides one after another), so that
// the work of different instances overlaps on the device.
// ---------------------------------------------------------------------------
extern "C" hmg_status hmg_solve_batch(hmg_ctx *ctx, int count, hmg_grid *const *grids, hmg_c64 *const *x,
                                      double rtol, int maxit, hmg_solve_info *const *info) {
    MarkRange mark_("hmg_solve_batch");
    if (!ctx || count < 0 || (count > 0 && (!grids || !x))) return hmg_fail(HMG_ERR_INVALID, "bad argument");
    hmg_status st = check_solve_args(rtol, maxit);
    if (st) return st;
    for (int q = 0; q < count; ++q)
        if (!grids[q] || !x[q] || grids[q]->ctx != ctx) return hmg_fail(HMG_ERR_INVALID, "bad grid %d", q);
    for (int q = 0; q < count; ++q)
        for (int p = 0; p < q; ++p)
            if (grids[p] == grids[q]) return hmg_fail(HMG_ERR_INVALID, "grid %d appears twice", q);
    HIPCHK(hipSetDevice(ctx->device));
    // per grid: a batched run, or one pending solve per right-hand side
    struct Item {
        int q, r;
    };
    std::vector<char> batched(count, 0);
    std::vector<BatchRun> bruns(count);
    std::vector<std::deque<Item>> per_grid(count);
    std::vector<SolveRun> runs(count);
    std::vector<int> live(count, 0);
    hmg_status worst = HMG_OK;
    auto start_next = [&](int q) -> hmg_status {
        if (per_grid[q].empty()) {
            live[q] = 0;
            return HMG_OK;
        }
        Item it = per_grid[q].front();
        run_init(runs[q], grids[q], &grids[q]->slot[it.r], grids[q]->stream, rtol, maxit);
        live[q] = 1;
        return run_begin(runs[q], 0);
    };
    for (int q = 0; q < count; ++q) {
        batched[q] = grid_batchable(grids[q]);
        if (batched[q]) {
            st = batch_begin(bruns[q], grids[q], rtol, maxit, 0, info ? info[q] : nullptr);
            live[q] = 1;
        } else {
            for (int r = 0; r < grids[q]->nrhs; ++r) per_grid[q].push_back(Item{q, r});
            st = start_next(q);
        }
        if (st) return st;
    }
    for (;;) {
        bool any = false;
        for (int q = 0; q < count; ++q) {
            if (!live[q]) continue;
            any = true;
            if (batched[q]) {
                while (bruns[q].inflight < 2) {
                    st = batch_issue(bruns[q]);
                    if (st) return st;
                }
            } else if (runs[q].inflight < 2) {
                st = run_issue(runs[q]);
                if (st) return st;
            }
        }
        if (!any) break;
        for (int q = 0; q < count; ++q) {
            if (!live[q]) continue;
            if (batched[q]) {
                BatchRun &B = bruns[q];
                if (B.inflight < 2) continue;
                st = batch_observe(B);
                if (st) return st;
                if (B.left == 0) {
                    HIPCHK(hipStreamSynchronize(grids[q]->stream));
                    size_t m0 = (size_t)grids[q]->lev[0].geo.M * grids[q]->lev[0].geo.M;
                    for (int r = 0; r < grids[q]->nrhs; ++r) {
                        HIPCHK(hipMemcpy(x[q] + m0 * r, grids[q]->slot[r].K.x, m0 * 16, hipMemcpyDeviceToHost));
                        if (B.status[r] != HMG_OK && worst == HMG_OK) worst = B.status[r];
                        if (info && info[q]) info[q][r].flags |= HMG_INFO_BATCHED;
                    }
                    live[q] = 0;
                }
                continue;
            }
            SolveRun &R = runs[q];
            if (R.inflight < 2) continue;
            int e = (R.issued - 2) & 1;
            HIPCHK(hipEventSynchronize(R.ev[e]));
            R.inflight--;
            bool over = R.issued > R.maxit + 4;
            if (run_done(R) || over) {
                Item it = per_grid[q].front();
                hmg_solve_info *inf = (info && info[q]) ? &info[q][it.r] : nullptr;
                hmg_status sr = run_finish(R, inf);
                if (sr == HMG_PENDING && !over) continue;
                if (sr == HMG_PENDING) sr = HMG_ERR_NOT_CONVERGED;
                if (sr != HMG_OK && sr != HMG_ERR_NOT_CONVERGED && sr != HMG_ERR_BREAKDOWN) return sr;
                if (sr != HMG_OK && worst == HMG_OK) worst = sr;
                size_t m0 = (size_t)grids[q]->lev[0].geo.M * grids[q]->lev[0].geo.M;
                HIPCHK(hipMemcpy(x[q] + m0 * it.r, R.S->K.x, m0 * 16, hipMemcpyDeviceToHost));
                per_grid[q].pop_front();
                st = start_next(q);
                if (st) return st;
            }
        }
    }
    return worst;
}

// ---------------------------------------------------------------------------
// request server (continuous batching)
// ---------------------------------------------------------------------------
struct Request {
    uint64_t            ticket = 0;
    int                 n = 0;
    double              h = 0.0;
    std::vector<double> k;
    std::vector<hmg_c64> f;
    hmg_opts            opts{};
    double              rtol = 1e-6;
    int                 maxit = 100;
    size_t              footprint = 0;
    int                 state = 0;      // 0 queued, 1 active, 2 finished
    std::atomic<bool>   cancel{false};
    hmg_grid           *grid = nullptr;
    bool                reuse = false;  // grid comes from the pool (reload in place)
    SolveRun            run;
    hmg_result          result{};
    std::vector<hmg_c64> x;
};

// Finish request q: copy its solution, return its grid to the pool (its
// memory stays allocated for the next request of that size), publish the
// result.
static void retire(hmg_ctx *ctx, Request *q, hmg_status status) {
    MarkRange mark_("hmg server retire");
    ServerState &S = *ctx->server;
    hmg_grid *keep = nullptr;
    if (q->grid) {
        if (status == HMG_OK || status == HMG_ERR_NOT_CONVERGED || status == HMG_ERR_BREAKDOWN) {
            size_t m0 = (size_t)(q->n + 2) * (q->n + 2);
            q->x.resize(m0);
            if (hipMemcpy(q->x.data(), q->grid->slot[0].K.x, m0 * 16, hipMemcpyDeviceToHost) != hipSuccess)
                status = HMG_ERR_DEVICE;
        } else {
            (void)hipStreamSynchronize(q->grid->stream);
        }
        if (status == HMG_ERR_DEVICE) hmg_grid_destroy(q->grid);
        else keep = q->grid;
        q->grid = nullptr;
    }
    std::lock_guard<std::mutex> lk(S.mu);
    if (keep) {
        // what the kept grid holds: its carved memory and its history (at
        // least this request's, maybe an earlier, longer one's)
        const size_t held = std::max(q->footprint, keep->bytes + (size_t)keep->hist_cap * 8 * keep->nrhs);
        S.pool.push_back(PoolEntry{keep, held});
        S.pooled += held;
    }
    if (q->state == 1) S.used -= q->footprint;
    q->state = 2;
    q->result.status = status;
    q->result.t_done = hmg_now() - ctx->t0;
    q->result.footprint_bytes = q->footprint;
    S.active.erase(std::remove(S.active.begin(), S.active.end(), q), S.active.end());
    S.cv.notify_all();
}

static void server_loop(hmg_ctx *ctx) {
    ServerState &S = *ctx->server;
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<Request *> admit;
        std::vector<hmg_grid *> evict;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait(lk, [&] { return S.quit || !S.queue.empty() || !S.active.empty(); });
            if (S.quit) return;
            while (!S.queue.empty()) {
                Request *q = S.queue.front();
                if (q->cancel.load()) {
                    S.queue.pop_front();
                    q->state = 2;
                    q->result.status = HMG_ERR_CANCELLED;
                    q->result.t_done = hmg_now() - ctx->t0;
                    S.cv.notify_all();
                    continue;
                }
                bool slot_ok = S.max_active <= 0 || (int)(S.active.size() + admit.size()) < S.max_active;
                if (!slot_ok) break;
                // an idle grid of the request's size and options takes it in
                // place; idle grids of other sizes give their memory back
                // (oldest first) only when the budget needs it
                // (its residual history must hold this request's maxit too,
                // or the solve would reallocate it)
                int match = -1;
                for (int e = (int)S.pool.size() - 1; e >= 0; --e)
                    if (grid_reusable(S.pool[e].grid, q->n, 1, q->opts) &&
                        S.pool[e].grid->hist_cap >= 2 * q->maxit + 2) {
                        match = e;
                        break;
                    }
                const size_t mine = match >= 0 ? S.pool[match].bytes : 0;
                size_t avail = ctx->budget - std::min(ctx->budget, S.used + S.pooled - mine);
                for (int e = 0; e < (int)S.pool.size() && q->footprint > avail;) {
                    if (e == match) {
                        ++e;
                        continue;
                    }
                    avail += S.pool[e].bytes;
                    S.pooled -= S.pool[e].bytes;
                    evict.push_back(S.pool[e].grid);
                    S.pool.erase(S.pool.begin() + e);
                    if (match > e) --match;
                }
                if (q->footprint > avail) break;
                S.queue.pop_front();
                if (match >= 0) {
                    q->grid = S.pool[match].grid;
                    q->reuse = true;
                    S.pooled -= S.pool[match].bytes;
                    S.pool.erase(S.pool.begin() + match);
                }
                S.used += q->footprint;
                q->state = 1;
                q->result.reused = q->reuse ? 1 : 0;
                q->result.t_admit = hmg_now() - ctx->t0;
                admit.push_back(q);
            }
        }
        for (hmg_grid *g : evict) hmg_grid_destroy(g);
        for (Request *q : admit) {
            hmg_status st;
            if (q->reuse) st = grid_reload(q->grid, q->h, q->k.data(), q->f.data());
            else st = hmg_grid_create(ctx, q->n, q->h, q->k.data(), q->f.data(), 1, &q->opts, &q->grid);
            if (st == HMG_OK) {
                run_init(q->run, q->grid, &q->grid->slot[0], q->grid->stream, q->rtol, q->maxit);
                st = run_begin(q->run, 0);
            }
            std::lock_guard<std::mutex> lk(S.mu);
            if (st != HMG_OK) {
                S.used -= q->footprint;
                q->state = 2;
                q->result.status = st;
                q->result.t_done = hmg_now() - ctx->t0;
                if (q->grid) hmg_grid_destroy(q->grid);
                q->grid = nullptr;
                S.cv.notify_all();
            } else {
                S.active.push_back(q);
            }
        }
        std::vector<Request *> act;
        {
            std::lock_guard<std::mutex> lk(S.mu);
            act = S.active;
        }
        // keep up to two iterations of every active solve queued (the streams
        // of different requests overlap on the device), then look at each
        // one's oldest iteration without blocking: a finished request does
        // not wait behind a slow one
        for (Request *q : act)
            while (q->run.inflight < 2 && !q->cancel.load()) {
                if (run_issue(q->run) != HMG_OK) break;
            }
        bool progress = false;
        for (Request *q : act) {
            SolveRun &R = q->run;
            if (q->cancel.load()) {
                retire(ctx, q, HMG_ERR_CANCELLED);
                progress = true;
                continue;
            }
            if (R.inflight == 0) continue;
            int e = (R.issued - R.inflight) & 1;
            hipError_t qe = hipEventQuery(R.ev[e]);
            if (qe == hipErrorNotReady) continue;
            progress = true;
            if (qe != hipSuccess) {
                retire(ctx, q, HMG_ERR_DEVICE);
                continue;
            }
            R.inflight--;
            bool over = R.issued > R.maxit + 4;
            if (run_done(R) || over) {
                hmg_solve_info inf{};
                hmg_status st = run_finish(R, &inf);
                if (st == HMG_PENDING && !over) continue;
                if (st == HMG_PENDING) st = HMG_ERR_NOT_CONVERGED;
                q->result.iters = inf.iters;
                q->result.rel_res_true = inf.rel_res_true;
                retire(ctx, q, st);
            }
        }
        if (!progress && !act.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

static void server_start(hmg_ctx *ctx) {
    ServerState &S = *ctx->server;
    if (S.running) return;
    S.running = true;
    S.quit = false;
    S.worker = std::thread(server_loop, ctx);
}

static void server_stop(hmg_ctx *ctx) {
    if (!ctx->server) return;
    ServerState &S = *ctx->server;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.quit = true;
        S.cv.notify_all();
    }
    if (S.worker.joinable()) S.worker.join();
    S.running = false;
    for (auto &kv : S.all) {
        Request *q = kv.second;
        if (q->grid) hmg_grid_destroy(q->grid);
        delete q;
    }
    for (PoolEntry &e : S.pool) hmg_grid_destroy(e.grid);
    S.pool.clear();
    S.pooled = 0;
    S.all.clear();
    S.queue.clear();
    S.active.clear();
}

extern "C" hmg_status hmg_submit(hmg_ctx *ctx, const hmg_request *req, uint64_t *ticket) {
    if (!ctx || !req || !ticket || !req->k) return hmg_fail(HMG_ERR_INVALID, "null argument");
    hmg_status st = check_solve_args(req->rtol, req->maxit);
    if (st) return st;
    if (!valid_hierarchy(req->n, req->opts.coarsest_n) || !(req->h > 0.0))
        return hmg_fail(HMG_ERR_INVALID, "bad grid size or spacing");
    size_t m0 = (size_t)(req->n + 2) * (req->n + 2);
    Request *q = new Request();
    q->n = req->n;
    q->h = req->h;
    q->k.assign(req->k, req->k + m0);
    if (req->f) q->f.assign(req->f, req->f + m0);
    else q->f.assign(m0, hmg_c64{0.0, 0.0});
    q->opts = req->opts;
    q->rtol = req->rtol;
    q->maxit = req->maxit;
    q->footprint = estimate_footprint(req->n, req->opts) + (size_t)(2 * req->maxit + 2) * 8;
    q->result.t_arrive = hmg_now() - ctx->t0;
    if (q->footprint > ctx->budget) {
        size_t need = q->footprint;
        delete q;
        return hmg_fail(HMG_ERR_TOO_LARGE, "request needs %zu bytes, budget is %zu", need, ctx->budget);
    }
    ServerState &S = *ctx->server;
    std::lock_guard<std::mutex> lk(S.mu);
    if (!S.running) server_start(ctx);
    q->ticket = S.next_ticket++;
    S.all[q->ticket] = q;
    S.queue.push_back(q);
    *ticket = q->ticket;
    S.cv.notify_all();
    return HMG_OK;
}

extern "C" hmg_status hmg_poll(hmg_ctx *ctx, uint64_t ticket, hmg_c64 *x_out, hmg_result *res) {
    if (!ctx) return hmg_fail(HMG_ERR_INVALID, "null context");
    ServerState &S = *ctx->server;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return hmg_fail(HMG_ERR_UNKNOWN_TICKET, "unknown ticket %llu", (unsigned long long)ticket);
    Request *q = it->second;
    if (q->state != 2) {
        if (res) {
            *res = q->result;
            res->status = HMG_PENDING;
        }
        return HMG_PENDING;
    }
    if (res) *res = q->result;
    if (x_out && !q->x.empty()) std::memcpy(x_out, q->x.data(), q->x.size() * sizeof(hmg_c64));
    hmg_status st = (hmg_status)q->result.status;
    S.all.erase(it);
    delete q;
    return st;
}

extern "C" hmg_status hmg_cancel(hmg_ctx *ctx, uint64_t ticket) {
    if (!ctx) return hmg_fail(HMG_ERR_INVALID, "null context");
    ServerState &S = *ctx->server;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return hmg_fail(HMG_ERR_UNKNOWN_TICKET, "unknown ticket");
    it->second->cancel.store(true);
    S.cv.notify_all();
    return HMG_OK;
}

extern "C" hmg_status hmg_ctx_set_max_active(hmg_ctx *ctx, int max_active) {
    if (!ctx || max_active < 0) return hmg_fail(HMG_ERR_INVALID, "bad argument");
    std::lock_guard<std::mutex> lk(ctx->server->mu);
    ctx->server->max_active = max_active;
    return HMG_OK;
}

extern "C" int hmg_solve_history(hmg_grid *g, int rhs, double *out, int cap) {
    if (!g || rhs < 0 || rhs >= g->nrhs || (!out && cap > 0)) {
        hmg_fail(HMG_ERR_INVALID, "bad argument");
        return -1;
    }
    Slot &S = g->slot[rhs];
    if (!S.K.hist || S.last_halfsteps < 0) return 0;
    int n = std::min(S.last_halfsteps + 1, S.hist_cap);
    int m = std::min(n, cap);
    if (m > 0 && hipMemcpy(out, S.K.hist, (size_t)m * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        hmg_fail(HMG_ERR_DEVICE, "history copy failed");
        return -1;
    }
    return n;
}
