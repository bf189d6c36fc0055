/*
 * host_driver.c -- drives the host side of libhmg through its C-ABI on small
 * problems: contexts, grids of both precisions and all variants, V-cycles,
 * solves with and without an initial guess, batches, the stationary cycle
 * solver with the ray correction, the request server (admission, reuse of
 * idle grids, cancellation, budget refusal) and argument checks.  Built
 * against a copy of the library whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer; a clean exit is the test.  Test infrastructure
 * only.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#include <unistd.h>

#include "hmg.h"

#define CHECK(call, ...)                                                          \
    do {                                                                          \
        hmg_status st_ = (call);                                                  \
        int ok_ = 0;                                                              \
        hmg_status acc_[] = {__VA_ARGS__};                                        \
        for (size_t q_ = 0; q_ < sizeof acc_ / sizeof acc_[0]; ++q_)              \
            ok_ |= st_ == acc_[q_];                                               \
        if (!ok_) {                                                               \
            fprintf(stderr, "%s:%d %s -> %d (%s)\n", __FILE__, __LINE__, #call,   \
                    (int)st_, hmg_last_error());                                  \
            exit(1);                                                              \
        }                                                                         \
    } while (0)

static void problem(int n, double kh, double **k, hmg_c64 **f, int nrhs) {
    int M = n + 2;
    *k = malloc((size_t)M * M * sizeof **k);
    *f = calloc((size_t)M * M * nrhs, sizeof **f);
    double h = 1.0 / (n + 1);
    for (int j = 0; j < M; ++j)
        for (int i = 0; i < M; ++i) (*k)[j * M + i] = kh / h * (j < M / 2 ? 1.0 : 1.3);
    for (int r = 0; r < nrhs; ++r) (*f)[(size_t)r * M * M + (M / 2 + r) * M + M / 2].re = 1.0 / (h * h);
}

static void sleep_ms(int ms) {
    struct timespec ts = {0, ms * 1000000L};
    nanosleep(&ts, NULL);
}

static void grids(hmg_ctx *ctx) {
    const int n = 63, nrhs = 2;
    const size_t m = (size_t)(n + 2) * (n + 2);
    double *k;
    hmg_c64 *f;
    problem(n, 0.3, &k, &f, nrhs);
    hmg_c64 *x = calloc(m * nrhs, sizeof *x), *z = calloc(m, sizeof *z);
    hmg_solve_info info[2];
    double hist[512];
    for (int variant = HMG_SL; variant <= HMG_HYB; ++variant)
        for (int prec = HMG_FP64; prec <= HMG_MIXED; ++prec) {
            hmg_opts o;
            hmg_opts_default(&o);
            o.variant = variant;
            o.precision = prec;
            hmg_grid *g = NULL;
            CHECK(hmg_grid_create(ctx, n, 1.0 / (n + 1), k, f, nrhs, &o, &g), HMG_OK);
            hmg_plan pl;
            CHECK(hmg_grid_plan(g, &pl), HMG_OK);
            CHECK(hmg_vcycle(g, f, z), HMG_OK);
            CHECK(hmg_solve(g, NULL, x, 1e-6, 200, info), HMG_OK, HMG_ERR_NOT_CONVERGED);
            CHECK(hmg_solve(g, x, x, 1e-8, 200, info), HMG_OK, HMG_ERR_NOT_CONVERGED);
            if (hmg_solve_history(g, 1, hist, 512) < 1) exit(2);
            CHECK(hmg_grid_set_rhs(g, 1, f), HMG_OK);
            CHECK(hmg_solve(g, NULL, x, 1e-6, 2, NULL), HMG_OK, HMG_ERR_NOT_CONVERGED);
            if (hmg_grid_footprint(g) == 0) exit(2);
            hmg_grid_destroy(g);
        }
    /* batch of two grids of different sizes and options */
    hmg_opts o1, o2;
    hmg_opts_default(&o1);
    hmg_opts_default(&o2);
    o2.relax_order = HMG_ORDER_LEX;
    o2.variant = HMG_SL;
    double *k2;
    hmg_c64 *f2;
    problem(31, 0.3, &k2, &f2, 1);
    hmg_grid *gb[2] = {NULL, NULL};
    CHECK(hmg_grid_create(ctx, n, 1.0 / (n + 1), k, f, nrhs, &o1, &gb[0]), HMG_OK);
    CHECK(hmg_grid_create(ctx, 31, 1.0 / 32, k2, f2, 1, &o2, &gb[1]), HMG_OK);
    hmg_c64 *x2 = calloc((size_t)33 * 33, sizeof *x2);
    hmg_c64 *xs[2] = {x, x2};
    hmg_solve_info i2[1];
    hmg_solve_info *is[2] = {info, i2};
    CHECK(hmg_solve_batch(ctx, 2, gb, xs, 1e-6, 200, is), HMG_OK, HMG_ERR_NOT_CONVERGED);
    hmg_grid_destroy(gb[0]);
    hmg_grid_destroy(gb[1]);
    /* ray correction and the stationary cycle solver */
    hmg_opts orr;
    hmg_opts_default(&orr);
    orr.variant = HMG_HLM;
    orr.ray_n = 3;
    hmg_grid *gr = NULL;
    CHECK(hmg_grid_create(ctx, n, 1.0 / (n + 1), k, f, 1, &orr, &gr), HMG_OK);
    CHECK(hmg_solve_cycles(gr, NULL, x, 1e-6, 20, info), HMG_OK, HMG_ERR_NOT_CONVERGED);
    CHECK(hmg_solve(gr, NULL, x, 1e-6, 200, info), HMG_OK, HMG_ERR_NOT_CONVERGED);
    hmg_grid_destroy(gr);
    /* argument checks */
    hmg_grid *bad = NULL;
    CHECK(hmg_grid_create(ctx, 64, 1.0 / 65, k, f, 1, NULL, &bad), HMG_ERR_INVALID);
    CHECK(hmg_grid_create(ctx, n, -1.0, k, f, 1, NULL, &bad), HMG_ERR_INVALID);
    CHECK(hmg_solve(NULL, NULL, x, 1e-6, 10, NULL), HMG_ERR_INVALID);
    free(k); free(f); free(k2); free(f2); free(x); free(x2); free(z);
}

static void serving(hmg_ctx *ctx) {
    const int sizes[] = {63, 127, 63, 31, 127, 63};
    const int count = 6;
    double *k[6];
    hmg_c64 *f[6];
    uint64_t t[6];
    for (int q = 0; q < count; ++q) problem(sizes[q], 0.3, &k[q], &f[q], 1);
    for (int pass = 0; pass < 2; ++pass) {
        CHECK(hmg_ctx_set_max_active(ctx, pass == 0 ? 0 : 1), HMG_OK);
        for (int q = 0; q < count; ++q) {
            hmg_request r;
            memset(&r, 0, sizeof r);
            r.n = sizes[q];
            r.h = 1.0 / (sizes[q] + 1);
            r.k = k[q];
            r.f = f[q];
            hmg_opts_default(&r.opts);
            r.opts.variant = q % 3;
            r.rtol = 1e-6;
            r.maxit = 300;
            CHECK(hmg_submit(ctx, &r, &t[q]), HMG_OK);
        }
        CHECK(hmg_cancel(ctx, t[count - 1]), HMG_OK);
        int left = count;
        int done[6] = {0};
        for (int spin = 0; left > 0 && spin < 60000; ++spin) {
            for (int q = 0; q < count; ++q) {
                if (done[q]) continue;
                size_t m = (size_t)(sizes[q] + 2) * (sizes[q] + 2);
                hmg_c64 *x = malloc(m * sizeof *x);
                hmg_result res;
                hmg_status st = hmg_poll(ctx, t[q], x, &res);
                free(x);
                if (st == HMG_PENDING) continue;
                if (st != HMG_OK && st != HMG_ERR_NOT_CONVERGED && !(q == count - 1 && st == HMG_ERR_CANCELLED)) {
                    fprintf(stderr, "request %d status %d\n", q, (int)st);
                    exit(1);
                }
                done[q] = 1;
                --left;
            }
            sleep_ms(1);
        }
        if (left) {
            fprintf(stderr, "serving did not finish\n");
            exit(1);
        }
    }
    CHECK(hmg_poll(ctx, 123456789, NULL, NULL), HMG_ERR_UNKNOWN_TICKET, HMG_ERR_INVALID);
    for (int q = 0; q < count; ++q) {
        free(k[q]);
        free(f[q]);
    }
}

int main(void) {
    hmg_ctx *ctx = NULL;
    CHECK(hmg_ctx_create(0, 0, &ctx), HMG_OK);
    grids(ctx);
    serving(ctx);
    hmg_ctx_destroy(ctx);
    /* a small budget: a request larger than it is refused at submit */
    CHECK(hmg_ctx_create(0, 1 << 20, &ctx), HMG_OK);
    double *k;
    hmg_c64 *f;
    problem(255, 0.3, &k, &f, 1);
    hmg_request r;
    memset(&r, 0, sizeof r);
    r.n = 255;
    r.h = 1.0 / 256;
    r.k = k;
    r.f = f;
    hmg_opts_default(&r.opts);
    r.rtol = 1e-6;
    r.maxit = 10;
    uint64_t t;
    CHECK(hmg_submit(ctx, &r, &t), HMG_ERR_TOO_LARGE);
    hmg_ctx_destroy(ctx);
    free(k);
    free(f);
    printf("host driver done\n");
    fflush(stdout);
    /* end without the process teardown: the ROCm runtime's own unload
     * order at exit trips a check of the sanitizer's device allocator that
     * has nothing to do with this library (everything above is released) */
    _exit(0);
}
