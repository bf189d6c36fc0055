/*
 * oracle_driver.c -- runs every entry point of the CPU oracle once on small
 * grids, for a build under AddressSanitizer and UndefinedBehaviorSanitizer.
 * A clean exit (status 0, no sanitizer report) is the test; the numbers are
 * checked elsewhere.  Test infrastructure only.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "hmg_oracle.h"

static unsigned long long rng_state = 88172645463325252ull;
static double urand(void) {   /* xorshift64, uniform in [0, 1) */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void layered_k(int n, double k0, double *k) {
    int M = n + 2;
    for (int j = 0; j < M; ++j)
        for (int i = 0; i < M; ++i) k[j * M + i] = k0 * (j < M / 2 ? 1.0 : 1.4) * (1.0 + 0.05 * (i % 3));
}

static orc_cplx *cfield(int n, int random) {
    size_t m = (size_t)(n + 2) * (n + 2);
    orc_cplx *a = calloc(m, sizeof *a);
    if (!a) exit(2);
    if (random)
        for (size_t p = 0; p < m; ++p) a[p] = (urand() - 0.5) + I * (urand() - 0.5);
    return a;
}

static void singles(int n, double h, const double *k) {
    size_t m = (size_t)(n + 2) * (n + 2);
    orc_cplx *u = cfield(n, 1), *f = cfield(n, 1), *o = cfield(n, 0);
    orc_apply(n, h, k, 0.0, u, o);
    orc_residual(n, h, k, 0.5, f, u, o);
    orc_gs_lex(n, h, k, 0.5, f, u);
    orc_gs_rb(n, h, k, 0.0, f, u);
    orc_kacz_lex(n, h, k, 0.0, f, u);
    orc_kacz_5c(n, h, k, 0.5, f, u);
    int nc = (n - 1) / 2;
    orc_cplx *fc = cfield(nc, 0);
    double *kc = malloc((size_t)(nc + 2) * (nc + 2) * sizeof *kc);
    orc_restrict_fw(n, o, fc);
    orc_prolong_add(nc, fc, u);
    orc_inject_k(n, k, kc);
    if (n <= 15) {
        orc_cplx *A = malloc(m * m * sizeof *A);
        int *piv = malloc(m * sizeof *piv);
        orc_dense(n, h, k, 0.5, A);
        if (orc_lu_factor((int)m, A, piv) != 0) exit(3);
        orc_lu_solve((int)m, A, piv, f);
        free(A);
        free(piv);
    }
    free(u); free(f); free(o); free(fc); free(kc);
}

static void solves(int n, double h, const double *k, int variant, int order) {
    size_t m = (size_t)(n + 2) * (n + 2);
    orc_opts o;
    orc_opts_default(&o);
    o.variant = variant;
    o.gs_order = o.kacz_order = order;
    orc_grid *g = orc_grid_create(n, h, k, &o);
    if (!g) exit(4);
    orc_plan pl;
    orc_grid_plan(g, &pl);
    orc_cplx *f = cfield(n, 1), *x = cfield(n, 0);
    double hist[4096];
    orc_info info;
    orc_vcycle(g, f, x);
    orc_bicgstab(g, f, x, 1e-6, 60, ORC_PREC_VCYCLE, &info, hist, 4096);
    orc_bicgstab_ex2(g, f, x, 1e-8, 40, ORC_PREC_VCYCLE, &info, hist, 4096, 3, 5, 0);
    orc_bicgstab_ex2(g, f, x, 1e-8, 40, ORC_PREC_VCYCLE, &info, hist, 4096, 0, 0, 4);
    orc_bicgstab_ex(g, f, x, 1e-6, 30, ORC_PREC_NONE, &info, hist, 64, 2);
    if (n <= 15) orc_bicgstab(g, f, x, 1e-10, 10, ORC_PREC_EXACT, &info, hist, 4096);
    orc_grid_set_mixed_ex(g, ORC_MIX_FUSED, 2, 7, 1, 1);
    orc_vcycle(g, f, x);
    orc_grid_set_mixed(g, ORC_MIX_ONEPASS, 1, 0, 0);
    orc_vcycle(g, f, x);
    orc_grid_set_mixed(g, ORC_MIX_OFF, 1, 0, 0);
    if (pl.nlev > 1) orc_grid_override_level(g, 0, ORC_SM_KACZ, 0.0, 0.0, 2, 2);
    orc_vcycle(g, f, x);
    if (orc_grid_set_ray(g, 3) == 0) {
        orc_ray_correct(g, f, x);
        orc_cycles(g, f, x, 1e-6, 5, hist);
        orc_bicgstab(g, f, x, 1e-6, 20, ORC_PREC_VCYCLE, &info, hist, 4096);
        orc_grid_set_ray(g, 0);
    }
    (void)m;
    free(f); free(x);
    orc_grid_destroy(g);
}

int main(void) {
    const int sizes[] = {7, 15, 31};
    for (int s = 0; s < 3; ++s) {
        int n = sizes[s];
        double h = 1.0 / (n + 1);
        double *k = malloc((size_t)(n + 2) * (n + 2) * sizeof *k);
        layered_k(n, 0.6 / h, k);
        singles(n, h, k);
        for (int v = ORC_SL; v <= ORC_HYB; ++v)
            for (int order = 0; order < 2; ++order) solves(n, h, k, v, order);
        free(k);
    }
    printf("oracle driver done\n");
    return 0;
}
