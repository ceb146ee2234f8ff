/*
 * Drives every entry point of the CPU oracle on small grids, for a build
 * with the address and undefined-behaviour sanitizers (test infrastructure:
 * compiled and run by tests/test_oracle_sanitize.py on the CPU).  Exits 0 when
 * every solve converges; the sanitizers abort on any invalid access.
 */
#include "../oracle/tpmg_oracle.c"

#include <stdio.h>

static unsigned long long g_state = 0x9E3779B97F4A7C15ull;
static double urand(void)
{
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static int check(int cond, const char *what)
{
    if (!cond) fprintf(stderr, "FAILED: %s\n", what);
    return cond ? 0 : 1;
}

static int run_case(int n, int nz, int levels, int direct, int graded)
{
    long m = (long)n * n * nz;
    double *c = (double *)malloc(sizeof(double) * 3 * m), *dz = (double *)malloc(sizeof(double) * nz);
    double *b = (double *)malloc(sizeof(double) * m), *x = (double *)malloc(sizeof(double) * m);
    double *y = (double *)malloc(sizeof(double) * m), *lam = (double *)malloc(sizeof(double) * m);
    float *bf = (float *)malloc(sizeof(float) * m), *yf = (float *)malloc(sizeof(float) * m);
    double *g = (double *)malloc(sizeof(double) * 3 * m);
    int bad = 0;
    for (long p = 0; p < 3 * m; ++p) c[p] = 1.0 + 0.5 * urand();
    for (int k = 0; k < nz; ++k) dz[k] = graded ? pow(1.05, k) : 1.0;
    for (long p = 0; p < m; ++p) { b[p] = urand() - 0.5; bf[p] = (float)b[p]; }
    oracle_problem *P = oracle_create(n, nz, levels, 1.0, 100.0, graded ? dz : NULL, c, c + m, c + 2 * m, 2, 2, 0.8,
                                      direct, 2);
    if (!P) { fprintf(stderr, "oracle_create failed\n"); return 1; }
    for (int l = 0; l < levels; ++l) {
        long ml = (long)oracle_level_n(P, l) * oracle_level_n(P, l) * nz;
        double *cl = (double *)malloc(sizeof(double) * 3 * ml);
        oracle_get_coeffs(P, l, cl, cl + ml, cl + 2 * ml);
        oracle_apply(P, l, b, y);
        oracle_apply_f(P, l, bf, yf);
        oracle_line_solve(P, l, b, y);
        oracle_line_solve_f(P, l, bf, yf);
        oracle_smooth(P, l, b, b, y);
        oracle_smooth_f(P, l, bf, bf, yf);
        if (l + 1 < levels) {
            oracle_restrict(P, l, b, y);
            oracle_restrict_f(P, l, bf, yf);
            memcpy(x, b, sizeof(double) * ml);
            oracle_prolong_add(P, l, y, x);
        }
        free(cl);
    }
    {
        long ml = (long)oracle_level_n(P, levels - 1) * oracle_level_n(P, levels - 1) * nz;
        double *A = (double *)malloc(sizeof(double) * ml * ml);
        oracle_dense(P, levels - 1, A);
        oracle_coarse_solve(P, b, y);
        oracle_coarse_solve_f(P, bf, yf);
        free(A);
    }
    oracle_vcycle(P, b, y);
    oracle_vcycle_f(P, bf, yf);
    double info[3], hist[201];
    int maxit = 200;
    double *tp = (double *)malloc(sizeof(double) * maxit * m), *tr = (double *)malloc(sizeof(double) * maxit * m);
    for (int mixed = 0; mixed <= 1; ++mixed)
        for (int flex = 0; flex <= 1; ++flex)
            for (int alt = 0; alt <= 1; ++alt) {
                int st = oracle_pcg(P, b, x, 1e-10, maxit, 0, mixed, flex, alt ? 0.4 : 0.0, hist, info, tp, tr);
                bad += check(st >= 0 && info[1] <= 2e-10, "pcg converged");
            }
    bad += check(oracle_pcg(P, b, x, 1e-12, maxit, 1, 0, 0, 0.0, NULL, info, NULL, NULL) >= 0, "pcg from x0");
    oracle_pcg(P, x, lam, 1e-10, maxit, 0, 0, 0, 0.0, NULL, NULL, NULL, NULL);
    oracle_face_gradient(P, lam, x, g, g + m, g + 2 * m);
    if (n >= 2) {
        double *mb = (double *)malloc(sizeof(double) * 4 * m), *mx = (double *)malloc(sizeof(double) * 4 * m);
        double *my = (double *)malloc(sizeof(double) * 4 * m);
        for (long p = 0; p < 4 * m; ++p) mb[p] = urand() - 0.5;
        for (long p = 0; p < m; ++p)
            if (p % nz == nz - 1) mb[2 * m + p] = 0.0;   /* no face above the top cell */
        oracle_mixed_apply(P, mb, my);
        oracle_mixed_precondition(P, 0, mb, my);
        oracle_mixed_precondition(P, 1, mb, my);
        int st = oracle_mixed_fgmres(P, mb, mx, 1e-8, 5, 300, 1, hist, info);
        bad += check(st >= 0 && info[1] <= 1e-7, "fgmres converged");
        free(mb); free(mx); free(my);
    }
    if (nz >= 2) {
        /* next-to-lowest order: the DG1 level over this hierarchy */
        oracle_dg1 *G = oracle_dg1_create(P);
        if (!G) { fprintf(stderr, "oracle_dg1_create failed\n"); return bad + 1; }
        long M1 = 6 * m, mc = 6 * nz;
        double *u1 = (double *)malloc(sizeof(double) * M1), *b1 = (double *)malloc(sizeof(double) * M1);
        double *y1 = (double *)malloc(sizeof(double) * M1), *e0 = (double *)malloc(sizeof(double) * m);
        double *blk = (double *)malloc(sizeof(double) * mc * mc);
        double *F = (double *)malloc(sizeof(double) * (long)n * n * mc * DG1_NF);
        for (long p = 0; p < M1; ++p) { u1[p] = urand() - 0.5; b1[p] = urand() - 0.5; }
        oracle_dg1_apply(G, u1, y1);
        oracle_dg1_line_solve(G, b1, y1);
        oracle_dg1_smooth(G, NULL, b1, y1);
        oracle_dg1_smooth(G, u1, b1, y1);
        oracle_dg1_restrict(G, b1, e0);
        oracle_dg1_prolong_add(G, e0, u1);
        oracle_dg1_column_block(G, n - 1, 0, blk);
        oracle_dg1_factors(G, F);
        oracle_dg1_vcycle(G, b1, y1);
        if (M1 <= 1200) {
            double *A1 = (double *)malloc(sizeof(double) * M1 * M1);
            oracle_dg1_dense(G, A1);
            free(A1);
        }
        int st = oracle_dg1_pcg(G, b1, u1, 1e-10, 300, hist, info);
        bad += check(st >= 0 && info[1] <= 2e-10, "dg1 pcg converged");
        oracle_dg1_destroy(G);
        free(u1); free(b1); free(y1); free(e0); free(blk); free(F);
    }
    oracle_destroy(P);
    free(c); free(dz); free(b); free(x); free(y); free(lam); free(bf); free(yf); free(g); free(tp); free(tr);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad += run_case(8, 5, 3, 1, 0);
    bad += run_case(8, 7, 2, 0, 1);
    bad += run_case(12, 3, 3, 0, 1);
    bad += run_case(4, 1, 1, 1, 0);
    bad += run_case(2, 4, 2, 1, 1);
    printf(bad ? "oracle sanitize driver: %d failures\n" : "oracle sanitize driver: ok\n", bad);
    return bad ? 1 : 0;
}
