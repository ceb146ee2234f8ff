/*
 * Plain CPU oracle for the tensor-product multigrid solve of the approximate
 * Helmholtz (pressure Schur-complement) operator of Mitchell & Mueller,
 * "High level implementation of geometric multigrid solvers for finite element
 * problems: applications in atmospheric modelling".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the obviously-correct reference the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product path never does.  It
 * shares no code with the GPU library.
 *
 * What it computes, in the paper's order:
 *   - the lumped operator H on a periodic n x n x nz column grid
 *     (Sec. 4.2, approximate Helmholtz operator with diagonal mass lumping),
 *     with the discrete scalings stated at oracle_create below;
 *   - coarse operators by rediscretisation on horizontally coarsened grids
 *     (Sec. 3.3 and Sec. 4.2.1: semi-coarsening, columns kept intact);
 *   - the vertical line smoother (Sec. 4.2, block-Jacobi with H_z) solved by
 *     the Thomas algorithm (Sec. 4.3.1);
 *   - restriction/prolongation by the natural embedding (Sec. 3.2);
 *   - the V-cycle (Sec. 3, two-grid cycle applied recursively);
 *   - an outer preconditioned CG on H (standard or flexible beta), with the
 *     V-cycle in double or in float;
 *   - the adjoint face gradient dJ/dc_f = -gamma_f (lambda_p - lambda_q)(x_p - x_q);
 *   - the velocity-pressure system around it, its Schur-complement
 *     preconditioner and the outer flexible GMRES (oracle_mixed.inc);
 *   - the next-to-lowest-order DG1 pressure level with its banded-LU line
 *     smoother and the p-coarsening to the lowest-order hierarchy
 *     (oracle_dg1.inc).
 *
 * Dot products accumulate in long double.  Loops over columns and vector
 * entries run as OpenMP `parallel for` when built with -fopenmp; nothing
 * depends on the thread count (dot products sum fixed blocks in order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_LEVELS 16

#define REAL double
#define SFX d
#include "oracle_level.inc"
#undef REAL
#undef SFX

#define REAL float
#define SFX f
#include "oracle_level.inc"
#undef REAL
#undef SFX

typedef struct {
    int n, nz, nlevels;
    double a_h, a_z;
    double *s;        /* [nz]   relative cell height s_k = dz_k / mean(dz)           */
    double *t;        /* [nz-1] relative face distance t_{k+1/2} = (s_k + s_{k+1})/2  */
    hier_d hd;        /* double hierarchy (the definition)                          */
    hier_f hf;        /* float copy, rounded from the double one                    */
} oracle_problem;

static long ncell(int n, int nz) { return (long)n * n * nz; }

static void free_level_d(level_d *L)
{
    free(L->cE); free(L->cN); free(L->cU); free(L->mu); free(L->wh); free(L->wz); free(L->chol);
}
static void free_level_f(level_f *L)
{
    free(L->cE); free(L->cN); free(L->cU); free(L->mu); free(L->wh); free(L->wz); free(L->chol);
}

void oracle_destroy(oracle_problem *P)
{
    if (!P) return;
    for (int l = 0; l < P->nlevels; ++l) {
        free_level_d(&P->hd.lev[l]);
        free_level_f(&P->hf.lev[l]);
    }
    free(P->s);
    free(P->t);
    free(P);
}

/*
 * Build the hierarchy.
 *
 * Discrete operator on level l (n_l = n / 2^l columns per side):
 *   mass        mu_{l,k} = 4^l s_k                 (M3 ~ cell volume)
 *   horizontal  w_f = a_h s_k c_f                  (face area^2 / lumped mass ~ dz)
 *   vertical    w_f = 4^l a_z c_f / t_{k+1/2}       (face area^2 / lumped mass ~ dx^2/dz)
 * which is the lumped form of H = M3 + w_c^2 (D_h M_inv^h D_h^T +
 * (1+w_N^2)^{-1} D_z M_inv^z D_z^T) for piecewise-constant pressure, with the
 * constant factors folded into a_h and a_z.
 *
 * Coarse face coefficients (rediscretisation with variable c_f): the mean of
 * the fine faces covering the coarse face.
 *
 * The graded-spacing scaling (s_k, t_{k+1/2}) and the face-mean coarsening
 * are readings of a paper that treats constant coefficients and no grading.
 * The scaling is pinned by finite-volume identities (exact fluxes of linear
 * profiles, horizontal Fourier modes on graded columns); the face-mean
 * coarsening is parity unpinned against the paper beyond the uniform limit
 * (closed-form spectrum) and the exact Galerkin relation of the coarse
 * operators.
 *
 * Inputs: cE, cN, cU in column-contiguous order for level 0; dz may be NULL
 * (uniform).  Returns NULL on invalid input.
 */
oracle_problem *oracle_create(int n, int nz, int nlevels, double a_h, double a_z, const double *dz,
                              const double *cE, const double *cN, const double *cU,
                              int nu_pre, int nu_post, double omega, int direct, int n_coarse)
{
    if (n < 1 || nz < 1 || nlevels < 1 || nlevels > OR_MAX_LEVELS) return NULL;
    if (n % (1 << (nlevels - 1)) != 0) return NULL;
    oracle_problem *P = (oracle_problem *)calloc(1, sizeof(oracle_problem));
    P->n = n; P->nz = nz; P->nlevels = nlevels; P->a_h = a_h; P->a_z = a_z;
    P->s = (double *)malloc(sizeof(double) * nz);
    P->t = (double *)malloc(sizeof(double) * (nz > 1 ? nz - 1 : 1));
    double mean = 0;
    for (int k = 0; k < nz; ++k) mean += dz ? dz[k] : 1.0;
    mean /= nz;
    for (int k = 0; k < nz; ++k) P->s[k] = (dz ? dz[k] : 1.0) / mean;
    for (int k = 0; k + 1 < nz; ++k) P->t[k] = 0.5 * (P->s[k] + P->s[k + 1]);

    hier_d *H = &P->hd;
    H->nlevels = nlevels; H->nu_pre = nu_pre; H->nu_post = nu_post;
    H->direct = direct; H->n_coarse = n_coarse; H->omega = omega;
    for (int l = 0; l < nlevels; ++l) {
        level_d *L = &H->lev[l];
        L->n = n >> l;
        L->nz = nz;
        long m = ncell(L->n, nz);
        L->cE = (double *)malloc(sizeof(double) * m);
        L->cN = (double *)malloc(sizeof(double) * m);
        L->cU = (double *)malloc(sizeof(double) * m);
        L->mu = (double *)malloc(sizeof(double) * nz);
        L->wh = (double *)malloc(sizeof(double) * nz);
        L->wz = (double *)malloc(sizeof(double) * nz);
        double four_l = ldexp(1.0, 2 * l);
        for (int k = 0; k < nz; ++k) {
            L->mu[k] = four_l * P->s[k];
            L->wh[k] = a_h * P->s[k];
            L->wz[k] = (k + 1 < nz) ? four_l * a_z / P->t[k] : 0.0;
        }
        if (l == 0) {
            memcpy(L->cE, cE, sizeof(double) * m);
            memcpy(L->cN, cN, sizeof(double) * m);
            memcpy(L->cU, cU, sizeof(double) * m);
        } else {
            const level_d *Fi = &H->lev[l - 1];
#pragma omp parallel for schedule(static)
            for (int J = 0; J < L->n; ++J)
                for (int I = 0; I < L->n; ++I)
                    for (int k = 0; k < nz; ++k) {
                        long p = at_d(L, I, J, k);
                        /* east face of (I,J): fine east faces of (2I+1, 2J) and (2I+1, 2J+1) */
                        L->cE[p] = 0.5 * (Fi->cE[at_d(Fi, 2 * I + 1, 2 * J, k)] +
                                          Fi->cE[at_d(Fi, 2 * I + 1, 2 * J + 1, k)]);
                        /* north face of (I,J): fine north faces of (2I, 2J+1) and (2I+1, 2J+1) */
                        L->cN[p] = 0.5 * (Fi->cN[at_d(Fi, 2 * I, 2 * J + 1, k)] +
                                          Fi->cN[at_d(Fi, 2 * I + 1, 2 * J + 1, k)]);
                        /* upper face: the four children's upper faces */
                        L->cU[p] = 0.25 * (Fi->cU[at_d(Fi, 2 * I, 2 * J, k)] +
                                           Fi->cU[at_d(Fi, 2 * I + 1, 2 * J, k)] +
                                           Fi->cU[at_d(Fi, 2 * I, 2 * J + 1, k)] +
                                           Fi->cU[at_d(Fi, 2 * I + 1, 2 * J + 1, k)]);
                    }
        }
    }

    /* float copy: every array rounded from the double hierarchy */
    hier_f *G = &P->hf;
    G->nlevels = nlevels; G->nu_pre = nu_pre; G->nu_post = nu_post;
    G->direct = direct; G->n_coarse = n_coarse; G->omega = (float)omega;
    for (int l = 0; l < nlevels; ++l) {
        level_d *L = &H->lev[l];
        level_f *M = &G->lev[l];
        M->n = L->n; M->nz = nz;
        long m = ncell(L->n, nz);
        M->cE = (float *)malloc(sizeof(float) * m);
        M->cN = (float *)malloc(sizeof(float) * m);
        M->cU = (float *)malloc(sizeof(float) * m);
        M->mu = (float *)malloc(sizeof(float) * nz);
        M->wh = (float *)malloc(sizeof(float) * nz);
        M->wz = (float *)malloc(sizeof(float) * nz);
#pragma omp parallel for schedule(static)
        for (long p = 0; p < m; ++p) {
            M->cE[p] = (float)L->cE[p];
            M->cN[p] = (float)L->cN[p];
            M->cU[p] = (float)L->cU[p];
        }
        for (int k = 0; k < nz; ++k) {
            M->mu[k] = (float)L->mu[k];
            M->wh[k] = (float)L->wh[k];
            M->wz[k] = (float)L->wz[k];
        }
    }

    if (direct) {
        level_d *L = &H->lev[nlevels - 1];
        level_f *M = &G->lev[nlevels - 1];
        long m = ncell(L->n, nz);
        if (m > 8192) { oracle_destroy(P); return NULL; }
        L->chol = (double *)malloc(sizeof(double) * m * m);
        dense_d(L, L->chol);
        M->chol = (float *)malloc(sizeof(float) * m * m);
        dense_f(M, M->chol);
        if (cholesky_d(L->chol, (int)m) != 0 || cholesky_f(M->chol, (int)m) != 0) {
            oracle_destroy(P);
            return NULL;
        }
    }
    return P;
}

int oracle_level_n(const oracle_problem *P, int l) { return P->hd.lev[l].n; }

/* Threads for the OpenMP loops (n <= 0 leaves the setting alone); the number
 * the next parallel loop will use. */
int oracle_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

void oracle_get_coeffs(const oracle_problem *P, int l, double *cE, double *cN, double *cU)
{
    const level_d *L = &P->hd.lev[l];
    long m = ncell(L->n, L->nz);
    memcpy(cE, L->cE, sizeof(double) * m);
    memcpy(cN, L->cN, sizeof(double) * m);
    memcpy(cU, L->cU, sizeof(double) * m);
}

void oracle_apply(const oracle_problem *P, int l, const double *x, double *y) { apply_d(&P->hd.lev[l], x, y); }
void oracle_apply_f(const oracle_problem *P, int l, const float *x, float *y) { apply_f(&P->hf.lev[l], x, y); }
void oracle_line_solve(const oracle_problem *P, int l, const double *r, double *x) { line_solve_d(&P->hd.lev[l], r, x); }
void oracle_line_solve_f(const oracle_problem *P, int l, const float *r, float *x) { line_solve_f(&P->hf.lev[l], r, x); }
void oracle_smooth(const oracle_problem *P, int l, const double *u, const double *b, double *u_out)
{
    smooth_d(&P->hd.lev[l], P->hd.omega, u, b, u_out);
}
void oracle_smooth_f(const oracle_problem *P, int l, const float *u, const float *b, float *u_out)
{
    smooth_f(&P->hf.lev[l], P->hf.omega, u, b, u_out);
}
void oracle_restrict(const oracle_problem *P, int l, const double *rf, double *bc)
{
    restrict_sum_d(&P->hd.lev[l], &P->hd.lev[l + 1], rf, bc);
}
void oracle_restrict_f(const oracle_problem *P, int l, const float *rf, float *bc)
{
    restrict_sum_f(&P->hf.lev[l], &P->hf.lev[l + 1], rf, bc);
}
void oracle_prolong_add(const oracle_problem *P, int l, const double *ec, double *uf)
{
    prolong_add_d(&P->hd.lev[l], &P->hd.lev[l + 1], ec, uf);
}
void oracle_prolong_add_f(const oracle_problem *P, int l, const float *ec, float *uf)
{
    prolong_add_f(&P->hf.lev[l], &P->hf.lev[l + 1], ec, uf);
}
void oracle_coarse_solve(const oracle_problem *P, const double *b, double *u) { coarse_solve_d(&P->hd, b, u); }
void oracle_coarse_solve_f(const oracle_problem *P, const float *b, float *u) { coarse_solve_f(&P->hf, b, u); }
void oracle_vcycle(const oracle_problem *P, const double *b, double *z) { vcycle_d(&P->hd, 0, b, z); }
void oracle_vcycle_f(const oracle_problem *P, const float *b, float *z) { vcycle_f(&P->hf, 0, b, z); }
void oracle_dense(const oracle_problem *P, int l, double *A) { dense_d(&P->hd.lev[l], A); }

/*
 * (a, b) accumulated in long double: the entries are summed in fixed blocks
 * of DOT_BLOCK consecutive products, then the block sums in order, so the
 * result does not depend on the number of threads.
 */
#define DOT_BLOCK 4096
static double dot(const double *a, const double *b, long m)
{
    long nb = (m + DOT_BLOCK - 1) / DOT_BLOCK;
    long double *part = (long double *)malloc(sizeof(long double) * (size_t)(nb > 0 ? nb : 1));
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nb; ++q) {
        long double s = 0;
        long hi = (q + 1) * DOT_BLOCK < m ? (q + 1) * DOT_BLOCK : m;
        for (long p = q * DOT_BLOCK; p < hi; ++p) s += (long double)a[p] * (long double)b[p];
        part[q] = s;
    }
    long double s = 0;
    for (long q = 0; q < nb; ++q) s += part[q];
    free(part);
    return (double)s;
}

/*
 * z = V(r): the double V-cycle, or the float V-cycle on fl32(r) returned as
 * double, with damping omega in every sweep.
 */
static void precondition_omega(const oracle_problem *P, int mixed, double omega, const double *r, double *z,
                               float *r32, float *z32, long m)
{
    if (!mixed) {
        hier_d H = P->hd;
        H.omega = omega;
        vcycle_d(&H, 0, r, z);
        return;
    }
    hier_f G = P->hf;
    G.omega = (float)omega;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < m; ++p) r32[p] = (float)r[p];
    vcycle_f(&G, 0, r32, z32);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < m; ++p) z[p] = (double)z32[p];
}

static void precondition(const oracle_problem *P, int mixed, const double *r, double *z, float *r32, float *z32, long m)
{
    precondition_omega(P, mixed, P->hd.omega, r, z, r32, z32, m);
}

/*
 * Preconditioned CG on H x = b with one V-cycle as preconditioner.
 *   r = b - H x0, z = V r, p = z
 *   repeat: q = H p; alpha = (r,z)/(p,q); x += alpha p; r -= alpha q;
 *           stop when ||r|| <= rtol ||b||;
 *           z_new = V r;
 *           standard: beta = (r,z_new)/(r_old,z_old);
 *           flexible: beta = -(z_new, q)/(p, q), the choice that makes the new
 *             direction H-conjugate to the last one whatever the
 *             preconditioner did (flexible CG with one stored direction,
 *             FCG(1) of Notay 2000; equal to (z_new, r - r_old)/(r_old, z_old));
 *           p = z_new + beta p
 * Sec. 5 notes that a preconditioner that changes between iterations needs
 * a flexible Krylov method; the FP32 V-cycle is such a preconditioner.
 *
 * omega_alt > 0 makes the preconditioner deliberately variable: the
 * applications of V with an odd index (the first is index 0) use the damping
 * omega_alt instead of the hierarchy's omega.  This exercises the flexible
 * recurrence with an SPD preconditioner that changes between iterations.
 *
 * Returns the number of iterations (applications of H to p), or -1 when the
 * iteration limit was reached, -2 on breakdown.  history[0..it] holds
 * ||r_i|| / ||b|| when non-NULL; info = {rel_residual, true_rel_residual,
 * iterations}.  When trace_p / trace_r are non-NULL (each maxit * m values)
 * they receive, for iteration i = 1, 2, ..., the direction p it used and the
 * residual r after its update, at offset (i - 1) * m.
 */
int oracle_pcg(const oracle_problem *P, const double *b, double *x, double rtol, int maxit,
               int x0_nonzero, int mixed, int flexible, double omega_alt, double *history, double *info,
               double *trace_p, double *trace_r)
{
    const level_d *L = &P->hd.lev[0];
    long m = ncell(L->n, L->nz);
    double *r = (double *)malloc(sizeof(double) * m);
    double *z = (double *)malloc(sizeof(double) * m);
    double *p = (double *)malloc(sizeof(double) * m);
    double *q = (double *)malloc(sizeof(double) * m);
    float *r32 = mixed ? (float *)malloc(sizeof(float) * m) : NULL;
    float *z32 = mixed ? (float *)malloc(sizeof(float) * m) : NULL;
    int status = -1, it = 0, napply = 0;
#define OMEGA_NEXT() ((omega_alt > 0 && (napply++ % 2) == 1) ? omega_alt : P->hd.omega)

    if (x0_nonzero) {
        apply_d(L, x, q);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < m; ++i) r[i] = b[i] - q[i];
    } else {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < m; ++i) { x[i] = 0; r[i] = b[i]; }
    }
    double bnorm = sqrt(dot(b, b, m));
    double rnorm = sqrt(dot(r, r, m));
    double rel = bnorm > 0 ? rnorm / bnorm : 0;
    if (history) history[0] = rel;
    if (bnorm == 0 || rnorm <= rtol * bnorm) {
        if (bnorm == 0) for (long i = 0; i < m; ++i) x[i] = 0;
        status = 0;
        goto done;
    }
    precondition_omega(P, mixed, OMEGA_NEXT(), r, z, r32, z32, m);
    memcpy(p, z, sizeof(double) * m);
    double rz = dot(r, z, m);
    for (it = 1; it <= maxit; ++it) {
        apply_d(L, p, q);
        double pq = dot(p, q, m);
        if (!(pq > 0) || !isfinite(rz)) { status = -2; break; }
        double alpha = rz / pq;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < m; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        if (trace_p) memcpy(trace_p + (long)(it - 1) * m, p, sizeof(double) * m);
        if (trace_r) memcpy(trace_r + (long)(it - 1) * m, r, sizeof(double) * m);
        rnorm = sqrt(dot(r, r, m));
        rel = rnorm / bnorm;
        if (history) history[it] = rel;
        if (rnorm <= rtol * bnorm) { status = it; break; }
        if (it == maxit) break;
        precondition_omega(P, mixed, OMEGA_NEXT(), r, z, r32, z32, m);
        double rz_new = dot(r, z, m);
        double beta = flexible ? -dot(z, q, m) / pq : rz_new / rz;
        rz = rz_new;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < m; ++i) p[i] = z[i] + beta * p[i];
    }
#undef OMEGA_NEXT
    if (it > maxit) it = maxit;
done:
    if (info) {
        apply_d(L, x, q);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < m; ++i) q[i] = b[i] - q[i];
        info[0] = rel;
        info[1] = bnorm > 0 ? sqrt(dot(q, q, m)) / bnorm : 0;
        info[2] = it;
    }
    free(r); free(z); free(p); free(q); free(r32); free(z32);
    return status;
}

/*
 * Adjoint face gradient of J(x(c)) with H(c) x = b and lambda = H^{-1} dJ/dx
 * (H is symmetric): dJ/dc_f = -lambda^T (dH/dc_f) x = -gamma_f (lambda_p - lambda_q)(x_p - x_q),
 * gamma_f = dw_f/dc_f on the finest level (a_h s_k horizontally, a_z / t_{k+1/2}
 * vertically).  The U slot above the top cell holds no face and gets 0.
 */
void oracle_face_gradient(const oracle_problem *P, const double *lam, const double *x,
                          double *gE, double *gN, double *gU)
{
    const level_d *L = &P->hd.lev[0];
#pragma omp parallel for schedule(static)
    for (int j = 0; j < L->n; ++j)
        for (int i = 0; i < L->n; ++i)
            for (int k = 0; k < L->nz; ++k) {
                long p = at_d(L, i, j, k);
                long e = at_d(L, i + 1, j, k), nn = at_d(L, i, j + 1, k);
                gE[p] = -L->wh[k] * (lam[p] - lam[e]) * (x[p] - x[e]);
                gN[p] = -L->wh[k] * (lam[p] - lam[nn]) * (x[p] - x[nn]);
                if (k + 1 < L->nz) {
                    long u = at_d(L, i, j, k + 1);
                    gU[p] = -L->wz[k] * (lam[p] - lam[u]) * (x[p] - x[u]);
                } else {
                    gU[p] = 0.0;
                }
            }
}

#include "oracle_mixed.inc"

#include "oracle_dg1.inc"
