/*
 * tpmg.h -- C interface of libtpmg: tensor-product geometric multigrid for the
 * strongly anisotropic pressure (Schur-complement) equation on thin extruded
 * meshes, after Mitchell & Mueller, "High level implementation of geometric
 * multigrid solvers for finite element problems: applications in atmospheric
 * modelling" (arXiv:1605.00492).  Hand-written HIP kernels for gfx950 (MI355X).
 *
 * PROBLEM (Sec. 4.2, the approximate Helmholtz operator with diagonally
 * lumped velocity mass).  Pressure is piecewise constant on a periodic n x n
 * grid of vertical columns, nz cells per column.  With s_k = dz_k / mean(dz)
 * and t_{k+1/2} = (s_k + s_{k+1})/2, multigrid level l (n_l = n / 2^l columns
 * per side, nz unchanged: horizontal semi-coarsening, Sec. 4.2.1) applies
 *     (H_l x)_p = mu_{l,k} x_p + sum over faces f of p:  w_f (x_p - x_q(f))
 *     mu_{l,k} = 4^l s_k
 *     east/north faces:  w_f = a_h s_k c_f
 *     upper faces (k < nz-1):  w_f = 4^l a_z c_f / t_{k+1/2}
 * No face lies below k = 0 or above k = nz-1 (u.n = 0 top and bottom,
 * Sec. 4.1).  Level-0 face coefficients c_f > 0 are the input; a coarse face
 * takes the mean of the fine faces covering it (rediscretisation, Sec. 3.3).
 *
 * METHOD.  Preconditioned CG on H_0 (FP64), preconditioned by one V-cycle
 * (Sec. 3, two-grid cycle applied recursively) whose smoother is the damped
 * vertical line relaxation u <- u + omega H_z^{-1}(b - H u) (Sec. 4.2),
 * H_z being the column-block part of H (tridiagonal, solved exactly per
 * column, Sec. 4.3.1).  Restriction sums the four horizontal children,
 * prolongation injects (natural embedding, Sec. 3.2).  The V-cycle may run in
 * FP32 while the outer CG stays FP64.
 *
 * LAYOUTS of device arrays:
 *   TPMG_LAYOUT_LEVEL_MAJOR  cells x[k][j][i], faces c[f][k][j][i]
 *   TPMG_LAYOUT_COLUMN_MAJOR (Sec. 4.3 ordering) cells x[j][i][k], faces c[j][i][k][f]
 * with i fastest in level-major, f in {E=0, N=1, U=2}.  Internally every
 * level is stored in tiles of 64 columns (col = j*n + i) whose nz levels are
 * contiguous, when n*n is a multiple of 64 (otherwise level-major); entry
 * points convert the caller's arrays on the way in and out.  The E face of cell
 * (i,j,k) joins (i+1 mod n, j, k), the N face joins (i, j+1 mod n, k), the U
 * face joins (i, j, k+1); the U slot of the top cell holds no face (its value
 * is ignored on input and its gradient is 0).
 *
 * OWNERSHIP.  The caller owns every device buffer, including the workspace
 * (at least tpmg_workspace_bytes bytes, 256-byte aligned).  The library
 * allocates no device memory.  A hierarchy handle aliases its workspace: free
 * the workspace only after tpmg_destroy.  Handles are not thread-safe;
 * different handles are independent.  Buffers passed to one call must not
 * alias each other unless stated.
 *
 * STREAMS.  `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  All work is queued on it.  apply/vcycle/smooth/restrict/
 * prolong/coarse/face_gradient are asynchronous; setup and solve synchronise
 * the stream (setup for validation and the optional host factorisation,
 * solve for its convergence tests).
 *
 * ERRORS.  Every call returns a tpmg_status; nothing throws across the
 * interface.  Arguments are validated on the host before any launch.
 * TPMG_ERR_DEVICE carries the HIP error text in tpmg_last_error().
 */
#ifndef TPMG_H
#define TPMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TPMG_OK = 0,
    TPMG_NOT_CONVERGED = 1,      /* warning: x holds the last iterate, info is filled  */
    TPMG_ERR_INVALID_ARG = -1,   /* NULL pointer, bad enum, bad parameter value        */
    TPMG_ERR_SHAPE = -2,         /* n, nz, nlevels inconsistent or out of range        */
    TPMG_ERR_NOT_SPD = -3,       /* a face coefficient or dz is not positive and finite */
    TPMG_ERR_WORKSPACE = -4,     /* workspace missing, too small or misaligned         */
    TPMG_ERR_DEVICE = -5,        /* a HIP call failed (see tpmg_last_error)            */
    TPMG_ERR_BREAKDOWN = -6      /* CG breakdown: (p, Hp) <= 0 or non-finite           */
} tpmg_status;

typedef enum { TPMG_LAYOUT_LEVEL_MAJOR = 0, TPMG_LAYOUT_COLUMN_MAJOR = 1 } tpmg_layout;
typedef enum { TPMG_FP64 = 0, TPMG_MIXED_FP32_VCYCLE = 1 } tpmg_precision;
typedef enum { TPMG_COARSE_DIRECT = 0, TPMG_COARSE_SMOOTH = 1 } tpmg_coarse;

/* Problem and multigrid description (all plain values; dz is a host array). */
typedef struct {
    int32_t n;          /* columns per side of the periodic grid, n % 2^(nlevels-1) == 0     */
    int32_t nz;         /* cells per column, 1 <= nz <= TPMG_MAX_NZ                          */
    int32_t nlevels;    /* multigrid levels, 1 <= nlevels <= TPMG_MAX_LEVELS                 */
    double a_h, a_z;    /* horizontal / vertical coupling scales (> 0; a_h may be 0)         */
    const double *dz;   /* host [nz] cell heights > 0, or NULL for uniform                   */
    int32_t nu_pre;     /* pre-smoothing sweeps per level  (>= 1)                            */
    int32_t nu_post;    /* post-smoothing sweeps per level (>= 1)                            */
    double omega;       /* smoother damping, 0 < omega <= 1 (0.8 in Sec. 5)                  */
    int32_t coarse;     /* tpmg_coarse: exact dense solve or n_coarse sweeps on the coarsest */
    int32_t n_coarse;   /* sweeps on the coarsest level in SMOOTH mode (>= 1)                */
    int32_t precision;  /* tpmg_precision of the V-cycle                                     */
} tpmg_desc;

#define TPMG_MAX_NZ 256
#define TPMG_MAX_LEVELS 12
#define TPMG_MAX_DIRECT_DOF 2048   /* largest coarsest level for TPMG_COARSE_DIRECT */

typedef struct {
    double rtol;         /* stop when ||r||_2 <= rtol ||b||_2 (recursive residual)            */
    int32_t maxit;       /* iteration limit (>= 0)                                            */
    int32_t x0_nonzero;  /* 1: x holds the initial guess; 0: start from x = 0                 */
    int32_t flexible;    /* 1: flexible CG, beta = -(z, H p)/(p, H p) with p the last
                            direction (FCG(1): the new direction is H-conjugate to it);
                            for the FP32 V-cycle, a preconditioner that is not exactly
                            stationary (Sec. 5 asks for a flexible Krylov method then).
                            0: beta = (r, z)/(r_old, z_old)                                 */
    double *history;     /* host [maxit+1] for ||r_i||/||b||, or NULL                         */
    double omega_alt;    /* 0, or in (0, 1]: V-cycles with an odd index (the first is 0) use
                            this damping instead of the hierarchy's omega, which makes the
                            preconditioner change between iterations (exercises the flexible
                            recurrence); the hierarchy's omega is restored on return          */
} tpmg_solve_opts;

typedef struct {
    int32_t iterations;        /* applications of H to a search direction               */
    int32_t converged;         /* 1 if the tolerance was met                            */
    double rel_residual;       /* last recursive ||r||/||b||                            */
    double true_rel_residual;  /* ||b - H x||/||b|| recomputed in FP64 at the end       */
} tpmg_solve_info;

typedef struct tpmg_hierarchy tpmg_hierarchy;

/* Workspace size for a description (validates it: SHAPE / INVALID_ARG / NOT_SPD for dz).
 * TPMG_ERR_SHAPE also for grids whose FP64 level arrays would reach 4 GiB
 * (n*n*nz >= 2^29; kernels use 32-bit byte offsets) or whose reductions would
 * exceed the partial-sum buffer (about 4.8e8 cells). */
tpmg_status tpmg_workspace_bytes(const tpmg_desc *desc, size_t *bytes);

/*
 * Build the level hierarchy (Sec. 3.1, 3.3): copy c (FP64, 3*n*n*nz values in
 * `layout`) into the workspace, check every real face coefficient is positive
 * and finite (TPMG_ERR_NOT_SPD), average faces onto coarse levels, make FP32
 * copies when precision is mixed, and in DIRECT mode factor and invert the
 * coarsest operator on the host (at most TPMG_MAX_DIRECT_DOF unknowns).
 * Synchronises `stream`.  *out receives the handle.  c is not referenced after
 * the call returns.
 */
tpmg_status tpmg_setup_hierarchy(const tpmg_desc *desc, const double *c_dev, int32_t layout,
                                 void *workspace_dev, size_t workspace_bytes, void *stream,
                                 tpmg_hierarchy **out);

/* Columns per side of a level, or -1 for an invalid handle/level. */
int32_t tpmg_level_n(const tpmg_hierarchy *h, int32_t level);

/*
 * y = H_level x (Sec. 4.2 operator on that level).  fp32 = 1 uses the FP32
 * coefficient copies and float buffers (mixed hierarchies only); otherwise
 * double buffers.  x, y: n_l*n_l*nz values in `layout`; must not alias.
 */
tpmg_status tpmg_apply_operator(const tpmg_hierarchy *h, int32_t level, int32_t fp32,
                                const void *x_dev, void *y_dev, int32_t layout, void *stream);

/*
 * For callers that cannot allocate device memory or touch a hierarchy's
 * internal vectors (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): y = H_level x exactly as
 * tpmg_apply_operator computes it (same kernels, bit-identical results), with
 * the layout staging in a library-owned static device array of 64 MiB per GPU
 * (held from the first call on that GPU until the process ends; looked up
 * with that GPU current) instead of the hierarchy's staging vectors.  It
 * calls no allocating routine.  At most 32 MiB per staged vector: levels of
 * up to 4,194,304 cells (fp32 = 0) or 8,388,608 cells (fp32 = 1), else
 * TPMG_ERR_WORKSPACE before any launch.  All calls on one GPU share the
 * array: calls that overlap on one GPU (other streams, other threads, other
 * handles) race.  Call with the hierarchy's GPU current.  Asynchronous.
 */
tpmg_status tpmg_apply_operator_static(const tpmg_hierarchy *h, int32_t level, int32_t fp32, const void *x_dev,
                                       void *y_dev, int32_t layout, void *stream);

/*
 * z = V b: one V-cycle from a zero initial guess on the finest level (the
 * preconditioner of Sec. 4.2.1).  fp32 as in tpmg_apply_operator.  b, z:
 * n*n*nz values in `layout`; must not alias.
 */
tpmg_status tpmg_vcycle(const tpmg_hierarchy *h, int32_t fp32, const void *b_dev, void *z_dev,
                        int32_t layout, void *stream);

/*
 * Solve H_0 x = b by preconditioned CG with one V-cycle per iteration (FP64
 * outer iteration; FP32 V-cycle on fl32(r) in mixed hierarchies).  b, x: FP64,
 * n*n*nz values in `layout`.  Returns TPMG_OK, TPMG_NOT_CONVERGED (x holds the
 * last iterate), TPMG_ERR_BREAKDOWN, or an argument/device error.  info may be
 * NULL; otherwise one more operator pass recomputes ||b - H x|| for
 * info->true_rel_residual (and, in level-major layout, writes x on the way).
 * Synchronises `stream`.
 */
tpmg_status tpmg_solve(const tpmg_hierarchy *h, const double *b_dev, double *x_dev, int32_t layout,
                       const tpmg_solve_opts *opts, tpmg_solve_info *info, void *stream);

/*
 * Adjoint face gradient for J(x) with H x = b and lambda = H^{-1} dJ/dx (H is
 * symmetric, so lambda comes from tpmg_solve on dJ/dx):
 *     dJ/dc_f = -gamma_f (lambda_p - lambda_q)(x_p - x_q),
 * gamma_f = a_h s_k (E, N faces), a_z / t_{k+1/2} (U faces); 0 in the U slot
 * of the top cell.  lambda, x: FP64 cells; grad: FP64 faces (3*n*n*nz),
 * overwritten; all in `layout`.
 */
tpmg_status tpmg_face_gradient(const tpmg_hierarchy *h, const double *lambda_dev,
                               const double *x_dev, double *grad_dev, int32_t layout, void *stream);

/*
 * Components of the V-cycle, exposed for testing and composition; level-major
 * buffers of the hierarchy's precision selected by fp32, staged through the
 * hierarchy's CG vectors (so these calls must not overlap a solve on the
 * same handle).
 *
 * tpmg_smooth: one damped line-relaxation sweep on a level (Sec. 4.2),
 *   u_out = u + omega H_z^{-1}(b - H u); u = NULL means u = 0.
 * tpmg_residual_restrict: b_coarse = R (b - H_level u) on level+1 (Sec. 3.2).
 * tpmg_prolong_smooth: u_out = S(u + P e), the correction from level+1 added
 *   by injection followed by one sweep (the first post-smoothing step).
 * tpmg_coarse_solve: the coarsest-level solve (dense, or n_coarse sweeps from 0).
 * tpmg_level_coefficients: copy of a level's face coefficients c[f][k][j][i].
 */
tpmg_status tpmg_smooth(const tpmg_hierarchy *h, int32_t level, int32_t fp32, const void *u_dev,
                        const void *b_dev, void *u_out_dev, void *stream);
tpmg_status tpmg_residual_restrict(const tpmg_hierarchy *h, int32_t level, int32_t fp32,
                                   const void *u_dev, const void *b_dev, void *b_coarse_dev,
                                   void *stream);
tpmg_status tpmg_prolong_smooth(const tpmg_hierarchy *h, int32_t level, int32_t fp32,
                                const void *u_dev, const void *e_coarse_dev, const void *b_dev,
                                void *u_out_dev, void *stream);
tpmg_status tpmg_coarse_solve(const tpmg_hierarchy *h, int32_t fp32, const void *b_dev,
                              void *u_dev, void *stream);
tpmg_status tpmg_level_coefficients(const tpmg_hierarchy *h, int32_t level, int32_t fp32,
                                    void *c_out_dev, void *stream);

/*
 * Kernel timing with HIP events recorded on the launch stream around every
 * launch of one kernel class (for bandwidth accounting).  enable: 0 off, 1 the
 * kernel classes below, 2 also every launch on each V-cycle level
 * (tpmg_profile_read_level; the extra events lengthen a V-cycle slightly).
 * Enabling resets the counters.  read synchronises the recorded events and
 * returns the summed duration and the launch count.
 */
typedef enum {
    TPMG_K_SWEEP = 0,        /* line sweep, general form, finest level          */
    TPMG_K_SWEEP0 = 1,       /* first pre-sweep from zero, finest level         */
    TPMG_K_PROLSWEEP = 2,    /* prolongation + sweep, finest level              */
    TPMG_K_RESTRICT = 3,     /* residual + restriction from the finest level    */
    TPMG_K_PCG_APPLY = 4,    /* CG direction update + operator apply            */
    TPMG_K_PCG_UPDATE = 5,   /* CG x / r update                                 */
    TPMG_K_VCYCLE = 6,       /* one whole V-cycle                               */
    TPMG_K_DG1_SWEEP = 7,    /* DG1 line sweep, general form (tpmg_dg1_*)       */
    TPMG_K_DG1_PCG_APPLY = 8,/* DG1 CG direction update + operator apply        */
    TPMG_K_DG1_VCYCLE = 9,   /* one whole DG1 (NLO) V-cycle                     */
    TPMG_K_COUNT = 10
} tpmg_kernel_class;
tpmg_status tpmg_profile_enable(tpmg_hierarchy *h, int32_t enable);
tpmg_status tpmg_profile_read(tpmg_hierarchy *h, int32_t kernel_class, double *total_ms,
                              int64_t *launches);
/* The same for every kernel that runs on V-cycle level `level` (its sweeps,
 * its residual + restriction, the prolongation sweep into it, the coarsest
 * solve), per launch: the per-level breakdown of a V-cycle (the view of the
 * paper's Tab. MultigridBreakdown).  Level-0 time inside the DG1 (NLO)
 * V-cycle counts on level 0. */
tpmg_status tpmg_profile_read_level(tpmg_hierarchy *h, int32_t level, double *total_ms, int64_t *launches);

/*
 * Plain device copy dst <- src of `bytes` bytes (multiple of 16, 16-byte
 * aligned, non-overlapping) by a streaming kernel: the reference point for
 * bandwidth and memory-counter calibration.  Asynchronous.
 */
tpmg_status tpmg_bandwidth_probe(void *dst_dev, const void *src_dev, size_t bytes, void *stream);

/* Release the handle (not the workspace).  NULL is accepted.  The small pinned
 * host block a hierarchy reads its CG scalars into (a few hundred bytes) stays
 * with the library and is reused by the next tpmg_setup_hierarchy. */
tpmg_status tpmg_destroy(tpmg_hierarchy *h);

/*
 * Velocity-pressure system around the pressure solve (Sec. 4.2,
 * Eq. PressureVelocitySystem with buoyancy eliminated), on the finest level,
 * FP64, level-major only.  A mixed vector holds four blocks of n*n*nz values,
 * [uE | uN | uU | p]: the normal velocity on the E, N and U face slots of each
 * cell (slot layout as the face coefficients; the U slot of the top cell
 * holds no face and must be 0 on input, and is 0 on output) and the pressure.
 * With the face weights w_f of the pressure operator (H = M3 + D W D^T):
 *   A (u, p) = (M u - D^T p, D u + M3 p),
 *   (D u)_p = outgoing minus incoming face values of cell p, (D^T x)_f = x_p - x_q,
 *   (M u)_f = u_f / w_f + 1/4 sum u_f' / sqrt(w_f w_f') over the same-direction
 *             faces f' that share a cell with f (a normalised lowest-order
 *             Raviart-Thomas mass whose diagonal is 1/w_f, so that its diagonal
 *             lumping (Eq. LumpedMass) gives exactly H).
 * Requires n >= 2 (TPMG_ERR_SHAPE).  These calls use the hierarchy's internal
 * vectors: they must not overlap other calls on the same handle.
 *
 * tpmg_mixed_apply: y = A x (asynchronous; x, y must not alias).
 * tpmg_mixed_precondition: z = P^{-1} r, the Schur-complement factorisation
 *   (Eq. SchurComplement) with the lumped inverse mass W for M^{-1} and one
 *   V-cycle for H^{-1} (FP32 V-cycle on fl32 when fp32 = 1, mixed hierarchies
 *   only): t = r_p - D W r_u, z_p = V t, z_u = W (r_u + D^T z_p).  Asynchronous.
 * tpmg_mixed_solve: restarted flexible GMRES (right preconditioning with
 *   P^{-1}, the V-cycle in the hierarchy's precision; Sec. 5 uses GMRES(30))
 *   from x = 0 until the Arnoldi residual estimate is <= rtol ||b||.
 *   Orthogonalisation: classical Gram-Schmidt twice, the second pass of each
 *   vector delayed into the next step's update (one pass over the basis per
 *   step); an immediate second pass when the first leaves projections above
 *   a tenth of the norm, and beyond 16 basis vectors (there selectively, when
 *   the first pass cancels more than a factor 1/sqrt(2) of the norm);
 *   fixed-order reductions.  Krylov vectors are kept unnormalised with their
 *   scales on the host.
 *   workspace: caller-owned device memory of at least
 *   tpmg_mixed_workspace_bytes(restart) bytes (2 restart + 1 mixed vectors
 *   plus reduction buffers), 256-byte aligned (TPMG_ERR_WORKSPACE otherwise).
 *   b and x must not alias; b is read throughout and left unchanged.  info->rel_residual is the final estimate,
 *   info->true_rel_residual = ||b - A x|| / ||b|| recomputed.  Returns TPMG_OK,
 *   TPMG_NOT_CONVERGED (x holds the last iterate), TPMG_ERR_BREAKDOWN or an
 *   argument/device error; TPMG_ERR_INVALID_ARG when b is not 0 in the U
 *   slots of the top cells.  Synchronises `stream`.
 */
#define TPMG_MAX_RESTART 256
typedef struct {
    double rtol;      /* relative tolerance on ||b - A x|| / ||b||               */
    int32_t restart;  /* Krylov vectors per cycle, 1..TPMG_MAX_RESTART           */
    int32_t maxit;    /* total iterations (applications of A)                    */
    double *history;  /* host [maxit + 1] residual estimates / ||b||, or NULL    */
} tpmg_mixed_opts;
tpmg_status tpmg_mixed_workspace_bytes(const tpmg_hierarchy *h, int32_t restart, size_t *bytes);
tpmg_status tpmg_mixed_apply(const tpmg_hierarchy *h, const double *x_dev, double *y_dev, void *stream);
tpmg_status tpmg_mixed_precondition(const tpmg_hierarchy *h, int32_t fp32, const double *r_dev, double *z_dev,
                                    void *stream);
tpmg_status tpmg_mixed_solve(const tpmg_hierarchy *h, const double *b_dev, double *x_dev, void *workspace_dev,
                             size_t workspace_bytes, const tpmg_mixed_opts *opts, tpmg_solve_info *info,
                             void *stream);

/*
 * Next-to-lowest-order (NLO) pressure level on the finest grid (Tab.
 * FiniteElements: DG_1 pressure, six unknowns per cell), its vertical line
 * smoother by a banded LU that is factorised once and applied per sweep
 * (Sec. 4.3.1: LAPACK dgbtrf at setup, dgbtrs per application), and the
 * p-coarsening to the lowest-order level by the natural embedding of DG_0
 * in DG_1 (Sec. 4.2.1); the lowest-order hierarchy of h is the rest of the
 * multigrid hierarchy.
 *
 * OPERATOR (a reading: the paper assembles its NLO operator with finite
 * element machinery it does not spell out).  Cell (i, j, k) has reference
 * coordinates xi, eta, zeta in [-1, 1] and unknowns u_{3v+h},
 *     u = sum_{v=0,1} sum_{h=0..2} u_{3v+h} l_v(zeta) psi_h(xi, eta),
 * psi = (1, xi, eta), l_0 = (1 - zeta)/2, l_1 = (1 + zeta)/2 (bottom and top
 * values of a linear function in the vertical).  With width 1 and height s_k,
 *     (H1 u, w) = sum over cells of  s_k <u w>
 *                 + 4 a_h s_k (c^x <u_xi w_xi> + c^y <u_eta w_eta>)
 *                 + 4 a_z c^z / s_k <u_zeta w_zeta>
 *               + sum over faces f of  w_f <[u] [w]>_f,
 * <.> the mean over the reference cell or face, [.] the jump across f,
 * w_f the lowest-order face weight (a_h s_k c_f east / north, a_z c_f /
 * t_{k+1/2} upper), c^x = (c_E + c_W)/2, c^y = (c_N + c_S)/2 of the cell's
 * own faces, c^z the mean of its vertical faces (the one face at the bottom
 * and top cells).  Symmetric positive definite; for cellwise constants it
 * is exactly the lowest-order operator (P^T H1 P = H_0).
 *
 * The column block H1_z (all couplings inside a column: cell terms, the
 * self parts of the horizontal faces, the vertical faces) is banded with 5
 * sub- and 5 super-diagonals in the row order r = 6 k + a; it is factorised
 * without pivoting (SPD), in FP64.  A mixed hierarchy stores the factors in
 * FP32 (half the bytes the sweeps stream; forward and back substitution still
 * run in FP64), so its line solves and sweeps use the FP32-rounded factors.
 * Smoother: u <- u + omega H1_z^{-1} (b - H1 u)
 * with the hierarchy's omega.  Transfers: P1 e0 adds e0 to u_0 and u_3 (the
 * bottom and top values of the constant mode); R1 = P1^T.  NLO V-cycle
 * from a zero guess: nu_pre DG1 sweeps, b0 = R1 (b - H1 u), one lowest-order
 * V-cycle of h on b0 (FP32 in a mixed hierarchy), u += P1 e0, nu_post DG1
 * sweeps.
 *
 * LAYOUT: DG1 vectors are FP64 arrays (6, nz, n, n): unknown a of cell
 * (i, j, k) at ((a nz + k) n + j) n + i.  Lowest-order vectors are level-major
 * (nz, n, n).  The hierarchy must have nz >= 2 and be used level-major; its
 * DG1 vectors must stay below 4 GiB (6 n^2 nz < 2^29) (TPMG_ERR_SHAPE).
 *
 * OWNERSHIP: the caller owns the DG1 workspace (tpmg_dg1_workspace_bytes,
 * 256-byte aligned: band factors of 66 n^2 nz values (doubles; floats in a
 * mixed hierarchy), nine DG1 vectors,
 * two lowest-order vectors); the handle aliases it and h.  Calls use the
 * reduction buffers and coarse-level vectors of h: they must not overlap
 * other calls on h.  Buffers of one call must not alias unless stated.
 */
typedef struct tpmg_dg1 tpmg_dg1;
tpmg_status tpmg_dg1_workspace_bytes(const tpmg_hierarchy *h, size_t *bytes);
/* Factorise every column block on the device (TPMG_ERR_NOT_SPD on a
 * non-positive pivot).  Synchronises `stream`. */
tpmg_status tpmg_dg1_setup(const tpmg_hierarchy *h, void *workspace_dev, size_t workspace_bytes, void *stream,
                           tpmg_dg1 **out);
/* y = H1 x (asynchronous). */
tpmg_status tpmg_dg1_apply(const tpmg_dg1 *g, const double *x_dev, double *y_dev, void *stream);
/* x = H1_z^{-1} r in every column: forward and back substitution with the
 * band factors (the per-application dgbtrs of Sec. 4.3.1; asynchronous). */
tpmg_status tpmg_dg1_line_solve(const tpmg_dg1 *g, const double *r_dev, double *x_dev, void *stream);
/* u_out = u + omega H1_z^{-1} (b - H1 u); u = NULL means u = 0 (asynchronous). */
tpmg_status tpmg_dg1_smooth(const tpmg_dg1 *g, const double *u_dev, const double *b_dev, double *u_out_dev,
                            void *stream);
/* b0 = R1 (b - H1 u), a lowest-order level-major vector (asynchronous). */
tpmg_status tpmg_dg1_residual_restrict(const tpmg_dg1 *g, const double *u_dev, const double *b_dev,
                                       double *b0_dev, void *stream);
/* u += P1 e0, in place (e0 lowest-order level-major; asynchronous). */
tpmg_status tpmg_dg1_prolong_add(const tpmg_dg1 *g, const double *e0_dev, double *u_dev, void *stream);
/* z = V1 b, the NLO V-cycle from a zero guess (asynchronous). */
tpmg_status tpmg_dg1_vcycle(const tpmg_dg1 *g, const double *b_dev, double *z_dev, void *stream);
/* CG on H1 x = b from x = 0 with one NLO V-cycle per iteration (FP64 outer
 * iteration; opts as for tpmg_solve, with x0_nonzero = 0 and omega_alt = 0
 * required).  Same return values as tpmg_solve.  Synchronises `stream`. */
tpmg_status tpmg_dg1_solve(const tpmg_dg1 *g, const double *b_dev, double *x_dev, const tpmg_solve_opts *opts,
                           tpmg_solve_info *info, void *stream);
/* Copy of the band factors, [col = j n + i][r][e] (n^2 x 6 nz x 11): L(r, r-5+e)
 * for e < 5, U(r, r) for e = 5, U(r, r+e-5) for e > 5 (0 outside the matrix).
 * In a mixed hierarchy: the stored FP32 values, with U(r, r) given as the
 * reciprocal of the stored FP32 value of 1 / U(r, r). */
tpmg_status tpmg_dg1_factors(const tpmg_dg1 *g, double *f_dev, void *stream);
/* Release the handle (not the workspace).  NULL is accepted.  The small pinned
 * host block a hierarchy reads its CG scalars into (a few hundred bytes) stays
 * with the library and is reused by the next tpmg_setup_hierarchy. */
tpmg_status tpmg_dg1_destroy(tpmg_dg1 *g);

const char *tpmg_status_string(tpmg_status s);
/* Last error text of a handle, or of the calling thread when h is NULL. */
const char *tpmg_last_error(const tpmg_hierarchy *h);

#ifdef __cplusplus
}
#endif
#endif /* TPMG_H */
