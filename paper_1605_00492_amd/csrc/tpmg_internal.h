// Internal declarations shared by the kernels (tpmg_kernels.hip) and the host
// driver (tpmg_host.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tpmg {

// Storage of every cell array of a level (the hierarchy's vectors and each
// of its three face arrays).  Columns col = j*n + i are grouped into tiles
// of W consecutive columns; a tile stores its nz levels one after the other,
// W values per level:
//   cell (col, k) at (col / W) * nz * W + k * W + col % W,
// with W = 64 when the plane is a multiple of 64 (a wavefront's 64 lanes
// read 256 or 512 contiguous bytes per level, and stepping k moves to the
// next contiguous segment), otherwise W = plane (plain level-major order).
// Any 64 aligned consecutive columns of one level are contiguous in both this
// and the level-major order, so converting kernels stay coalesced.
__host__ __device__ inline int tile_width(int plane) { return (plane & 63) == 0 ? 64 : plane; }
// index of (col, 0); (col, k) is at cell_base + k * tile_width(plane)
__host__ __device__ inline size_t cell_base(size_t col, int plane, int nz)
{
    return (plane & 63) == 0 ? (col >> 6) * (size_t)nz * 64 + (col & 63) : col;
}
__host__ __device__ inline size_t cell_index(size_t col, int k, int plane, int nz)
{
    return cell_base(col, plane, nz) + (size_t)k * tile_width(plane);
}

// One multigrid level as the kernels see it (cells and faces in the tiled
// storage above; faces c[f] for f in {E, N, U}, each an nz * plane array).
template <typename T>
struct Level {
    int n;          // columns per side
    int nz;         // cells per column
    int plane;      // n * n
    const T *c;     // [3][nz * plane]; U slot of the top cell holds 0
    const T *mu;    // [nz]  mass 4^l s_k
    const T *wh;    // [nz]  horizontal factor a_h s_k
    const T *wz;    // [nz]  vertical factor 4^l a_z / t_{k+1/2}; wz[nz-1] = 0
    // Kernels that walk a chunk of a column take an unguarded path when the
    // chunk lies inside it; 0 forces the guarded path everywhere (for
    // comparison; TPMG_FULL_CHUNKS=0).
    int full_chunks = 1;
};

// Forms of the line-relaxation sweep kernel.
enum SweepMode : int {
    SWEEP_ZERO = 0,     // u = 0:        out = omega H_z^{-1} b
    SWEEP_GENERAL = 1,  //               out = u + omega H_z^{-1} (b - H u)
    SWEEP_PROLONG = 2,  // u <- u + P e: out = u + omega H_z^{-1} (b - H u)
};

// Scalars of the CG iteration, kept in device memory so that kernels read
// alpha / beta without a host round trip.
struct Scalars {
    double bb;        // (b, b)
    double rr;        // (r, r)
    double rz;        // (r, z) of the current z
    double pq;        // (p, H p) of the last direction
    double alpha;
    double beta;
    double tt;        // (b - H x, b - H x) of the final iterate
    int32_t breakdown;
    int32_t pad;
};

enum FinalizeStage : int {
    ST_BB = 0,
    ST_RR = 1,
    ST_RZ_FIRST = 3,
    ST_RZ = 4,
    ST_PQ = 5,
    ST_TT = 6,
};

// Upper bound on per-dot partial sums (one per workgroup) in any reduction.
constexpr int kMaxPartials = 1 << 19;
// Segments of the first reduction stage when a dot has many partials; the
// stage buffer holds 2 * kReduceSegs doubles.
constexpr int kReduceSegs = 512;

// ---- launchers (kernels.hip) --------------------------------------------
// Each returns the launch status.  Shapes are validated by the caller.
template <typename T>
hipError_t launch_sweep(const Level<T> &L, int mode, const T *u, const T *b, T *out,
                        const T *ec, T omega, hipStream_t s);
template <typename T>
hipError_t launch_apply(const Level<T> &L, const T *x, T *y, hipStream_t s);
template <typename T>
hipError_t launch_resid_restrict(const Level<T> &L, const T *u, const T *b, T *bc, hipStream_t s);
template <typename T>
hipError_t launch_coarse_gemv(const T *ainv, int m, const T *b, T *x, hipStream_t s);

// Face means onto level l+1 (FP64, and FP32 when c_coarse32 is given).
hipError_t launch_coarsen(const Level<double> &F, double *c_coarse, float *c_coarse32, hipStream_t s);
hipError_t launch_cast(const double *src, float *dst, size_t n, hipStream_t s);
// Caller's faces -> level-0 storage (FP64, and FP32 when dst32 is given),
// counting real faces that are not positive and finite into *bad.
hipError_t launch_copy_coeffs(const double *src, int layout, double *dst, float *dst32, int plane, int nz, int *bad,
                              hipStream_t s);
hipError_t launch_fill(double *x, double v, size_t n, hipStream_t s);
// Caller's cells (layout 0 level-major, 1 column-major; elem = 4 or 8 bytes)
// <-> the tiled storage of a level with this plane; cells_in also writes a
// second copy to dst2 when given.
hipError_t launch_cells_in(const void *src, int layout, void *dst, void *dst2, int plane, int nz, int elem,
                           hipStream_t s);
hipError_t launch_cells_out(const void *src, void *dst, int layout, int plane, int nz, int elem, hipStream_t s);
// Solve start from x = 0 with a level-major b: r = b (and fl32(r) into r32
// when given) in tiled storage, b and x = 0 there when given (may be null),
// partial sums of (b, b).
hipError_t launch_solve_start(const double *bsrc, double *b, double *r, float *r32, double *x, int plane, int nz,
                              double *partials, int *nblocks_out, hipStream_t s);
// column-major -> level-major cell transpose (elem = 4 or 8 bytes)
hipError_t launch_cells_to_level(const void *src, void *dst, int plane, int nz, int elem,
                                 hipStream_t s);
hipError_t launch_faces_to_column(const double *src, double *dst, int plane, int nz,
                                  hipStream_t s);

// CG building blocks (FP64).  Partial sums go to `partials`; nblocks_out
// receives the number of partials written per value.
// p_new = z + beta p_old, q = H p_new, partial sums of (p_new, q)
hipError_t launch_pcg_apply(const Level<double> &L, const double *z, const float *z32,
                            const double *p_old, double *p_new, double *q, const Scalars *sc,
                            int first, double *partials, int *nblocks_out, hipStream_t s);
// x += alpha p (x = alpha p without reading x when x_first), r -= alpha q,
// r32 = fl32(r) when given, partial sums of (r, r)
hipError_t launch_pcg_update(size_t n, double *x, const double *p, double *r, const double *q,
                             float *r32, const Scalars *sc, double *partials, int x_first,
                             int *nblocks_out, hipStream_t s);
// partial sums of (a, b) and, when c is given, of (c, b) (two values per
// block); b is b32 when given
hipError_t launch_dot(size_t n, const double *a, const double *b, const float *b32,
                      double *partials, int *nblocks_out, hipStream_t s, const double *c = nullptr);
// r = b - H x (r null: the norm only) and partial sums of (r, r); b in the
// level's storage, or level-major with b_level; with xout non-null, x is also
// copied there in level-major order.
hipError_t launch_residual(const Level<double> &L, const double *x, const double *b, int b_level, double *r,
                           double *xout, double *partials, int *nblocks_out, hipStream_t s);
hipError_t launch_finalize(const double *partials, int nblocks, int nvals, Scalars *sc, int stage,
                           int flexible, double *stage_buf, hipStream_t s);
hipError_t launch_face_gradient(const Level<double> &L, const double *lam, const double *x,
                                double *g, hipStream_t s);
hipError_t launch_probe_copy(void *dst, const void *src, size_t bytes, hipStream_t s);

// ---- velocity-pressure system (mixed.hip), finest level, FP64 ----------------
// Vectors of the outer GMRES combined per kernel launch.
constexpr int kMultiMax = 16;
hipError_t launch_mixed_apply(const Level<double> &L, const double *x, double *y, hipStream_t s);
// t = a (r_p - D W r_u) (and fl32(t) into t32 when given)
hipError_t launch_mixed_pre1(const Level<double> &L, const double *r, double a, double *t, float *t32, hipStream_t s);
// z_u = W (a r_u + D^T y), z_p = y, y from y64 or y32
hipError_t launch_mixed_pre2(const Level<double> &L, const double *r, double a, const double *y64, const float *y32,
                             double *z, hipStream_t s);
// out[i] = (w, v_i), i < nv <= kMultiMax, fixed-order reductions
hipError_t launch_multidot(size_t n, const double *w, const double *const *v, int nv, double *partials,
                           double *stage, double *out, hipStream_t s);
// y += sum a_i v_i; norm_partials (optional) receives the partial sums of (y, y)
hipError_t launch_multiaxpy(size_t n, double *y, const double *const *v, const double *a, int nv,
                            double *norm_partials, int *nblocks_out, hipStream_t s);
// y += sum a_i v_i, then out[i] = (y, v_i) for i < nv and out[nv] = (y, y)
// (nv + 1 values: partials, stage and out hold kMultiMax + 2 of them)
hipError_t launch_multiaxpy_dot(size_t n, double *y, const double *const *v, const double *a, int nv,
                                double *partials, double *stage, double *out, hipStream_t s);
// Delayed reorthogonalisation step: u <- q = u * inv_rho - sum ca_i v_i,
// w <- w' = w - sum cw_i v_i - hq q, then out[i] = (sd_i v_i, w') for i < nv,
// out[nv] = (q, w'), out[nv + 1] = (w', w') (nv + 2 <= kMultiMax + 2 values)
hipError_t launch_corr_axpy_dot(size_t n, double *u, double *w, const double *const *v, const double *ca,
                                const double *cw, const double *sd, int nv, double inv_rho, double hq,
                                double *partials, double *stage, double *out, hipStream_t s);
// y = a x + b z (z == nullptr: y = a x); y may alias z
hipError_t launch_axpby(size_t n, double a, const double *x, double b, const double *z, double *y, hipStream_t s);
// out[v] = fixed-order sum of the G partials of value v (v < nvals <= kMultiMax)
hipError_t launch_sum_partials(const double *partials, int G, int nvals, double *stage, double *out, hipStream_t s);

// ---- next-to-lowest-order (DG1) level (dg1.hip), FP64 ------------------------
// The DG1 level on the finest grid: six unknowns per cell, vectors in the
// tiled storage with 6 nz rows per column (row a nz + k holds unknown a of
// cell k), the faces of level 0, and per-k scalars.
struct Dg1Level {
    int n, nz, plane;
    const double *c;    // level-0 faces [3][nz * plane] (tiled storage, nz rows)
    const double *tab;  // [5][nz]: s_k, a_h s_k, 4 a_h s_k, 4 a_z / s_k, a_z / t_{k+1/2} (0 at the top)
    int fac32;          // band factors stored in FP32 (computed in FP64, used in FP64 arithmetic)
};
enum Dg1Sweep : int {
    DG1_SWEEP_ZERO = 0,     // out = omega H1_z^{-1} b
    DG1_SWEEP_GENERAL = 1,  // out = u + omega H1_z^{-1} (b - H1 u)
    DG1_SWEEP_SOLVE = 2,    // out = H1_z^{-1} b
};
// Band LU of every column block into fac (6 nz rows x 11 entries per column,
// tiled by 64 columns); non-positive pivots are counted into *bad.
hipError_t launch_dg1_factor(const Dg1Level &G, void *fac, int *bad, hipStream_t s);
hipError_t launch_dg1_sweep(const Dg1Level &G, const void *fac, int mode, const double *u, const double *b,
                            double *out, double omega, hipStream_t s);
hipError_t launch_dg1_apply(const Dg1Level &G, const double *x, double *y, hipStream_t s);
// r = b - H1 x (r may be null) and partial sums of (r, r)
hipError_t launch_dg1_residual(const Dg1Level &G, const double *x, const double *b, double *r, double *partials,
                               int *nblocks_out, hipStream_t s);
// p_new = z + beta p_old (z when first), q = H1 p_new, partial sums of (p_new, q)
hipError_t launch_dg1_pcg_apply(const Dg1Level &G, const double *z, const double *p_old, double *p_new, double *q,
                                const Scalars *sc, int first, double *partials, int *nblocks_out, hipStream_t s);
// b0 = R1 (b - H1 u) into a lowest-order level-0 vector (float when fp32)
hipError_t launch_dg1_resid_restrict(const Dg1Level &G, const double *u, const double *b, void *b0, int fp32,
                                     hipStream_t s);
// u += P1 e0 (e0 a lowest-order level-0 vector, float when fp32)
hipError_t launch_dg1_prolong(const Dg1Level &G, const void *e0, int fp32, double *u, hipStream_t s);
// factors as [col][row][entry] with U(r, r) in entry 5
hipError_t launch_dg1_factors_out(const Dg1Level &G, const void *fac, double *dst, hipStream_t s);

// Sweep chunking for a precision, sweep mode and column height: M cells per chunk, CPW
// chunks per wavefront, P wavefronts per 64-column tile; false if nz is not
// supported.
bool sweep_shape(int nz, bool fp32, int mode, int *M, int *CPW, int *P);

}  // namespace tpmg
