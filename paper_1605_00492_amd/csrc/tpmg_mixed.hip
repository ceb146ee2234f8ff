// HIP kernels for the velocity-pressure system around the pressure solve
// (Mitchell & Mueller, Sec. 4.2, Eq. PressureVelocitySystem with buoyancy
// eliminated), its Schur-complement preconditioner (Eq. SchurComplement with
// the lumped mass of Eq. LumpedMass) and the vector kernels of the outer
// restarted GMRES (Sec. 5).
//
// Finest level only, FP64, mixed vectors [uE | uN | uU | p] in the caller's
// level-major order (the face coefficients and the V-cycle's vectors in the
// level's tiled storage):
// four blocks of m = n^2 nz values, face slot f of cell p joining p to its
// east / north / upper neighbour, the U slot of the top cell unused (0).
// With the face weights w_f of the pressure operator H = M3 + D W D^T:
//   (M u)_f   = u_f / w_f + 1/4 sum_{f'} u_f' / sqrt(w_f w_f')
//               (f' = same-direction faces sharing a cell with f: the
//               normalised lowest-order Raviart-Thomas mass, diagonal 1/w_f),
//   (D u)_p   = outgoing minus incoming face values of cell p,
//   (D^T x)_f = x_p - x_q,
//   A (u, p)  = (M u - D^T p, D u + M3 p).
// All kernels stream: thread = (column, chunk of KC cells along k).
#include <type_traits>

#include "tpmg_device.h"

namespace tpmg {

namespace {

constexpr int kMixedKC = 16;

// Buffer descriptors of the three face-coefficient arrays and 32-bit byte
// offsets: column in the lane offset, k plane in the wave-uniform offset
// (arrays hold < 2^32 bytes).  Mixed vectors are the caller's level-major
// blocks (offsets v*, level stride vstride); the face coefficients and the
// pressure-solve vectors use the level's tiled storage (offsets o*, stride
// pstride).
struct MixedRows {
    Rsrc cE, cN, cU;
    unsigned oc, oe, ow, on, os, pstride;
    unsigned vc, ve, vw, vn, vs, vstride;
    __device__ MixedRows(const Level<double> &L, unsigned col)
    {
        const size_t m = (size_t)L.nz * L.plane;
        cE = make_rsrc(L.c, m * 8);
        cN = make_rsrc(L.c + m, m * 8);
        cU = make_rsrc(L.c + 2 * m, m * 8);
        const Nbr nb = neighbours(col, L.n, L.plane);
        oc = cell_off(L, col);
        oe = cell_off(L, nb.e);
        ow = cell_off(L, nb.w);
        on = cell_off(L, nb.n);
        os = cell_off(L, nb.s);
        pstride = (unsigned)tile_width(L.plane) * 8u;
        vc = col * 8u;
        ve = nb.e * 8u;
        vw = nb.w * 8u;
        vn = nb.n * 8u;
        vs = nb.s * 8u;
        vstride = (unsigned)L.plane * 8u;
    }
};

__device__ __forceinline__ double ld(Rsrc r, unsigned voff, unsigned soff) { return bload(double(), r, voff, soff); }

// y = A x.
__global__ __launch_bounds__(kStreamThreads) void k_mixed_apply(Level<double> L, const double *__restrict__ x,
                                                                double *__restrict__ y)
{
    int col, k0;
    bool active;
    stream_coords<kMixedKC>(L, col, k0, active);
    const int nz = L.nz;
    const size_t m = (size_t)nz * L.plane;
    const MixedRows R(L, col);
    const Rsrc xE = make_rsrc(x, m * 8), xN = make_rsrc(x + m, m * 8), xU = make_rsrc(x + 2 * m, m * 8),
               xP = make_rsrc(x + 3 * m, m * 8);
    const Rsrc yE = make_rsrc(y, m * 8), yN = make_rsrc(y + m, m * 8), yU = make_rsrc(y + 2 * m, m * 8),
               yP = make_rsrc(y + 3 * m, m * 8);
    const unsigned oo = active ? R.vc : 0xFFFFFFFFu;  // inactive lanes write nothing
    // vertical window: U face below the cell (weight, value), the cell's own
    // U face (weight, value) and the pressure of the cell
    double wUm = 0, xUm = 0;
    if (k0 > 0 && k0 - 1 < nz - 1) {
        wUm = L.wz[k0 - 1] * ld(R.cU, R.oc, (unsigned)(k0 - 1) * R.pstride);
        xUm = ld(xU, R.vc, (unsigned)(k0 - 1) * R.vstride);
    }
#pragma unroll
    for (int t = 0; t < kMixedKC; ++t) {
        const int k = k0 + t;
        if (k < nz) {
            const unsigned sk = (unsigned)k * R.pstride, vk = (unsigned)k * R.vstride;
            const double h = L.wh[k];
            const double xp = ld(xP, R.vc, vk);
            // east faces: own, west neighbour's, east neighbour's
            const double we = h * ld(R.cE, R.oc, sk), ww = h * ld(R.cE, R.ow, sk), wee = h * ld(R.cE, R.oe, sk);
            const double xe = ld(xE, R.vc, vk), xw = ld(xE, R.vw, vk), xee = ld(xE, R.ve, vk);
            const double ye = xe / we + 0.25 * (xw / sqrt(we * ww) + xee / sqrt(we * wee)) - (xp - ld(xP, R.ve, vk));
            // north faces
            const double wn = h * ld(R.cN, R.oc, sk), ws = h * ld(R.cN, R.os, sk), wnn = h * ld(R.cN, R.on, sk);
            const double xn = ld(xN, R.vc, vk), xs = ld(xN, R.vs, vk), xnn = ld(xN, R.vn, vk);
            const double yn = xn / wn + 0.25 * (xs / sqrt(wn * ws) + xnn / sqrt(wn * wnn)) - (xp - ld(xP, R.vn, vk));
            // upper face (none above the top cell)
            double yu = 0, xu = 0, wu = 0;
            if (k + 1 < nz) {
                const unsigned sp = sk + R.pstride, vp = vk + R.vstride;
                wu = L.wz[k] * ld(R.cU, R.oc, sk);
                xu = ld(xU, R.vc, vk);
                double acc = xu / wu;
                if (k >= 1) acc += 0.25 * xUm / sqrt(wu * wUm);
                if (k + 2 < nz) acc += 0.25 * ld(xU, R.vc, vp) / sqrt(wu * (L.wz[k + 1] * ld(R.cU, R.oc, sp)));
                yu = acc - (xp - ld(xP, R.vc, vp));
            }
            const double yp = (xe - xw) + (xn - xs) + (xu - xUm) + L.mu[k] * xp;
            bstore(ye, yE, oo, vk);
            bstore(yn, yN, oo, vk);
            bstore(yu, yU, oo, vk);
            bstore(yp, yP, oo, vk);
            wUm = wu;
            xUm = xu;
        }
    }
}

// t = a (r_p - D (W r_u)); also fl32(t) when t32 is given.
__global__ __launch_bounds__(kStreamThreads) void k_mixed_pre1(Level<double> L, const double *__restrict__ r, double a,
                                                               double *__restrict__ t, float *__restrict__ t32)
{
    int col, k0;
    bool active;
    stream_coords<kMixedKC>(L, col, k0, active);
    const int nz = L.nz;
    const size_t m = (size_t)nz * L.plane;
    const MixedRows R(L, col);
    const Rsrc rE = make_rsrc(r, m * 8), rN = make_rsrc(r + m, m * 8), rU = make_rsrc(r + 2 * m, m * 8),
               rP = make_rsrc(r + 3 * m, m * 8);
    const Rsrc rt = make_rsrc(t, m * 8), rt32 = make_rsrc(t32, t32 ? m * 4 : 0);
    // t (tiled storage, the V-cycle's input)
    const unsigned oo = active ? R.oc : 0xFFFFFFFFu;
    const unsigned oo32 = active ? R.oc / 2 : 0xFFFFFFFFu;
    double fUm = 0;  // W r on the U face below
    if (k0 > 0 && k0 - 1 < nz - 1)
        fUm = L.wz[k0 - 1] * ld(R.cU, R.oc, (unsigned)(k0 - 1) * R.pstride) *
              ld(rU, R.vc, (unsigned)(k0 - 1) * R.vstride);
#pragma unroll
    for (int tt = 0; tt < kMixedKC; ++tt) {
        const int k = k0 + tt;
        if (k < nz) {
            const unsigned sk = (unsigned)k * R.pstride, vk = (unsigned)k * R.vstride;
            const double h = L.wh[k];
            const double fU = (k + 1 < nz) ? L.wz[k] * ld(R.cU, R.oc, sk) * ld(rU, R.vc, vk) : 0.0;
            const double div = (h * ld(R.cE, R.oc, sk) * ld(rE, R.vc, vk) - h * ld(R.cE, R.ow, sk) * ld(rE, R.vw, vk)) +
                               (h * ld(R.cN, R.oc, sk) * ld(rN, R.vc, vk) - h * ld(R.cN, R.os, sk) * ld(rN, R.vs, vk)) +
                               (fU - fUm);
            const double tv = a * (ld(rP, R.vc, vk) - div);
            bstore(tv, rt, oo, sk);
            if (t32) bstore((float)tv, rt32, oo32, sk / 2);
            fUm = fU;
        }
    }
}

// z_u = W (a r_u + D^T y), z_p = y, with y in FP64 (y64) or FP32 (y32).
__global__ __launch_bounds__(kStreamThreads) void k_mixed_pre2(Level<double> L, const double *__restrict__ r, double a,
                                                               const double *__restrict__ y64,
                                                               const float *__restrict__ y32, double *__restrict__ z)
{
    int col, k0;
    bool active;
    stream_coords<kMixedKC>(L, col, k0, active);
    const int nz = L.nz;
    const size_t m = (size_t)nz * L.plane;
    const MixedRows R(L, col);
    const Rsrc rE = make_rsrc(r, m * 8), rN = make_rsrc(r + m, m * 8), rU = make_rsrc(r + 2 * m, m * 8);
    const Rsrc zE = make_rsrc(z, m * 8), zN = make_rsrc(z + m, m * 8), zU = make_rsrc(z + 2 * m, m * 8),
               zP = make_rsrc(z + 3 * m, m * 8);
    // y: the V-cycle's output, tiled storage
    const bool f32 = y32 != nullptr;
    const Rsrc ry = f32 ? make_rsrc(y32, m * 4) : make_rsrc(y64, m * 8);
    auto Y = [&](unsigned voff, unsigned soff) -> double {
        return f32 ? (double)bload(float(), ry, voff / 2, soff / 2) : bload(double(), ry, voff, soff);
    };
    const unsigned oo = active ? R.vc : 0xFFFFFFFFu;
#pragma unroll
    for (int tt = 0; tt < kMixedKC; ++tt) {
        const int k = k0 + tt;
        if (k < nz) {
            const unsigned sk = (unsigned)k * R.pstride, vk = (unsigned)k * R.vstride;
            const double h = L.wh[k];
            const double yp = Y(R.oc, sk);
            const double ze = h * ld(R.cE, R.oc, sk) * (a * ld(rE, R.vc, vk) + (yp - Y(R.oe, sk)));
            const double zn = h * ld(R.cN, R.oc, sk) * (a * ld(rN, R.vc, vk) + (yp - Y(R.on, sk)));
            const double zu = (k + 1 < nz)
                                  ? L.wz[k] * ld(R.cU, R.oc, sk) * (a * ld(rU, R.vc, vk) + (yp - Y(R.oc, sk + R.pstride)))
                                  : 0.0;
            bstore(ze, zE, oo, vk);
            bstore(zn, zN, oo, vk);
            bstore(zu, zU, oo, vk);
            bstore(yp, zP, oo, vk);
        }
    }
}

// ---- vector kernels of the outer GMRES -------------------------------------

struct VecSet {
    const double *v[kMultiMax];
    double a[kMultiMax];
};

// partials[i * G + block] = block part of (w, v_i), i < NV.
template <int NV>
__global__ __launch_bounds__(256) void k_multidot(size_t n, const double *__restrict__ w, VecSet S,
                                                  double *__restrict__ partials)
{
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256) {
        const double wq = w[g];
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += wq * S.v[i][g];
    }
    block_partials<NV>(acc, partials, gridDim.x, blockIdx.x);
}

// y += sum_i a_i v_i; with partials, also the block parts of (y, y) afterwards.
template <int NV>
__global__ __launch_bounds__(256) void k_multiaxpy(size_t n, double *__restrict__ y, VecSet S,
                                                   double *__restrict__ partials)
{
    double nrm = 0.0;
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256) {
        double s = y[g];
#pragma unroll
        for (int i = 0; i < NV; ++i) s += S.a[i] * S.v[i][g];
        y[g] = s;
        nrm += s * s;
    }
    if (partials) {
        double v[1] = {nrm};
        block_partials<1>(v, partials, gridDim.x, blockIdx.x);
    }
}

// y += sum_i a_i v_i, then the block parts of (y, v_i), i < NV, and (y, y):
// the second Gram-Schmidt pass's dots ride on the first pass's update.
template <int NV>
__global__ __launch_bounds__(256) void k_multiaxpy_dot(size_t n, double *__restrict__ y, VecSet S,
                                                       double *__restrict__ partials)
{
    double acc[NV + 1];
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256) {
        double v[NV];
        double s = y[g];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            v[i] = S.v[i][g];
            s += S.a[i] * v[i];
        }
        y[g] = s;
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += s * v[i];
        acc[NV] += s * s;
    }
    block_partials<NV + 1>(acc, partials, gridDim.x, blockIdx.x);
}

// Delayed reorthogonalisation (one pass over the basis per Arnoldi step).
// u holds the previous step's once-orthogonalised vector; it is corrected
// and normalised here, q = u / rho - sum_i ca_i v_i, while the new vector is
// orthogonalised against the corrected basis, w' = w - sum_i cw_i v_i - hq q,
// and the block parts of (sd_i v_i, w'), i < NV, (q, w') and (w', w') are
// formed for the next step's correction.  u <- q and w <- w' in place.
struct CorrSet {
    const double *v[kMultiMax];
    double ca[kMultiMax], cw[kMultiMax], sd[kMultiMax];
};

template <int NV>
__global__ __launch_bounds__(256) void k_corr_axpy_dot(size_t n, double *__restrict__ u, double *__restrict__ w,
                                                       CorrSet S, double inv_rho, double hq,
                                                       double *__restrict__ partials)
{
    double acc[NV + 2];
#pragma unroll
    for (int i = 0; i < NV + 2; ++i) acc[i] = 0.0;
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256) {
        double v[NV];
        double q = u[g] * inv_rho, y = w[g];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            v[i] = S.v[i][g];
            q -= S.ca[i] * v[i];
            y -= S.cw[i] * v[i];
        }
        y -= hq * q;
        u[g] = q;
        w[g] = y;
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += S.sd[i] * v[i] * y;
        acc[NV] += q * y;
        acc[NV + 1] += y * y;
    }
    block_partials<NV + 2>(acc, partials, gridDim.x, blockIdx.x);
}

// y = a x + b z (z may be null: y = a x).
__global__ __launch_bounds__(256) void k_axpby(size_t n, double a, const double *__restrict__ x, double b,
                                               const double *__restrict__ z, double *__restrict__ y)
{
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256)
        y[g] = z ? a * x[g] + b * z[g] : a * x[g];
}

// out[v] = fixed-order sum of the G values partials[v * G ...].
__global__ __launch_bounds__(256) void k_sum_values(const double *__restrict__ partials, int G,
                                                    double *__restrict__ out)
{
    __shared__ double sh[256];
    const int v = blockIdx.x;
    const double *pv = partials + (size_t)v * G;
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) s += pv[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = sh[0];
}

template <int NV>
void launch_multidot_n(size_t n, const double *w, const VecSet &S, double *partials, int G, hipStream_t s)
{
    hipLaunchKernelGGL((k_multidot<NV>), dim3(G), dim3(256), 0, s, n, w, S, partials);
}

template <int NV>
void launch_multiaxpy_n(size_t n, double *y, const VecSet &S, double *partials, int G, hipStream_t s)
{
    hipLaunchKernelGGL((k_multiaxpy<NV>), dim3(G), dim3(256), 0, s, n, y, S, partials);
}

template <int NV>
void launch_multiaxpy_dot_n(size_t n, double *y, const VecSet &S, double *partials, int G, hipStream_t s)
{
    hipLaunchKernelGGL((k_multiaxpy_dot<NV>), dim3(G), dim3(256), 0, s, n, y, S, partials);
}

template <int NV>
void launch_corr_n(size_t n, double *u, double *w, const CorrSet &S, double inv_rho, double hq, double *partials,
                   int G, hipStream_t s)
{
    hipLaunchKernelGGL((k_corr_axpy_dot<NV>), dim3(G), dim3(256), 0, s, n, u, w, S, inv_rho, hq, partials);
}

// Calls f(std::integral_constant<int, NV>) for 1 <= nv <= kMultiMax.
template <int NV = 1, class F>
void dispatch_nv(int nv, F &&f)
{
    if constexpr (NV < kMultiMax) {
        if (nv > NV) {
            dispatch_nv<NV + 1>(nv, f);
            return;
        }
    }
    f(std::integral_constant<int, NV>());
}

// Partials per dot of the vector kernels: about four elements per thread,
// within the partial-sum buffer.
int vec_grid(size_t n) { return grid_for(n, 4, 256); }

}  // namespace

hipError_t launch_mixed_apply(const Level<double> &L, const double *x, double *y, hipStream_t s)
{
    const int ncb = (L.plane + kStreamThreads - 1) / kStreamThreads;
    const int G = ncb * ((L.nz + kMixedKC - 1) / kMixedKC);
    hipLaunchKernelGGL(k_mixed_apply, dim3(G), dim3(kStreamThreads), 0, s, L, x, y);
    return hipGetLastError();
}

hipError_t launch_mixed_pre1(const Level<double> &L, const double *r, double a, double *t, float *t32, hipStream_t s)
{
    const int ncb = (L.plane + kStreamThreads - 1) / kStreamThreads;
    const int G = ncb * ((L.nz + kMixedKC - 1) / kMixedKC);
    hipLaunchKernelGGL(k_mixed_pre1, dim3(G), dim3(kStreamThreads), 0, s, L, r, a, t, t32);
    return hipGetLastError();
}

hipError_t launch_mixed_pre2(const Level<double> &L, const double *r, double a, const double *y64, const float *y32,
                             double *z, hipStream_t s)
{
    const int ncb = (L.plane + kStreamThreads - 1) / kStreamThreads;
    const int G = ncb * ((L.nz + kMixedKC - 1) / kMixedKC);
    hipLaunchKernelGGL(k_mixed_pre2, dim3(G), dim3(kStreamThreads), 0, s, L, r, a, y64, y32, z);
    return hipGetLastError();
}

hipError_t launch_multidot(size_t n, const double *w, const double *const *v, int nv, double *partials,
                           double *stage, double *out, hipStream_t s)
{
    if (nv < 1 || nv > kMultiMax) return hipErrorInvalidValue;
    VecSet S{};
    for (int i = 0; i < nv; ++i) S.v[i] = v[i];
    const int G = vec_grid(n);
    dispatch_nv(nv, [&](auto NVc) { launch_multidot_n<decltype(NVc)::value>(n, w, S, partials, G, s); });
    return launch_sum_partials(partials, G, nv, stage, out, s);
}

hipError_t launch_multiaxpy(size_t n, double *y, const double *const *v, const double *a, int nv,
                            double *norm_partials, int *nblocks_out, hipStream_t s)
{
    if (nv < 1 || nv > kMultiMax) return hipErrorInvalidValue;
    VecSet S{};
    for (int i = 0; i < nv; ++i) {
        S.v[i] = v[i];
        S.a[i] = a[i];
    }
    const int G = vec_grid(n);
    if (nblocks_out) *nblocks_out = G;
    dispatch_nv(nv, [&](auto NVc) { launch_multiaxpy_n<decltype(NVc)::value>(n, y, S, norm_partials, G, s); });
    return hipGetLastError();
}

hipError_t launch_multiaxpy_dot(size_t n, double *y, const double *const *v, const double *a, int nv,
                                double *partials, double *stage, double *out, hipStream_t s)
{
    if (nv < 1 || nv > kMultiMax) return hipErrorInvalidValue;
    VecSet S{};
    for (int i = 0; i < nv; ++i) {
        S.v[i] = v[i];
        S.a[i] = a[i];
    }
    const int G = vec_grid(n);
    dispatch_nv(nv, [&](auto NVc) { launch_multiaxpy_dot_n<decltype(NVc)::value>(n, y, S, partials, G, s); });
    return launch_sum_partials(partials, G, nv + 1, stage, out, s);
}

hipError_t launch_corr_axpy_dot(size_t n, double *u, double *w, const double *const *v, const double *ca,
                                const double *cw, const double *sd, int nv, double inv_rho, double hq,
                                double *partials, double *stage, double *out, hipStream_t s)
{
    if (nv < 1 || nv > kMultiMax) return hipErrorInvalidValue;
    CorrSet S{};
    for (int i = 0; i < nv; ++i) {
        S.v[i] = v[i];
        S.ca[i] = ca[i];
        S.cw[i] = cw[i];
        S.sd[i] = sd[i];
    }
    const int G = vec_grid(n);
    dispatch_nv(nv, [&](auto NVc) { launch_corr_n<decltype(NVc)::value>(n, u, w, S, inv_rho, hq, partials, G, s); });
    return launch_sum_partials(partials, G, nv + 2, stage, out, s);
}

hipError_t launch_axpby(size_t n, double a, const double *x, double b, const double *z, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n, 1)), dim3(256), 0, s, n, a, x, b, z, y);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partials, int G, int nvals, double *stage, double *out, hipStream_t s)
{
    if (G > 8 * kReduceSegs) {
        hipLaunchKernelGGL(k_reduce_partials, dim3(kReduceSegs, nvals), dim3(256), 0, s, partials, G, stage);
        partials = stage;
        G = kReduceSegs;
    }
    hipLaunchKernelGGL(k_sum_values, dim3(nvals), dim3(256), 0, s, partials, G, out);
    return hipGetLastError();
}

}  // namespace tpmg
