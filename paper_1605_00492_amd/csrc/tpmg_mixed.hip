// HIP kernels for the velocity-pressure system around the pressure solve
// (Mitchell & Mueller, Sec. 4.2, Eq. PressureVelocitySystem with buoyancy
// eliminated), its Schur-complement preconditioner (Eq. SchurComplement with
// the lumped mass of Eq. LumpedMass) and the vector kernels of the outer
// restarted GMRES (Sec. 5).
//
// Finest level only, FP64, level-major mixed vectors [uE | uN | uU | p]:
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

__device__ __forceinline__ double wface_h(const Level<double> &L, const double *c, size_t o, int k)
{
    return L.wh[k] * c[o];
}

// y = A x.
__global__ __launch_bounds__(kStreamThreads) void k_mixed_apply(Level<double> L, const double *__restrict__ x,
                                                                double *__restrict__ y)
{
    int col, k0;
    bool active;
    stream_coords<kMixedKC>(L, col, k0, active);
    const int nz = L.nz, plane = L.plane;
    const size_t m = (size_t)nz * plane;
    const Nbr nb = neighbours(col, L.n, plane);
    const double *xE = x, *xN = x + m, *xU = x + 2 * m, *xP = x + 3 * m;
    double *yE = y, *yN = y + m, *yU = y + 2 * m, *yP = y + 3 * m;
    const double *cE = L.c, *cN = L.c + m, *cU = L.c + 2 * m;
    // vertical window: U face below the cell (weight, value)
    double wUm = 0, xUm = 0;
    if (k0 > 0 && k0 - 1 < nz - 1) {
        const size_t om = (size_t)(k0 - 1) * plane + col;
        wUm = L.wz[k0 - 1] * cU[om];
        xUm = xU[om];
    }
#pragma unroll 2
    for (int t = 0; t < kMixedKC; ++t) {
        const int k = k0 + t;
        if (k >= nz) break;
        const size_t o = (size_t)k * plane;
        const size_t pc = o + col;
        const double xp = xP[pc];
        // east faces: own, west neighbour's, east neighbour's
        const double we = wface_h(L, cE, pc, k), ww = wface_h(L, cE, o + nb.w, k), wee = wface_h(L, cE, o + nb.e, k);
        const double xe = xE[pc], xw = xE[o + nb.w], xee = xE[o + nb.e];
        const double ye = xe / we + 0.25 * (xw / sqrt(we * ww) + xee / sqrt(we * wee)) - (xp - xP[o + nb.e]);
        // north faces
        const double wn = wface_h(L, cN, pc, k), ws = wface_h(L, cN, o + nb.s, k), wnn = wface_h(L, cN, o + nb.n, k);
        const double xn = xN[pc], xs = xN[o + nb.s], xnn = xN[o + nb.n];
        const double yn = xn / wn + 0.25 * (xs / sqrt(wn * ws) + xnn / sqrt(wn * wnn)) - (xp - xP[o + nb.n]);
        // upper face (none above the top cell)
        double yu = 0, xu = 0, wu = 0;
        if (k + 1 < nz) {
            wu = L.wz[k] * cU[pc];
            xu = xU[pc];
            double acc = xu / wu;
            if (k >= 1) acc += 0.25 * xUm / sqrt(wu * wUm);
            if (k + 2 < nz) {
                const double wup = L.wz[k + 1] * cU[pc + plane];
                acc += 0.25 * xU[pc + plane] / sqrt(wu * wup);
            }
            yu = acc - (xp - xP[pc + plane]);
        }
        const double yp = (xe - xw) + (xn - xs) + (xu - xUm) + L.mu[k] * xp;
        if (active) {
            yE[pc] = ye;
            yN[pc] = yn;
            yU[pc] = yu;
            yP[pc] = yp;
        }
        wUm = wu;
        xUm = xu;
    }
}

// t = r_p - D (W r_u); also fl32(t) when t32 is given.
__global__ __launch_bounds__(kStreamThreads) void k_mixed_pre1(Level<double> L, const double *__restrict__ r,
                                                               double *__restrict__ t, float *__restrict__ t32)
{
    int col, k0;
    bool active;
    stream_coords<kMixedKC>(L, col, k0, active);
    const int nz = L.nz, plane = L.plane;
    const size_t m = (size_t)nz * plane;
    const Nbr nb = neighbours(col, L.n, plane);
    const double *rE = r, *rN = r + m, *rU = r + 2 * m, *rP = r + 3 * m;
    const double *cE = L.c, *cN = L.c + m, *cU = L.c + 2 * m;
    double fUm = 0;  // W r on the U face below
    if (k0 > 0 && k0 - 1 < nz - 1) {
        const size_t om = (size_t)(k0 - 1) * plane + col;
        fUm = L.wz[k0 - 1] * cU[om] * rU[om];
    }
#pragma unroll 4
    for (int tt = 0; tt < kMixedKC; ++tt) {
        const int k = k0 + tt;
        if (k >= nz) break;
        const size_t o = (size_t)k * plane;
        const size_t pc = o + col;
        const double h = L.wh[k];
        const double fU = (k + 1 < nz) ? L.wz[k] * cU[pc] * rU[pc] : 0.0;
        const double div = (h * cE[pc] * rE[pc] - h * cE[o + nb.w] * rE[o + nb.w]) +
                           (h * cN[pc] * rN[pc] - h * cN[o + nb.s] * rN[o + nb.s]) + (fU - fUm);
        const double tv = rP[pc] - div;
        if (active) {
            t[pc] = tv;
            if (t32) t32[pc] = (float)tv;
        }
        fUm = fU;
    }
}

// z_u = W (r_u + D^T y), z_p = y, with y in FP64 (y64) or FP32 (y32).
__global__ __launch_bounds__(kStreamThreads) void k_mixed_pre2(Level<double> L, const double *__restrict__ r,
                                                               const double *__restrict__ y64,
                                                               const float *__restrict__ y32, double *__restrict__ z)
{
    int col, k0;
    bool active;
    stream_coords<kMixedKC>(L, col, k0, active);
    const int nz = L.nz, plane = L.plane;
    const size_t m = (size_t)nz * plane;
    const Nbr nb = neighbours(col, L.n, plane);
    const double *rE = r, *rN = r + m, *rU = r + 2 * m;
    double *zE = z, *zN = z + m, *zU = z + 2 * m, *zP = z + 3 * m;
    const double *cE = L.c, *cN = L.c + m, *cU = L.c + 2 * m;
    auto Y = [&](size_t q) -> double { return y32 ? (double)y32[q] : y64[q]; };
#pragma unroll 4
    for (int tt = 0; tt < kMixedKC; ++tt) {
        const int k = k0 + tt;
        if (k >= nz) break;
        const size_t o = (size_t)k * plane;
        const size_t pc = o + col;
        const double h = L.wh[k];
        const double yp = Y(pc);
        const double ze = h * cE[pc] * (rE[pc] + (yp - Y(o + nb.e)));
        const double zn = h * cN[pc] * (rN[pc] + (yp - Y(o + nb.n)));
        const double zu = (k + 1 < nz) ? L.wz[k] * cU[pc] * (rU[pc] + (yp - Y(pc + plane))) : 0.0;
        if (active) {
            zE[pc] = ze;
            zN[pc] = zn;
            zU[pc] = zu;
            zP[pc] = yp;
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

hipError_t launch_mixed_pre1(const Level<double> &L, const double *r, double *t, float *t32, hipStream_t s)
{
    const int ncb = (L.plane + kStreamThreads - 1) / kStreamThreads;
    const int G = ncb * ((L.nz + kMixedKC - 1) / kMixedKC);
    hipLaunchKernelGGL(k_mixed_pre1, dim3(G), dim3(kStreamThreads), 0, s, L, r, t, t32);
    return hipGetLastError();
}

hipError_t launch_mixed_pre2(const Level<double> &L, const double *r, const double *y64, const float *y32, double *z,
                             hipStream_t s)
{
    const int ncb = (L.plane + kStreamThreads - 1) / kStreamThreads;
    const int G = ncb * ((L.nz + kMixedKC - 1) / kMixedKC);
    hipLaunchKernelGGL(k_mixed_pre2, dim3(G), dim3(kStreamThreads), 0, s, L, r, y64, y32, z);
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
