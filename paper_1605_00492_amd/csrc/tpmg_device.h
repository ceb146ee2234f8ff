// Device helpers shared by the kernel sources (tpmg_kernels.hip,
// tpmg_mixed.hip): XCD-aware block order, buffer-descriptor loads and stores,
// periodic neighbours, fixed-order block reductions, and small host helpers
// for launch shapes.  Not part of the public interface.
#pragma once

#include <cstdlib>

#include "tpmg_internal.h"

namespace tpmg {

namespace {

constexpr int kXcds = 8;
constexpr int kStreamThreads = 256;
// Elementwise CG kernels: workgroups of 256 (1024 streamed slower on MI355X).
constexpr int kCgThreads = 256;
constexpr double kDblMax = 1.7976931348623157e308;

// Workgroups are dispatched to the XCDs round-robin.  Renumber them so that
// each XCD processes one contiguous range of tiles (neighbouring rows share
// that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int G)
{
    const int per = G / kXcds, rem = G % kXcds;
    const int x = b % kXcds, idx = b / kXcds;
    return (x < rem) ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

// 1/x: the hardware reciprocal in FP32 (1 ulp), IEEE division in FP64.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Element idx of a wave-uniform row pointer, with the byte offset formed in
// 32 bits so that the load uses a scalar base + 32-bit vector offset (rows
// hold fewer than 2^29 elements).
template <typename T>
__device__ __forceinline__ T ldrow(const T *base, unsigned idx)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * (unsigned)sizeof(T));
}

// Raw buffer access: a 128-bit descriptor per array (scalar registers), a
// per-lane byte offset and a wave-uniform byte offset (the k plane).  Reads
// beyond the descriptor's size return 0 and writes beyond it are dropped.
// Arrays addressed this way hold fewer than 2^32 bytes.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit data format (gfx9 family)

__device__ __forceinline__ Rsrc make_rsrc(const void *p, size_t bytes)
{
    const unsigned n = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, kRsrcWord3);
}

// AUX: the cache policy of the access; kNT (2) marks it non-temporal, a
// stream the L2 should give up first (data read or written once), so that
// lines other workgroups will read again stay resident.
constexpr int kNT = 2;
template <int AUX = 0>
__device__ __forceinline__ float bload(float, Rsrc r, unsigned voff, unsigned soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ double bload(double, Rsrc r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ void bstore(float v, Rsrc r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void bstore(double v, Rsrc r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          (int)voff, (int)soff, AUX);
}

struct Nbr {
    int e, w, n, s;
};

// Periodic horizontal neighbours of column `col` on an n x n plane.
__device__ __forceinline__ Nbr neighbours(int col, int n, int plane)
{
    const int i = col % n, j = col / n;
    Nbr r;
    r.e = (i + 1 == n) ? col + 1 - n : col + 1;
    r.w = (i == 0) ? col + n - 1 : col - 1;
    r.n = (j + 1 == n) ? col + n - plane : col + n;
    r.s = (j == 0) ? col + plane - n : col - n;
    return r;
}

// Parent column on the next coarser level (natural embedding).
__device__ __forceinline__ int parent(int col, int n)
{
    const int i = col % n, j = col / n;
    return (j >> 1) * (n >> 1) + (i >> 1);
}

// Deterministic block reduction of NV values: wavefront shuffle, then the
// wavefront sums in fixed order; thread 0 writes partials[v * G + bid].
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *partials, int G, int bid)
{
    __shared__ double sh[NV][16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += __shfl_down(v[i], off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[i][w] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = 0.0;
            for (int q = 0; q < nw; ++q) s += sh[i][q];
            partials[(size_t)i * G + bid] = s;
        }
    }
}

// First stage for many partials: workgroup (s, v) sums the contiguous segment
// s of value v's G partials in a fixed order, so the single-workgroup
// finalisation reads kReduceSegs values instead of G.
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ partials, int G,
                                                         double *__restrict__ out)
{
    const int v = blockIdx.y, seg = blockIdx.x;
    const int lo = (int)((long long)G * seg / kReduceSegs), hi = (int)((long long)G * (seg + 1) / kReduceSegs);
    const double *pv = partials + (size_t)v * G;
    double acc = 0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) acc += pv[i];
    double vv[1] = {acc};
    block_partials<1>(vv, out + (size_t)v * kReduceSegs, kReduceSegs, seg);
}

// Byte offset of cell (col, 0) of a level's tiled storage; level k adds
// k * tile_width(plane) * sizeof(T) (arrays hold fewer than 2^32 bytes).
template <typename T>
__device__ __forceinline__ unsigned cell_off(const Level<T> &L, unsigned col)
{
    return (unsigned)cell_base(col, L.plane, L.nz) * (unsigned)sizeof(T);
}

// Kernels that visit a level's storage element by element (256 threads per
// workgroup): wavefront w covers elements 64 w .. 64 w + 63, so in the tiled
// storage it covers one (tile, k) and its division stays scalar.
__device__ __forceinline__ unsigned storage_wave()
{
    return blockIdx.x * 4u + (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}
// (col, k) of storage element g = 64 w + lane of a level (g < 2^31).
__device__ __forceinline__ void storage_coords(unsigned g, unsigned w, int plane, int nz, unsigned &col, int &k)
{
    if ((plane & 63) == 0) {
        const unsigned tile = w / (unsigned)nz;
        k = (int)(w - tile * (unsigned)nz);
        col = tile * 64u + (g & 63u);
    } else {
        k = (int)(g / (unsigned)plane);
        col = g - (unsigned)k * (unsigned)plane;
    }
}

// Streaming stencils: thread = (column, chunk of KC cells along k), blocks
// of kStreamThreads columns, the k-chunks outermost.
template <int KC, typename T>
__device__ __forceinline__ void stream_coords(const Level<T> &L, int &col, int &k0, bool &active)
{
    const int ncb = (L.plane + kStreamThreads - 1) / kStreamThreads;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int kc = blk / ncb, cb = blk % ncb;
    col = cb * kStreamThreads + threadIdx.x;
    k0 = kc * KC;
    active = col < L.plane;
    if (!active) col = 0;
}

// One stencil row of H: buffer descriptors and lane offsets shared by the
// streaming kernels (operator apply, residual, CG direction update).
template <typename T>
struct StencilRows {
    Rsrc rE, rN, rU;
    unsigned oc, oe, ow, on, os, pstride;
    __device__ StencilRows(const Level<T> &L, unsigned col)
    {
        const size_t fstride = (size_t)L.nz * L.plane;
        rE = make_rsrc(L.c, fstride * sizeof(T));
        rN = make_rsrc(L.c + fstride, fstride * sizeof(T));
        rU = make_rsrc(L.c + 2 * fstride, fstride * sizeof(T));
        const Nbr nb = neighbours(col, L.n, L.plane);
        oc = cell_off<T>(L, col);
        oe = cell_off<T>(L, nb.e);
        ow = cell_off<T>(L, nb.w);
        on = cell_off<T>(L, nb.n);
        os = cell_off<T>(L, nb.s);
        pstride = (unsigned)tile_width(L.plane) * sizeof(T);
    }
};

inline int grid_for(size_t n, int per_thread = 4, int block = 256)
{
    size_t g = (n + (size_t)block * per_thread - 1) / ((size_t)block * per_thread);
    if (g < 1) g = 1;
    if (g > (size_t)kMaxPartials) g = kMaxPartials;
    return (int)g;
}

// Tuning overrides (environment): TPMG_SWEEP_M = cells per chunk (4, 8, 16),
// TPMG_SWEEP_CPW = chunks per wavefront (1, 2), TPMG_SWEEP_BI / _BJ = tile
// block shape, TPMG_KCHUNK = cells along k per thread of the streaming
// kernels (4, 8, 16); -1 when unset.
inline int env_int(const char *name)
{
    const char *v = getenv(name);
    return v ? atoi(v) : -1;
}

}  // namespace

}  // namespace tpmg
