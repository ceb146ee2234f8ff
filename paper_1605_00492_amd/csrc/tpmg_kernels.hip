// HIP kernels for gfx950 (MI355X): tensor-product multigrid on the lumped
// pressure operator of Mitchell & Mueller (Sec. 4.2) with vertical line
// relaxation (Sec. 4.2, 4.3.1), 2x2 horizontal transfers (Sec. 3.2) and the
// CG building blocks of the outer solve.
//
// Every kernel is bandwidth-bound (about 0.5 flop/byte), so the design is
// about HBM traffic, not the matrix cores:
//  * tiled storage (64 columns per tile, the tile's levels contiguous): a
//    wavefront holds the 64 columns of a tile, so every load of a level is
//    one 256- or 512-byte segment and stepping k reads the next segment
//    (sequential streams per wavefront; the level-major order, whose levels
//    lie a whole plane apart, streamed 10 % slower in the sweep);
//  * horizontal neighbours come through the caches from the same or the
//    adjacent rows, which the XCD-aware block order keeps in one XCD's L2;
//  * vertical neighbours live in registers (sliding window along k);
//  * the column solve keeps its whole state in registers: a column is split
//    into P chunks of M cells, one wavefront per chunk, each chunk eliminated
//    locally and the P chunks coupled through a small system in LDS.
#include <cstdlib>
#include <type_traits>

#include "tpmg_device.h"

namespace tpmg {

namespace {

// ---------------------------------------------------------------------------
// Line relaxation sweep.
//
//   out = u + omega * H_z^{-1} (b - H u)          (Sec. 4.2, block Jacobi)
//
// A column of nz cells is split into Q chunks of M cells.  A workgroup holds
// the chunks of 64 columns; each of its P wavefronts advances CPW chunks in
// lockstep (chunk q = c * P + p), so one step of a wavefront issues the loads
// of CPW cells at once.  For each chunk a lane
//  1. streams k upward, forming the residual r_k, the row excess
//       e_k = delta_k + w_{k-1/2} e_{k-1} / (w_{k-1/2} + e_{k-1})
//     (delta_k = mass + horizontal couplings), pivots p_k = e_k + w_{k+1/2}
//     and the forward eliminations of r and of the unit coupling to the
//     chunk below (all terms positive: no cancellation in the pivots);
//  2. back-substitutes to the chunk solution xp with the neighbouring chunks
//     held at zero, the spike vectors alpha, beta (response to the cell just
//     below / above the chunk) and, in FP32, gamma = T^{-1} delta (response to
//     the row excesses; alpha + beta + gamma = 1, so 1 - alpha - beta is never
//     formed by subtraction in FP32);
//  3. publishes the chunk-end values to LDS; wavefront 0 solves, per column,
//     the system coupling first/last cells of all chunks by a forward /
//     backward recurrence over chunks whose denominators are sums of positive
//     terms;
//  4. forms x = xp + alpha x_below + beta x_above and writes u + omega x.
// The per-lane state (u, xp, alpha, beta[, gamma] for CPW x M cells) stays in
// registers; loads use buffer descriptors with a per-k scalar offset.
// ---------------------------------------------------------------------------
// Elimination state of one chunk of one column (one lane): the chunk's
// forward-eliminated right-hand side sy, the responses se / sg to a unit
// value just below / above the chunk and, in FP32, sd = T^{-1} delta.
template <typename T, int M>
struct ChunkState {
    static constexpr bool kGamma = sizeof(T) == 4;
    T sy[M], se[M], sg[M], sd[kGamma ? M : 1];
    T e_prev, y_prev, eta_prev, g_prev, c_prev;

    __device__ __forceinline__ void init()
    {
        e_prev = T(1);
        y_prev = eta_prev = g_prev = c_prev = T(0);
    }
    // Cell t of the chunk: residual r, diagonal excess delta (mass plus
    // horizontal couplings), couplings wU above and wD below.
    __device__ __forceinline__ void step(int t, T r, T delta, T wU, T wD)
    {
        const T e = (t == 0) ? delta + wD : delta + wD * e_prev * recip(wD + e_prev);
        const T ip = recip(e + wU);
        const T g = wU * ip;
        const T y = (t == 0) ? r : r + g_prev * y_prev;
        const T eta = (t == 0) ? wD : g_prev * eta_prev;
        sy[t] = y * ip;
        se[t] = eta * ip;
        sg[t] = g;
        if constexpr (kGamma) {
            const T cg = (t == 0) ? delta : delta + g_prev * c_prev;
            sd[t] = cg * ip;
            c_prev = cg;
        }
        e_prev = e;
        y_prev = y;
        eta_prev = eta;
        g_prev = g;
    }
    // rows beyond the column: decoupled identity rows (x = 0)
    __device__ __forceinline__ void identity(int t)
    {
        sy[t] = se[t] = sg[t] = T(0);
        if constexpr (kGamma) sd[t] = T(1);
    }
    // Back substitution inside the chunk: xp, alpha (unit value below), beta
    // (unit value above) and, in FP32, gamma (row excesses; chunk ends only).
    // Then the chunk-end values go to rp[8][64] for the coupling system.
    __device__ __forceinline__ void backsub_publish(T *rp, int lane)
    {
        T gam_s = 0, gam_e = 0;
        T xn = 0, an = 0, bn = 0, cn = 0;
#pragma unroll
        for (int t = M - 1; t >= 0; --t) {
            const T g = sg[t];
            const T xp = sy[t] + g * xn;
            const T al = se[t] + g * an;
            const T be = (t == M - 1) ? g : g * bn;
            if constexpr (kGamma) {
                const T ga = sd[t] + g * cn;
                if (t == M - 1) gam_e = ga;
                cn = ga;
            }
            sy[t] = xp;
            se[t] = al;
            sg[t] = be;
            xn = xp;
            an = al;
            bn = be;
        }
        if constexpr (kGamma) {
            gam_s = cn;
        } else {
            gam_s = T(1) - se[0] - sg[0];
            gam_e = T(1) - se[M - 1] - sg[M - 1];
        }
        rp[lane] = sy[0];
        rp[64 + lane] = se[0];
        rp[128 + lane] = sg[0];
        rp[192 + lane] = gam_s;
        rp[256 + lane] = sy[M - 1];
        rp[320 + lane] = se[M - 1];
        rp[384 + lane] = sg[M - 1];
        rp[448 + lane] = gam_e;
    }
    // Chunk solution at cell t given the cells just below / above the chunk.
    __device__ __forceinline__ T value(int t, T xlo, T xhi) const { return sy[t] + se[t] * xlo + sg[t] * xhi; }
};

// The system coupling the chunks of one column (lane), solved by one
// wavefront.  Chunk q, first cell F_q and last cell L_q:
//   F_q = xs + as L_{q-1} + bs F_{q+1},   L_q = xe + ae L_{q-1} + be F_{q+1}.
// Forward over chunks with L_{q-1} = phi + psi F_q gives
//   F_q = sig + tau F_{q+1},  L_q = phi' + psi' F_{q+1},
// where 1 - as psi = (bs + gs) + as (1 - psi) and 1 - psi is carried by its
// own positive recurrence.  On return red[q][4][.] = L_q, red[q][5][.] = F_q.
template <typename T>
__device__ __forceinline__ void coupling_solve(T *red, int Q, int lane)
{
    T phi = 0, psi = 0, psib = 1;
    for (int q = 0; q < Q; ++q) {
        T *rq = red + (size_t)q * 512;
        const T xs = rq[lane], as = rq[64 + lane], bs = rq[128 + lane], gs = rq[192 + lane];
        const T xe = rq[256 + lane], ae = rq[320 + lane], be = rq[384 + lane], ge = rq[448 + lane];
        const T den = (bs + gs) + as * psib;
        const T rden = recip(den);
        const T sig = (xs + as * phi) * rden;
        const T tau = bs * rden;
        const T phin = xe + ae * (phi + psi * sig);
        const T psin = be + ae * psi * tau;
        const T psibn = ge + ae * (psib + psi * gs) * rden;
        rq[lane] = sig;
        rq[64 + lane] = tau;
        rq[128 + lane] = phin;
        rq[192 + lane] = psin;
        phi = phin;
        psi = psin;
        psib = psibn;
    }
    T Fn = 0;
    for (int q = Q - 1; q >= 0; --q) {
        T *rq = red + (size_t)q * 512;
        const T F = rq[lane] + rq[64 + lane] * Fn;
        const T Lq = rq[128 + lane] + rq[192 + lane] * Fn;
        rq[256 + lane] = Lq;
        rq[320 + lane] = F;
        Fn = F;
    }
}

template <typename T>
struct SweepRaw {
    T uup, uE, uW, uN, uS, b, cE, cEw, cN, cNs, cU, eup;
};

// Wavefront shifts by one lane (DPP): lane i receives v from lane i - 1
// (lane_from_prev) or i + 1 (lane_from_next); the lane without a source
// (0, resp. 63) keeps `edge`.  All 64 lanes must be active.
__device__ __forceinline__ int dpp_shr1(int edge, int v) { return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_shl1(int edge, int v) { return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xF, 0xF, false); }
__device__ __forceinline__ float lane_from_prev(float edge, float v)
{
    return __int_as_float(dpp_shr1(__float_as_int(edge), __float_as_int(v)));
}
__device__ __forceinline__ float lane_from_next(float edge, float v)
{
    return __int_as_float(dpp_shl1(__float_as_int(edge), __float_as_int(v)));
}
__device__ __forceinline__ double lane_from_prev(double edge, double v)
{
    const long long e = __double_as_longlong(edge), x = __double_as_longlong(v);
    const int lo = dpp_shr1((int)e, (int)x), hi = dpp_shr1((int)(e >> 32), (int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_from_next(double edge, double v)
{
    const long long e = __double_as_longlong(edge), x = __double_as_longlong(v);
    const int lo = dpp_shl1((int)e, (int)x), hi = dpp_shl1((int)(e >> 32), (int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Tile order of the sweep: tiles (64 columns of one row) are grouped into
// blocks of bi tiles x bj rows numbered consecutively, so that the workgroups
// resident on one XCD cover a compact patch and share neighbouring rows in L2.
__device__ __forceinline__ int sweep_tile(int t, int n, int bi, int bj)
{
    if (bi <= 0 || (n & 63)) return t;
    const int TR = n >> 6;
    if (TR % bi || n % bj) return t;
    const int per = bi * bj, B = t / per, r = t % per, nbi = TR / bi;
    const int it = (B % nbi) * bi + r % bi, j = (B / nbi) * bj + r / bi;
    return j * TR + it;
}

// A cell offset split into a per-lane part (vector register) and a
// wave-uniform part (scalar register, added to the k-plane offset).
struct Off {
    unsigned v, s;
};

// Per-lane part of the offset of coarse column ic in a row of a tiled level
// whose rows are whole tiles.
__device__ __forceinline__ unsigned row_lane_off(unsigned ic, int nz, unsigned S)
{
    return ((ic >> 6) * (unsigned)nz * 64u + (ic & 63u)) * S;
}

// RM (row mode) 1 and 2: the rows are whole tiles (n % 64 == 0; for the
// prolongation sweep also n / 2 % 64 == 0).  A wavefront then covers 64
// columns of one row, so its north / south (and parent) rows are
// wave-uniform offsets: the buffers are addressed from the lowest of the rows
// involved, with the row part of every offset in a scalar register and only
// the centre, east and west columns (and their parents) per lane.  At its
// 64-VGPR bound the FP32 prolongation sweep then spills 8 instead of 16
// bytes per lane (0.80 vs 0.86 ms at 1024^2 x 128).  RM 2 also takes the
// east / west values of u from the neighbouring lanes (one load at the tile
// edges instead of two per cell) and, in the prolongation sweep, reads one
// parent row less: 13 instead of 16 loads per cell and no spill.
//
// The FP32 prolongation sweep with 8-cell chunks needs more than 64 VGPRs
// with per-lane offsets for all five neighbours; held to 64 (eight
// wavefronts per SIMD, two 1024-thread workgroups per CU) it ran 0.86
// instead of 1.11 ms at 1024^2 x 128.  With per-lane offsets (RM 0: levels
// whose rows are not whole tiles, all small) it is not held, since the spill
// costs more than occupancy gains on a level that fills few CUs.
// CP: cache policy of the data read or written once per cell (b, c_U, the
// output): kNT leaves L2 to the data other workgroups read again (u and c_N
// by the north / south rows, c_E by the east column).
//
// Launch bounds: the FP32 prolongation sweep (8-cell chunks) is held to 64
// VGPRs and the FP64 sweep from zero (16-cell chunks) to 128, so that two
// workgroups share a CU (measured at 1024^2 x 128: FP64 sweep from zero 1.06
// vs 1.21 ms with 28 bytes/lane of spill; the FP64 general sweep, held the
// same way, spills 188 bytes/lane and ran slower).
template <typename T, int M, int CPW, int MODE, int LB, int RM, bool FULL>
constexpr int sweep_min_waves()
{
    if (MODE == SWEEP_PROLONG && LB == 1024 && sizeof(T) == 4 && M == 8 && CPW == 1 && RM != 0 && !FULL) return 8;
    if (MODE == SWEEP_ZERO && LB == 512 && sizeof(T) == 8 && M == 16 && CPW == 1) return 4;
    return 1;
}

template <typename T, int M, int CPW, int MODE, int LB, int RM, int CP, bool FULL>
__global__ __launch_bounds__(LB, (sweep_min_waves<T, M, CPW, MODE, LB, RM, FULL>())) void k_sweep(Level<T> L, const T *__restrict__ u, const T *__restrict__ b,
                                              T *__restrict__ out, const T *__restrict__ ec, T omega,
                                              int tbi, int tbj)
{
    constexpr unsigned S = sizeof(T);
    constexpr bool ROWS = RM != 0;
    // XL: east / west values of u from the neighbouring lanes; XP: in the
    // prolongation sweep, the parent correction of the cell carried along k
    // and reused for whichever of its north / south neighbours shares it.
    constexpr bool XL = RM == 2 && MODE != SWEEP_ZERO;
    constexpr bool XP = XL && MODE == SWEEP_PROLONG;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *red = reinterpret_cast<T *>(smem_raw);  // [Q][8][64]

    const int lane = threadIdx.x & 63;
    const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int P = blockDim.x >> 6;
    const int Q = P * CPW;
    const int tile = sweep_tile(xcd_remap(blockIdx.x, gridDim.x), L.n, tbi, tbj);
    const int col = tile * 64 + lane;
    const int nz = L.nz, plane = L.plane;
    const bool active = ROWS || col < plane;
    const unsigned cc = active ? col : 0;
    const size_t fstride = (size_t)nz * plane;
    const unsigned pstride = (unsigned)tile_width(plane) * S;
    const int nc = L.n >> 1, planec = nc * nc;
    const unsigned cstride = (unsigned)tile_width(planec) * S;

    // Fine offsets C (centre), E, W, N, Sx and parent offsets PC .. PS;
    // fine buffers start at byte fbase, the coarse one at cbase.
    // X (with XL): the neighbour across the tile edge, west for lane 0 and
    // east for lane 63 (the other lanes read their own cell); PX its parent;
    // PO the parent row that differs from the cell's own.
    Off C, E, W, N, Sx, X{0, 0}, PC{0, 0}, PE{0, 0}, PW{0, 0}, PN{0, 0}, PS{0, 0}, PX{0, 0}, PO{0, 0};
    size_t fbase = 0, cbase = 0;
    bool jodd = false;
    if constexpr (ROWS) {
        const int TR = L.n >> 6, j = tile / TR, ti = tile - j * TR;
        const int jn = (j + 1 == L.n) ? 0 : j + 1, js = (j == 0) ? L.n - 1 : j - 1;
        const int j0 = min(j, min(jn, js));
        const unsigned rowb = (unsigned)TR * nz * 64u * S, tileb = (unsigned)nz * 64u * S;
        fbase = (size_t)j0 * rowb;
        const unsigned ov = (unsigned)ti * tileb + (unsigned)lane * S;
        const unsigned oe = lane < 63 ? ov + S : (unsigned)(ti + 1 == TR ? 0 : ti + 1) * tileb;
        const unsigned ow = lane > 0 ? ov - S : (unsigned)(ti == 0 ? TR - 1 : ti - 1) * tileb + 63u * S;
        const unsigned sc = (unsigned)(j - j0) * rowb;
        C = {ov, sc};
        E = {oe, sc};
        W = {ow, sc};
        N = {ov, (unsigned)(jn - j0) * rowb};
        Sx = {ov, (unsigned)(js - j0) * rowb};
        X = {lane == 0 ? ow : (lane == 63 ? oe : ov), sc};
        jodd = j & 1;
        if (MODE == SWEEP_PROLONG) {
            const int jc = j >> 1, jcn = jn >> 1, jcs = js >> 1, jc0 = min(jc, min(jcn, jcs));
            const unsigned rowc = (unsigned)(nc >> 6) * nz * 64u * S;
            cbase = (size_t)jc0 * rowc;
            const unsigned i = (unsigned)(ti * 64 + lane);
            const unsigned ie = (i + 1 == (unsigned)L.n) ? 0u : i + 1, iw = (i == 0) ? (unsigned)L.n - 1 : i - 1;
            const unsigned pv = row_lane_off(i >> 1, nz, S), scc = (unsigned)(jc - jc0) * rowc;
            PC = {pv, scc};
            PE = {row_lane_off(ie >> 1, nz, S), scc};
            PW = {row_lane_off(iw >> 1, nz, S), scc};
            PN = {pv, (unsigned)(jcn - jc0) * rowc};
            PS = {pv, (unsigned)(jcs - jc0) * rowc};
            PX = lane == 0 ? PW : (lane == 63 ? PE : PC);
            // j even: the north neighbour has the cell's parent row, j odd
            // the south one (rows 2 jc and 2 jc + 1 share parent row jc)
            PO = jodd ? PN : PS;
        }
    } else {
        const Nbr nb = neighbours(cc, L.n, plane);
        C = {cell_off(L, cc), 0u};
        E = {cell_off(L, nb.e), 0u};
        W = {cell_off(L, nb.w), 0u};
        N = {cell_off(L, nb.n), 0u};
        Sx = {cell_off(L, nb.s), 0u};
        if (MODE == SWEEP_PROLONG) {
            // Prolongation: every u value read is u + e(parent) (injection).
            auto poff = [&](int q) { return Off{(unsigned)cell_base(parent(q, L.n), planec, nz) * S, 0u}; };
            PC = poff(cc);
            PE = poff(nb.e);
            PW = poff(nb.w);
            PN = poff(nb.n);
            PS = poff(nb.s);
        }
    }
    auto rs = [&](const T *a, size_t base, size_t bytes) {
        return make_rsrc(reinterpret_cast<const char *>(a) + base, bytes - base);
    };
    const size_t fbytes = fstride * S;
    const Rsrc rb = rs(b, fbase, fbytes);
    const Rsrc rE = rs(L.c, fbase, fbytes);
    const Rsrc rN = rs(L.c + fstride, fbase, fbytes);
    const Rsrc rU = rs(L.c + 2 * fstride, fbase, fbytes);
    const Rsrc ru = MODE == SWEEP_ZERO ? make_rsrc(u, 0) : rs(u, fbase, fbytes);
    const Rsrc re = MODE == SWEEP_PROLONG ? rs(ec, cbase, (size_t)nz * planec * S) : make_rsrc(ec, 0);
    auto ld = [&](const Rsrc &r, Off o, int k) -> T { return bload(T(), r, o.v, o.s + (unsigned)k * pstride); };
    auto ld1 = [&](const Rsrc &r, Off o, int k) -> T {
        return bload<CP>(T(), r, o.v, o.s + (unsigned)k * pstride);
    };
    auto le = [&](Off po, int k) -> T { return bload(T(), re, po.v, po.s + (unsigned)k * cstride); };
    auto U = [&](int k, Off o, Off po) -> T {
        T v = ld(ru, o, k);
        if (MODE == SWEEP_PROLONG) v += le(po, k);
        return v;
    };


    ChunkState<T, M> cs[CPW];
    T su[CPW][M];
    T u_dn[CPW], u_c[CPW], wD[CPW], e_c[CPW];
    int k0[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        k0[c] = (c * P + p) * M;
        u_dn[c] = u_c[c] = wD[c] = e_c[c] = T(0);
        if (k0[c] < nz) {
            if (k0[c] > 0) {
                wD[c] = L.wz[k0[c] - 1] * ld(rU, C, k0[c] - 1);
                if (MODE != SWEEP_ZERO) u_dn[c] = U(k0[c] - 1, C, PC);
            }
            if constexpr (XP) {
                e_c[c] = le(PC, k0[c]);
                u_c[c] = ld(ru, C, k0[c]) + e_c[c];
            } else if (MODE != SWEEP_ZERO) {
                u_c[c] = U(k0[c], C, PC);
            }
        }
        cs[c].init();
    }

    // The cells of a step are guarded by k < nz (a branch; loads are not moved
    // across it, so each step waits for its own loads).  FULL (every chunk
    // lies inside the column) drops the guards, and the scheduler issues the
    // next cells' loads early.  The host selects it for the FP32 sweep from
    // zero, whose 6 loads per cell left too few in flight (1024^2 x 128:
    // 0.476 vs 0.500 ms).  The sweeps that read u (10-13 loads per cell) and
    // the FP64 sweeps were slower unguarded (general 0.80 vs 0.63 ms,
    // prolongation 0.93 vs 0.78 ms, FP64 from zero 1.15 vs 1.03 ms): with
    // every cell's loads issued at once a CU holds far more data in flight
    // than its L1.
#pragma unroll
    for (int t = 0; t < M; ++t) {
        // loads of the CPW cells of this step (wave-uniform validity)
        SweepRaw<T> R[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int k = k0[c] + t;
            if (FULL || k < nz) {
                R[c].b = ld1(rb, C, k);
                R[c].cE = ld(rE, C, k);
                R[c].cEw = ld(rE, W, k);
                R[c].cN = ld(rN, C, k);
                R[c].cNs = ld(rN, Sx, k);
                R[c].cU = ld1(rU, C, k);
                R[c].uup = R[c].uE = R[c].uW = R[c].uN = R[c].uS = R[c].eup = T(0);
                // inside a full chunk only its last cell can be the top
                const bool up = (FULL && t + 1 < M) || k + 1 < nz;
                if constexpr (XP) {
                    if (up) {
                        R[c].eup = le(PC, k + 1);
                        R[c].uup = ld(ru, C, k + 1) + R[c].eup;
                    }
                    R[c].uE = U(k, X, PX);
                    const T eo = le(PO, k);
                    R[c].uN = ld(ru, N, k) + (jodd ? eo : e_c[c]);
                    R[c].uS = ld(ru, Sx, k) + (jodd ? e_c[c] : eo);
                } else if (MODE != SWEEP_ZERO) {
                    if (up) R[c].uup = U(k + 1, C, PC);
                    if constexpr (XL) {
                        R[c].uE = U(k, X, PX);
                    } else {
                        R[c].uE = U(k, E, PE);
                        R[c].uW = U(k, W, PW);
                    }
                    R[c].uN = U(k, N, PN);
                    R[c].uS = U(k, Sx, PS);
                }
            }
        }
        // arithmetic
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int k = k0[c] + t;
            if (FULL || k < nz) {
                const T h = L.wh[k];
                const T mu = L.mu[k];
                const T wE = h * R[c].cE;
                const T wW = h * R[c].cEw;
                const T wN = h * R[c].cN;
                const T wS = h * R[c].cNs;
                const T wU = L.wz[k] * R[c].cU;
                const T delta = mu + wE + wW + wN + wS;
                const T uc = u_c[c];
                T r = R[c].b;
                if (MODE != SWEEP_ZERO) {
                    T uE = R[c].uE, uW = R[c].uW;
                    if constexpr (XL) {
                        // R.uE holds the value across the tile edge (lanes 0, 63)
                        uW = lane_from_prev(R[c].uE, uc);
                        uE = lane_from_next(R[c].uE, uc);
                    }
                    const T Hu = mu * uc + wE * (uc - uE) + wW * (uc - uW) + wN * (uc - R[c].uN) +
                                 wS * (uc - R[c].uS) + wU * (uc - R[c].uup) + wD[c] * (uc - u_dn[c]);
                    r -= Hu;
                }
                cs[c].step(t, r, delta, wU, wD[c]);
                su[c][t] = uc;
                u_dn[c] = uc;
                u_c[c] = R[c].uup;
                if constexpr (XP) e_c[c] = R[c].eup;
                wD[c] = wU;
            } else {
                cs[c].identity(t);
                su[c][t] = T(0);
            }
        }
    }

#pragma unroll
    for (int c = 0; c < CPW; ++c) cs[c].backsub_publish(red + (size_t)(c * P + p) * 512, lane);
    __syncthreads();
    if (p == 0) coupling_solve(red, Q, lane);
    __syncthreads();
    const Rsrc ro = rs(out, fbase, fbytes);
    const unsigned oo = active ? C.v : 0xFFFFFFFFu;  // inactive lanes write nothing (C.s = 0 there)
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int q = c * P + p;
        const T xlo = (q > 0) ? red[(size_t)(q - 1) * 512 + 256 + lane] : T(0);
        const T xhi = (q + 1 < Q) ? red[(size_t)(q + 1) * 512 + 320 + lane] : T(0);
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const int k = k0[c] + t;
            if (k < nz)
                bstore<CP>(su[c][t] + omega * cs[c].value(t, xlo, xhi), ro, oo, C.s + (unsigned)k * pstride);
        }
    }
}

// ---------------------------------------------------------------------------
// y = H x on one level.  Thread = (column, chunk of KC cells along k).
// ---------------------------------------------------------------------------
template <typename T, int KC>
__global__ __launch_bounds__(kStreamThreads) void k_apply(Level<T> L, const T *__restrict__ x,
                                                          T *__restrict__ y)
{
    int col, k0;
    bool active;
    stream_coords<KC>(L, col, k0, active);
    const int nz = L.nz;
    const StencilRows<T> R(L, col);
    const size_t fbytes = (size_t)nz * L.plane * sizeof(T);
    const Rsrc rx = make_rsrc(x, fbytes), ry = make_rsrc(y, fbytes);
    const unsigned oo = active ? R.oc : 0xFFFFFFFFu;
    T xm = 0, wD = 0;
    if (k0 > 0) {
        const unsigned sm = (unsigned)(k0 - 1) * R.pstride;
        xm = bload(T(), rx, R.oc, sm);
        wD = L.wz[k0 - 1] * bload(T(), R.rU, R.oc, sm);
    }
    T xc = bload(T(), rx, R.oc, (unsigned)k0 * R.pstride);
#pragma unroll
    for (int t = 0; t < KC; ++t) {
        const int k = k0 + t;
        if (k < nz) {
            const unsigned sk = (unsigned)k * R.pstride;
            const T xp = (k + 1 < nz) ? bload(T(), rx, R.oc, sk + R.pstride) : T(0);
            const T h = L.wh[k];
            const T wU = L.wz[k] * bload(T(), R.rU, R.oc, sk);
            const T acc = L.mu[k] * xc + h * bload(T(), R.rE, R.oc, sk) * (xc - bload(T(), rx, R.oe, sk)) +
                          h * bload(T(), R.rE, R.ow, sk) * (xc - bload(T(), rx, R.ow, sk)) +
                          h * bload(T(), R.rN, R.oc, sk) * (xc - bload(T(), rx, R.on, sk)) +
                          h * bload(T(), R.rN, R.os, sk) * (xc - bload(T(), rx, R.os, sk)) + wU * (xc - xp) +
                          wD * (xc - xm);
            bstore(acc, ry, oo, sk);
            xm = xc;
            xc = xp;
            wD = wU;
        }
    }
}

// ---------------------------------------------------------------------------
// b_c = R (b - H u): residual on the fine level summed over the four children
// of each coarse cell (Sec. 3.2).  Couplings between the four children cancel
// in the sum, so only the eight outer horizontal faces and the vertical faces
// enter.  Thread = (coarse column, chunk of KC cells).
// ---------------------------------------------------------------------------
template <typename T, int KC>
__global__ __launch_bounds__(kStreamThreads) void k_resid_restrict(Level<T> L, const T *__restrict__ u,
                                                                   const T *__restrict__ b,
                                                                   T *__restrict__ bc)
{
    constexpr unsigned S = sizeof(T);
    const int n = L.n, nz = L.nz, plane = L.plane;
    const int nc = n >> 1, planec = nc * nc;
    const int ncb = (planec + kStreamThreads - 1) / kStreamThreads;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int kc = blk / ncb, cb = blk % ncb;
    int ccol = cb * kStreamThreads + threadIdx.x;
    const bool active = ccol < planec;
    if (!active) ccol = 0;
    const int k0 = kc * KC;
    const int I = ccol % nc, J = ccol / nc;
    const int i0 = 2 * I, j0 = 2 * J;
    const int iw = (i0 == 0) ? n - 1 : i0 - 1;
    const int ie = (i0 + 2 == n) ? 0 : i0 + 2;
    const int js = (j0 == 0) ? n - 1 : j0 - 1;
    const int jn = (j0 + 2 == n) ? 0 : j0 + 2;
    // the four children a=(i0,j0) b=(i0+1,j0) c=(i0,j0+1) d=(i0+1,j0+1), byte
    // offsets (i0 is even, so a and b, c and d share a 64-column tile)
    auto off = [&](int i, int j) { return cell_off(L, (unsigned)(j * n + i)); };
    const unsigned q0 = off(i0, j0), q1 = q0 + S, q2 = off(i0, j0 + 1), q3 = q2 + S;
    const unsigned qw0 = off(iw, j0), qw1 = off(iw, j0 + 1);    // west of a, c
    const unsigned qe0 = off(ie, j0), qe1 = off(ie, j0 + 1);    // east of b, d
    const unsigned qs0 = off(i0, js), qs1 = qs0 + S;            // south of a, b
    const unsigned qn0 = off(i0, jn), qn1 = qn0 + S;            // north of c, d
    const unsigned q[4] = {q0, q1, q2, q3};
    const size_t fbytes = (size_t)nz * plane * S;
    const Rsrc ru = make_rsrc(u, fbytes), rb = make_rsrc(b, fbytes);
    const Rsrc rE = make_rsrc(L.c, fbytes), rN = make_rsrc(L.c + (size_t)nz * plane, fbytes);
    const Rsrc rU = make_rsrc(L.c + 2 * (size_t)nz * plane, fbytes);
    const Rsrc rc = make_rsrc(bc, (size_t)nz * planec * S);
    const unsigned pstride = (unsigned)tile_width(plane) * S, cstride = (unsigned)tile_width(planec) * S;
    const unsigned oo = active ? (unsigned)cell_base(ccol, planec, nz) * S : 0xFFFFFFFFu;

    T um[4], uc[4], wD[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        um[a] = 0;
        wD[a] = 0;
        if (k0 > 0) {
            const unsigned sm = (unsigned)(k0 - 1) * pstride;
            um[a] = bload(T(), ru, q[a], sm);
            wD[a] = L.wz[k0 - 1] * bload(T(), rU, q[a], sm);
        }
        uc[a] = bload(T(), ru, q[a], (unsigned)k0 * pstride);
    }
#pragma unroll
    for (int t = 0; t < KC; ++t) {
        const int k = k0 + t;
        if (k < nz) {
            const unsigned sk = (unsigned)k * pstride;
            const T h = L.wh[k], mu = L.mu[k], wz = L.wz[k];
            T up[4], wU[4];
            T s = 0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                up[a] = (k + 1 < nz) ? bload(T(), ru, q[a], sk + pstride) : T(0);
                wU[a] = wz * bload(T(), rU, q[a], sk);
                s += bload(T(), rb, q[a], sk) - mu * uc[a] - wU[a] * (uc[a] - up[a]) - wD[a] * (uc[a] - um[a]);
            }
            s -= h * bload(T(), rE, qw0, sk) * (uc[0] - bload(T(), ru, qw0, sk));
            s -= h * bload(T(), rE, qw1, sk) * (uc[2] - bload(T(), ru, qw1, sk));
            s -= h * bload(T(), rE, q1, sk) * (uc[1] - bload(T(), ru, qe0, sk));
            s -= h * bload(T(), rE, q3, sk) * (uc[3] - bload(T(), ru, qe1, sk));
            s -= h * bload(T(), rN, qs0, sk) * (uc[0] - bload(T(), ru, qs0, sk));
            s -= h * bload(T(), rN, qs1, sk) * (uc[1] - bload(T(), ru, qs1, sk));
            s -= h * bload(T(), rN, q2, sk) * (uc[2] - bload(T(), ru, qn0, sk));
            s -= h * bload(T(), rN, q3, sk) * (uc[3] - bload(T(), ru, qn1, sk));
            bstore(s, rc, oo, (unsigned)k * cstride);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                um[a] = uc[a];
                uc[a] = up[a];
                wD[a] = wU[a];
            }
        }
    }
}

// The same restriction for levels whose rows are whole tiles (n a multiple
// of 64), with the access pattern of the sweep: a workgroup of two
// wavefronts owns fine rows 2J and 2J+1 of one 64-column tile and a chunk of
// KC levels; each lane streams its fine column, forming r = b - H u cell by
// cell (every load a contiguous segment), adds the horizontal child pair by
// a lane exchange, and wavefront 0 adds row 2J+1's pair sums from LDS and
// writes the 32 coarse values of the tile per level.  XL: the east / west
// values of u come from the neighbouring lanes (one load at the tile edges).
template <typename T, int KC, int CP, bool XL>
__global__ __launch_bounds__(128) void k_resid_restrict_rows(Level<T> L, const T *__restrict__ u,
                                                             const T *__restrict__ b, T *__restrict__ bc)
{
    constexpr unsigned S = sizeof(T);
    __shared__ T pair[KC][32];
    const int n = L.n, nz = L.nz, TR = n >> 6, nc = n >> 1, planec = nc * nc;
    const int nkc = (nz + KC - 1) / KC, npairs = nc * TR;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int kc = blk / npairs, pr = blk % npairs;
    const int J = pr / TR, t = pr % TR;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int j = 2 * J + w;
    const unsigned col = (unsigned)(j * n + t * 64 + lane);
    const int k0 = kc * KC;
    const StencilRows<T> R(L, col);
    const size_t fbytes = (size_t)nz * L.plane * S;
    const Rsrc ru = make_rsrc(u, fbytes), rb = make_rsrc(b, fbytes);
    T rs[KC];
    T um = 0, wD = 0;
    if (k0 > 0) {
        const unsigned sm = (unsigned)(k0 - 1) * R.pstride;
        um = bload(T(), ru, R.oc, sm);
        wD = L.wz[k0 - 1] * bload(T(), R.rU, R.oc, sm);
    }
    T uc = bload(T(), ru, R.oc, (unsigned)k0 * R.pstride);
    const unsigned ox = lane == 0 ? R.ow : (lane == 63 ? R.oe : R.oc);
#pragma unroll
    for (int q = 0; q < KC; ++q) {
        const int k = k0 + q;
        rs[q] = T(0);
        if (k < nz) {
            const unsigned sk = (unsigned)k * R.pstride;
            const T up = (k + 1 < nz) ? bload(T(), ru, R.oc, sk + R.pstride) : T(0);
            const T h = L.wh[k];
            const T wU = L.wz[k] * bload<CP>(T(), R.rU, R.oc, sk);
            T uE, uW;
            if constexpr (XL) {
                const T ux = bload(T(), ru, ox, sk);
                uE = lane_from_next(ux, uc);
                uW = lane_from_prev(ux, uc);
            } else {
                uE = bload(T(), ru, R.oe, sk);
                uW = bload(T(), ru, R.ow, sk);
            }
            const T hu = L.mu[k] * uc + h * bload(T(), R.rE, R.oc, sk) * (uc - uE) +
                         h * bload(T(), R.rE, R.ow, sk) * (uc - uW) +
                         h * bload(T(), R.rN, R.oc, sk) * (uc - bload(T(), ru, R.on, sk)) +
                         h * bload(T(), R.rN, R.os, sk) * (uc - bload(T(), ru, R.os, sk)) + wU * (uc - up) +
                         wD * (uc - um);
            const T r = bload<CP>(T(), rb, R.oc, sk) - hu;
            rs[q] = r + __shfl_xor(r, 1, 64);  // children (2I, j) + (2I+1, j)
            um = uc;
            uc = up;
            wD = wU;
        }
    }
    if (w == 1 && !(lane & 1)) {
#pragma unroll
        for (int q = 0; q < KC; ++q) pair[q][lane >> 1] = rs[q];
    }
    __syncthreads();
    if (w == 0 && !(lane & 1)) {
        const unsigned ccol = (unsigned)(J * nc + t * 32 + (lane >> 1));
        const unsigned oo = (unsigned)cell_base(ccol, planec, nz) * S;
        const unsigned cstride = (unsigned)tile_width(planec) * S;
        const Rsrc rc = make_rsrc(bc, (size_t)nz * planec * S);
#pragma unroll
        for (int q = 0; q < KC; ++q) {
            const int k = k0 + q;
            if (k < nz) bstore<CP>(rs[q] + pair[q][lane >> 1], rc, oo, (unsigned)k * cstride);
        }
    }
}

// Coarsest level, dense mode: x = A^{-1} b with A^{-1} symmetric (row t read
// as column t, so a wavefront reads consecutive addresses).
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_gemv(const T *__restrict__ ainv, int m,
                                                     const T *__restrict__ b, T *__restrict__ x)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= m) return;
    T acc = 0;
#pragma unroll 8
    for (int j = 0; j < m; ++j) acc += ainv[(size_t)j * m + t] * b[j];
    x[t] = acc;
}

// ---- setup kernels ---------------------------------------------------------

// Level l+1 faces from level l: mean of the fine faces covering each coarse
// face.  Thread = one coarse cell, in storage order.
__global__ __launch_bounds__(256) void k_coarsen(Level<double> F, double *__restrict__ cc,
                                                 float *__restrict__ cc32)
{
    const int n = F.n, nz = F.nz, nc = n >> 1, planec = nc * nc;
    const unsigned total = (unsigned)planec * nz;
    const unsigned w = storage_wave(), g = w * 64u + (threadIdx.x & 63u);
    if (g >= total) return;
    unsigned ccol;
    int k;
    storage_coords(g, w, planec, nz, ccol, k);
    const int I = (int)(ccol % nc), J = (int)(ccol / nc);
    const size_t fs = (size_t)nz * F.plane, cs = (size_t)nz * planec;
    const double *cE = F.c, *cN = F.c + fs, *cU = F.c + 2 * fs;
    auto at = [&](int i, int j) { return cell_index((size_t)j * n + i, k, F.plane, nz); };
    const int i = 2 * I, j = 2 * J;  // child (2I, 2J)
    const double e = 0.5 * (cE[at(i + 1, j)] + cE[at(i + 1, j + 1)]);
    const double nn = 0.5 * (cN[at(i, j + 1)] + cN[at(i + 1, j + 1)]);
    const double u = 0.25 * (cU[at(i, j)] + cU[at(i + 1, j)] + cU[at(i, j + 1)] + cU[at(i + 1, j + 1)]);
    cc[g] = e;
    cc[cs + g] = nn;
    cc[2 * cs + g] = u;
    if (cc32) {
        cc32[g] = (float)e;
        cc32[cs + g] = (float)nn;
        cc32[2 * cs + g] = (float)u;
    }
}

__global__ __launch_bounds__(256) void k_cast(const double *__restrict__ s, float *__restrict__ d,
                                              size_t n)
{
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256)
        d[g] = (float)s[g];
}

// Input faces (either layout) -> tiled level-0 storage with the top U slot
// zeroed, an FP32 copy when dst32 is given, and the count of real faces whose
// value is not positive and finite added to *bad.  Thread = destination value.
__global__ __launch_bounds__(256) void k_copy_coeffs(const double *__restrict__ src, int layout,
                                                     double *__restrict__ dst, float *__restrict__ dst32,
                                                     int plane, int nz, int *__restrict__ bad)
{
    const unsigned per = (unsigned)plane * nz;
    const int f = blockIdx.y;
    const unsigned w = storage_wave(), g = w * 64u + (threadIdx.x & 63u);
    if (g >= per) return;
    // level-major source: thread = source element (sequential reads);
    // column-major source: thread = destination element
    unsigned col;
    int k;
    size_t o = g;
    double v;
    if (layout == 0) {
        v = src[(size_t)f * per + g];
        if ((plane & 63) == 0) {
            const unsigned cpb = (unsigned)plane >> 6, kk = w / cpb, tile = w - kk * cpb;
            k = (int)kk;
            o = ((size_t)tile * nz + kk) * 64 + (g & 63u);
        } else {
            k = (int)(g / (unsigned)plane);
        }
    } else {
        storage_coords(g, w, plane, nz, col, k);
        v = src[((size_t)col * nz + k) * 3 + f];
    }
    if (f == 2 && k == nz - 1)
        v = 0.0;
    else if (!(v > 0.0) || !(v <= kDblMax))
        atomicAdd(bad, 1);
    o += (size_t)f * per;
    dst[o] = v;
    if (dst32) dst32[o] = (float)v;
}

__global__ __launch_bounds__(256) void k_fill(double *__restrict__ x, double v, size_t n)
{
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256) x[g] = v;
}


// Transposes of consecutive R x C row-major matrices (element type E)
// through LDS, 32 x 32 blocks; the grid covers every block of every matrix.
template <typename E>
__global__ __launch_bounds__(256) void k_transpose(const E *__restrict__ src, E *__restrict__ dst,
                                                   int R, int C)
{
    __shared__ E tile[32][33];
    const int tiles_c = (C + 31) / 32, tiles = tiles_c * ((R + 31) / 32);
    const unsigned batch = blockIdx.x / tiles, t = blockIdx.x % tiles;
    src += (size_t)batch * R * C;
    dst += (size_t)batch * R * C;
    const int bx = (int)(t % tiles_c) * 32, by = (int)(t / tiles_c) * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int yy = ty; yy < 32; yy += 8) {
        const int r = by + yy, c = bx + tx;
        if (r < R && c < C) tile[yy][tx] = src[(size_t)r * C + c];
    }
    __syncthreads();
    for (int yy = ty; yy < 32; yy += 8) {
        const int c = bx + yy, r = by + tx;
        if (r < R && c < C) dst[(size_t)c * R + r] = tile[tx][yy];
    }
}

// Level-major faces [3][nz][plane] -> column-major [plane][nz][3].
__global__ __launch_bounds__(256) void k_faces_to_column(const double *__restrict__ src,
                                                         double *__restrict__ dst, int plane, int nz)
{
    const size_t per = (size_t)plane * nz;
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < 3 * per; g += (size_t)gridDim.x * 256) {
        const int f = (int)(g / per);
        const size_t r = g % per;
        const int k = (int)(r / plane), col = (int)(r % plane);
        dst[((size_t)col * nz + k) * 3 + f] = src[g];
    }
}

// Level-major [nz][plane] <-> tiled storage.  64 aligned columns of one level
// are contiguous in both orders, so both sides are coalesced; the threads
// follow the order of the source (sequential reads, 512-byte scattered
// writes: 374 vs 530 us for 1 GiB on MI355X the other way round).
template <typename E>
__global__ __launch_bounds__(256) void k_level_to_tiled(const E *__restrict__ src, E *__restrict__ dst,
                                                        E *__restrict__ dst2, int plane, int nz)
{
    const unsigned w = storage_wave(), g = w * 64u + (threadIdx.x & 63u);
    if (g >= (unsigned)plane * nz) return;
    const E v = src[g];
    size_t o = g;  // plane not a multiple of 64: both orders agree
    if ((plane & 63) == 0) {
        const unsigned cpb = (unsigned)plane >> 6, k = w / cpb, tile = w - k * cpb;
        o = ((size_t)tile * nz + k) * 64 + (g & 63u);
    }
    dst[o] = v;
    if (dst2) dst2[o] = v;
}

template <typename E>
__global__ __launch_bounds__(256) void k_tiled_to_level(const E *__restrict__ src, E *__restrict__ dst, int plane,
                                                        int nz)
{
    const unsigned w = storage_wave(), g = w * 64u + (threadIdx.x & 63u);
    if (g >= (unsigned)plane * nz) return;
    unsigned col;
    int k;
    storage_coords(g, w, plane, nz, col, k);
    dst[(size_t)k * plane + col] = src[g];
}

// Start of a solve from x = 0 with the caller's level-major b: r = b in
// tiled storage (and fl32(r) when r32 is given), b and x = 0 there when they
// are given, and partial sums of (b, b).  Threads follow the source order,
// four or more elements each.
__global__ __launch_bounds__(256) void k_solve_start(const double *__restrict__ bsrc, double *__restrict__ b,
                                                     double *__restrict__ r, float *__restrict__ r32,
                                                     double *__restrict__ x, int plane, int nz,
                                                     double *__restrict__ partials)
{
    const size_t total = (size_t)plane * nz;
    const unsigned cpb = (unsigned)plane >> 6;
    double acc = 0.0;
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (size_t)gridDim.x * 256) {
        const double v = bsrc[g];
        size_t o = g;  // plane not a multiple of 64: both orders agree
        if ((plane & 63) == 0) {
            const unsigned w = (unsigned)__builtin_amdgcn_readfirstlane((unsigned)(g >> 6));
            const unsigned k = w / cpb, tile = w - k * cpb;
            o = ((size_t)tile * nz + k) * 64 + (g & 63);
        }
        if (b) b[o] = v;
        r[o] = v;
        if (r32) r32[o] = (float)v;
        if (x) x[o] = 0.0;
        acc += v * v;
    }
    double vv[1] = {acc};
    block_partials<1>(vv, partials, gridDim.x, blockIdx.x);
}

// ---- CG kernels (FP64) -----------------------------------------------------

// p_new = z + beta p_old (p_new = z on the first iteration), q = H p_new, and
// partial sums of (p_new, q).  Neighbour values of p_new are formed on the fly from z and p_old, so p_old
// and p_new must be different buffers.  z is FP32 (mixed) or FP64 (ZT).
//
// The kernel is bound by memory latency (its wavefronts walk their k-chunk
// level by level), so each wavefront issues level k + 1's loads before it
// forms level k, and holds z in its stored type until it is used: two
// levels in flight at 80 VGPRs (6 wavefronts per SIMD) instead of one at
// 54 (8 per SIMD); 1.45 vs 1.74 ms at 1024^2 x 128 with FP32 z.
// CP: cache policy of c_U and of the p, q stores (read or written once).
// XL (rows of whole tiles): p_new at the east / west neighbours comes from
// the neighbouring lanes, formed there by the same expression (one pair of
// loads at the tile edges instead of two pairs per cell).
// RW = 4 (with XL): the workgroup's four wavefronts take the same tile in
// four consecutive rows; p_new and c_N of a level go through LDS, so the
// inner rows take their north / south p_new and the south face from the
// neighbouring wavefront instead of loading z, p_old and c_N there (only the
// outer rows of the four load them).  1024^2 x 128: 1.343 vs 1.383 ms (8 rows
// per workgroup: 1.368 ms).  The (p, q) partial sums then group other
// columns per workgroup.
template <int KC, typename ZT, int CP, bool XL, int RW = 0>
__global__ __launch_bounds__(kStreamThreads) void k_pcg_apply(Level<double> L, const ZT *__restrict__ zt,
                                                              const double *__restrict__ p_old,
                                                              double *__restrict__ p_new,
                                                              double *__restrict__ q,
                                                              const Scalars *__restrict__ sc, int first,
                                                              double *__restrict__ partials)
{
    int col, k0;
    bool active;
    constexpr bool R4 = RW != 0;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if constexpr (R4) {
        // blocks: (k-chunk, group of RW rows, tile column), row groups outer
        const int TR = L.n >> 6, per_kc = (L.n / RW) * TR;
        const int blk = xcd_remap(blockIdx.x, gridDim.x);
        const int kc = blk / per_kc, r = blk % per_kc;
        col = (RW * (r / TR) + wv) * L.n + (r % TR) * 64 + (int)(threadIdx.x & 63);
        k0 = kc * KC;
        active = true;
    } else {
        stream_coords<KC>(L, col, k0, active);
    }
    const int nz = L.nz;
    const StencilRows<double> R(L, col);
    const size_t n = (size_t)nz * L.plane;
    constexpr unsigned ZS = sizeof(ZT);
    const Rsrc rz = make_rsrc(zt, n * ZS);
    const Rsrc rp = make_rsrc(p_old, first ? 0 : n * 8);
    const Rsrc rpn = make_rsrc(p_new, n * 8), rq = make_rsrc(q, n * 8);
    const unsigned zs = (unsigned)tile_width(L.plane) * ZS;
    const double beta = first ? 0.0 : sc->beta;
    // lane offsets are in bytes of a double; z offsets scale by ZS / 8
    auto zo = [](unsigned o) { return ZS == 8 ? o : o >> 1; };
    auto ZL = [&](int k, unsigned o) -> ZT { return bload(ZT(), rz, zo(o), (unsigned)k * zs); };
    auto PL = [&](int k, unsigned o) -> double {
        return first ? 0.0 : bload(double(), rp, o, (unsigned)k * R.pstride);
    };
    // Explicit fused multiply-adds in a fixed order: every form of the kernel
    // (lane exchange or loads) then rounds identically, whatever the
    // compiler would contract.
    auto comb = [&](ZT zz, double pp) -> double { return first ? (double)zz : __builtin_fma(beta, pp, (double)zz); };
    struct Raw {
        ZT zE, zW, zN, zS, zu;
        double pE, pW, pN, pS, pu, cE, cEw, cN, cNs, cU;
    };
    const int lane = threadIdx.x & 63;
    const unsigned ox = lane == 0 ? R.ow : (lane == 63 ? R.oe : R.oc);
    auto load = [&](int k) {
        Raw w;
        const unsigned sk = (unsigned)k * R.pstride;
        if constexpr (XL) {
            // the value across the tile edge (lanes 0 and 63)
            w.zE = ZL(k, ox);
            w.pE = PL(k, ox);
            w.zW = ZT(0);
            w.pW = 0.0;
        } else {
            w.zE = ZL(k, R.oe);
            w.zW = ZL(k, R.ow);
            w.pE = PL(k, R.oe);
            w.pW = PL(k, R.ow);
        }
        w.zN = ZT(0);
        w.zS = ZT(0);
        w.pN = 0.0;
        w.pS = 0.0;
        w.cNs = 0.0;
        if (!R4 || wv == RW - 1) {
            w.zN = ZL(k, R.on);
            w.pN = PL(k, R.on);
        }
        if (!R4 || wv == 0) {
            w.zS = ZL(k, R.os);
            w.pS = PL(k, R.os);
            w.cNs = bload(double(), R.rN, R.os, sk);
        }
        w.cE = bload(double(), R.rE, R.oc, sk);
        w.cEw = bload(double(), R.rE, R.ow, sk);
        w.cN = bload(double(), R.rN, R.oc, sk);
        w.cU = bload<CP>(double(), R.rU, R.oc, sk);
        w.zu = ZT(0);
        w.pu = 0.0;
        if (k + 1 < nz) {
            w.zu = ZL(k + 1, R.oc);
            w.pu = PL(k + 1, R.oc);
        }
        return w;
    };
    const unsigned oo = active ? R.oc : 0xFFFFFFFFu;
    double pm = 0, wD = 0;
    if (k0 > 0) {
        pm = comb(ZL(k0 - 1, R.oc), PL(k0 - 1, R.oc));
        wD = L.wz[k0 - 1] * bload(double(), R.rU, R.oc, (unsigned)(k0 - 1) * R.pstride);
    }
    double pc = comb(ZL(k0, R.oc), PL(k0, R.oc));
    double acc_pq = 0;
    Raw cur = load(k0);
#pragma unroll
    for (int t = 0; t < KC; ++t) {
        const int k = k0 + t;
        if (k < nz) {
            Raw nxt = cur;
            if (t + 1 < KC && k + 1 < nz) nxt = load(k + 1);
            const unsigned sk = (unsigned)k * R.pstride;
            const double pp = comb(cur.zu, cur.pu);
            const double h = L.wh[k];
            const double wU = L.wz[k] * cur.cU;
            double pE, pW;
            if constexpr (XL) {
                const double px = comb(cur.zE, cur.pE);
                pE = lane_from_next(px, pc);
                pW = lane_from_prev(px, pc);
            } else {
                pE = comb(cur.zE, cur.pE);
                pW = comb(cur.zW, cur.pW);
            }
            double pN, pS, cNs;
            if constexpr (R4) {
                // double-buffered by level: slot t & 1 serves level k and is
                // written again (for level k + 2) only after the barrier of
                // level k + 1, which every wavefront reaches only after
                // reading the slot for level k
                __shared__ double xp[2][R4 ? RW : 1][64], xc[2][R4 ? RW : 1][64];
                const int sl = t & 1;
                xp[sl][wv][lane] = pc;
                xc[sl][wv][lane] = cur.cN;
                __syncthreads();
                pN = wv == RW - 1 ? comb(cur.zN, cur.pN) : xp[sl][wv + 1][lane];
                pS = wv == 0 ? comb(cur.zS, cur.pS) : xp[sl][wv - 1][lane];
                cNs = wv == 0 ? cur.cNs : xc[sl][wv - 1][lane];
            } else {
                pN = comb(cur.zN, cur.pN);
                pS = comb(cur.zS, cur.pS);
                cNs = cur.cNs;
            }
            double qq = L.mu[k] * pc;
            qq = __builtin_fma(h * cur.cE, pc - pE, qq);
            qq = __builtin_fma(h * cur.cEw, pc - pW, qq);
            qq = __builtin_fma(h * cur.cN, pc - pN, qq);
            qq = __builtin_fma(h * cNs, pc - pS, qq);
            qq = __builtin_fma(wU, pc - pp, qq);
            qq = __builtin_fma(wD, pc - pm, qq);
            bstore<CP>(pc, rpn, oo, sk);
            bstore<CP>(qq, rq, oo, sk);
            if (active) acc_pq += pc * qq;
            pm = pc;
            pc = pp;
            wD = wU;
            cur = nxt;
        }
    }
    double v[1] = {acc_pq};
    block_partials<1>(v, partials, gridDim.x, blockIdx.x);
}

// r = b - H x (r may be null: the norm only), and partial sums of (r, r).
// b is in the level's storage, or level-major when b_level is set.  With
// xout, x is also written there in level-major order (the end of a solve:
// the copy of the iterate to the caller rides on this pass).
// The stencil sum is formed by explicit fused multiply-adds in a fixed order,
// so both forms round alike.  XL (rows of whole tiles): east / west x from
// the neighbouring lanes, as in k_pcg_apply (1024^2 x 128: 1.427 vs 1.444 ms;
// passing the north / south rows through LDS on four-row workgroups, as
// k_pcg_apply does, gained nothing more here: without a lookahead this
// kernel waits on each level's loads, not on their number).
template <int KC, bool XL = false>
__global__ __launch_bounds__(kStreamThreads) void k_residual(Level<double> L, const double *__restrict__ x,
                                                             const double *__restrict__ b, int b_level,
                                                             double *__restrict__ r,
                                                             double *__restrict__ xout,
                                                             double *__restrict__ partials)
{
    int col, k0;
    bool active;
    stream_coords<KC>(L, col, k0, active);
    const int nz = L.nz, lane = threadIdx.x & 63;
    const StencilRows<double> R(L, col);
    const size_t fbytes = (size_t)nz * L.plane * 8;
    const Rsrc rx = make_rsrc(x, fbytes), rb = make_rsrc(b, fbytes), rr = make_rsrc(r, r ? fbytes : 0);
    const Rsrc rxo = make_rsrc(xout, xout ? fbytes : 0);
    const unsigned oo = active ? R.oc : 0xFFFFFFFFu, ol = active ? (unsigned)col * 8u : 0xFFFFFFFFu;
    const unsigned lstride = (unsigned)L.plane * 8u;
    // the value across the tile edge (lanes 0 and 63) for the lane exchange
    const unsigned ox = lane == 0 ? R.ow : (lane == 63 ? R.oe : R.oc);
    double xm = 0, wD = 0;
    if (k0 > 0) {
        const unsigned sm = (unsigned)(k0 - 1) * R.pstride;
        xm = bload(double(), rx, R.oc, sm);
        wD = L.wz[k0 - 1] * bload(double(), R.rU, R.oc, sm);
    }
    double xc = bload(double(), rx, R.oc, (unsigned)k0 * R.pstride);
    double acc = 0;
#pragma unroll
    for (int t = 0; t < KC; ++t) {
        const int k = k0 + t;
        if (k < nz) {
            const unsigned sk = (unsigned)k * R.pstride;
            const double xp = (k + 1 < nz) ? bload(double(), rx, R.oc, sk + R.pstride) : 0.0;
            const double h = L.wh[k];
            const double wU = L.wz[k] * bload(double(), R.rU, R.oc, sk);
            const double cE = bload(double(), R.rE, R.oc, sk), cEw = bload(double(), R.rE, R.ow, sk);
            const double cN = bload(double(), R.rN, R.oc, sk);
            double xE, xW;
            if constexpr (XL) {
                const double xx = bload(double(), rx, ox, sk);
                xE = lane_from_next(xx, xc);
                xW = lane_from_prev(xx, xc);
            } else {
                xE = bload(double(), rx, R.oe, sk);
                xW = bload(double(), rx, R.ow, sk);
            }
            const double xN = bload(double(), rx, R.on, sk), xS = bload(double(), rx, R.os, sk);
            const double cNs = bload(double(), R.rN, R.os, sk);
            double hx = L.mu[k] * xc;
            hx = __builtin_fma(h * cE, xc - xE, hx);
            hx = __builtin_fma(h * cEw, xc - xW, hx);
            hx = __builtin_fma(h * cN, xc - xN, hx);
            hx = __builtin_fma(h * cNs, xc - xS, hx);
            hx = __builtin_fma(wU, xc - xp, hx);
            hx = __builtin_fma(wD, xc - xm, hx);
            const double bv = b_level ? bload(double(), rb, ol, (unsigned)k * lstride) : bload(double(), rb, R.oc, sk);
            const double rv = bv - hx;
            if (r) bstore(rv, rr, oo, sk);
            if (xout) bstore(xc, rxo, ol, (unsigned)k * lstride);
            if (active) acc += rv * rv;
            xm = xc;
            xc = xp;
            wD = wU;
        }
    }
    double v[1] = {acc};
    block_partials<1>(v, partials, gridDim.x, blockIdx.x);
}

// x += alpha p; r -= alpha q; partial sums of (r, r); optionally
// r32 = fl32(r) for the FP32 V-cycle.
__global__ __launch_bounds__(kCgThreads) void k_pcg_update(size_t n, double *__restrict__ x,
                                                    const double *__restrict__ p, double *__restrict__ r,
                                                    const double *__restrict__ q, float *__restrict__ r32,
                                                    const Scalars *__restrict__ sc,
                                                    double *__restrict__ partials, int x_first)
{
    const double alpha = sc->alpha;
    double rr = 0;
    for (size_t g = (size_t)blockIdx.x * kCgThreads + threadIdx.x; g < n; g += (size_t)gridDim.x * kCgThreads) {
        if (x_first)
            x[g] = alpha * p[g];  // first step from x = 0: x is not read
        else
            x[g] += alpha * p[g];
        const double rv = r[g] - alpha * q[g];
        r[g] = rv;
        rr += rv * rv;
        if (r32) r32[g] = (float)rv;
    }
    double v[1] = {rr};
    block_partials<1>(v, partials, gridDim.x, blockIdx.x);
}

// Partial sums of (a, b) and, when c is given, of (c, b); b is FP64 or, when
// b32 is given, FP32.
__global__ __launch_bounds__(kCgThreads) void k_dot(size_t n, const double *__restrict__ a,
                                                    const double *__restrict__ b, const float *__restrict__ b32,
                                                    const double *__restrict__ c, double *__restrict__ partials)
{
    double s = 0, t = 0;
    for (size_t g = (size_t)blockIdx.x * kCgThreads + threadIdx.x; g < n; g += (size_t)gridDim.x * kCgThreads) {
        const double bv = b32 ? (double)b32[g] : b[g];
        s += a[g] * bv;
        if (c) t += c[g] * bv;
    }
    if (c) {
        double v[2] = {s, t};
        block_partials<2>(v, partials, gridDim.x, blockIdx.x);
    } else {
        double v[1] = {s};
        block_partials<1>(v, partials, gridDim.x, blockIdx.x);
    }
}

// Fixed-order sum of the partials and the scalar recurrences of CG.
__global__ __launch_bounds__(1024) void k_finalize(const double *__restrict__ partials, int G, int nvals,
                                                   Scalars *__restrict__ sc, int stage, int flexible)
{
    __shared__ double sh[2][1024];
    for (int v = 0; v < nvals; ++v) {
        // four independent accumulators (fixed order for a given G)
        const double *pv = partials + (size_t)v * G;
        double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        int i = threadIdx.x;
        for (; i + 3 * 1024 < G; i += 4 * 1024) {
            s0 += pv[i];
            s1 += pv[i + 1024];
            s2 += pv[i + 2048];
            s3 += pv[i + 3072];
        }
        for (; i < G; i += 1024) s0 += pv[i];
        sh[v][threadIdx.x] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int v = 0; v < nvals; ++v) sh[v][threadIdx.x] += sh[v][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double s0 = sh[0][0], s1 = (nvals > 1) ? sh[1][0] : 0.0;
    switch (stage) {
    case ST_BB: sc->bb = s0; break;
    case ST_RR: sc->rr = s0; break;
    case ST_RZ_FIRST:
        sc->rz = s0;
        sc->beta = 0.0;
        if (!(fabs(s0) <= kDblMax)) sc->breakdown = 1;
        break;
    case ST_RZ: {
        // s0 = (r, z_new); flexible (FCG(1)): s1 = (q, z_new) with q = H p of
        // the last iteration, beta = -(z_new, H p) / (p, H p), which makes the
        // new direction H-conjugate to the last one
        sc->beta = flexible ? -s1 / sc->pq : s0 / sc->rz;
        sc->rz = s0;
        if (!(fabs(sc->beta) <= kDblMax)) sc->breakdown = 1;
        break;
    }
    case ST_PQ: {
        sc->pq = s0;
        const double a = sc->rz / s0;
        if (!(s0 > 0.0) || !(fabs(a) <= kDblMax)) {
            sc->breakdown = 1;
            sc->alpha = 0.0;
        } else {
            sc->alpha = a;
        }
        break;
    }
    case ST_TT: sc->tt = s0; break;
    default: break;
    }
}

// dJ/dc_f = -gamma_f (lambda_p - lambda_q)(x_p - x_q) on level-0 faces.
// NT: the gradient (written once, never read back here) with non-temporal
// stores.  (Unrolling a full chunk without guards was slower, 1.29 vs
// 1.22 ms at 1024^2 x 128; the east value by lane exchange gained 0.5 %.)
template <int KC, bool NT>
__global__ __launch_bounds__(kStreamThreads) void k_face_gradient(Level<double> L,
                                                                  const double *__restrict__ lam,
                                                                  const double *__restrict__ x,
                                                                  double *__restrict__ g)
{
    int col, k0;
    bool active;
    stream_coords<KC>(L, col, k0, active);
    const int nz = L.nz, plane = L.plane;
    const Nbr nb = neighbours(col, L.n, plane);
    const size_t fstride = (size_t)nz * plane;
    double lc = (k0 < nz) ? lam[(size_t)k0 * plane + col] : 0.0;
    double xc = (k0 < nz) ? x[(size_t)k0 * plane + col] : 0.0;
    for (int t = 0; t < KC; ++t) {
        const int k = k0 + t;
        if (k >= nz) break;
        const size_t o = (size_t)k * plane;
        const double h = L.wh[k];
        const double lu = (k + 1 < nz) ? lam[o + plane + col] : 0.0;
        const double xu = (k + 1 < nz) ? x[o + plane + col] : 0.0;
        const double gE = -h * (lc - lam[o + nb.e]) * (xc - x[o + nb.e]);
        const double gN = -h * (lc - lam[o + nb.n]) * (xc - x[o + nb.n]);
        const double gU = (k + 1 < nz) ? -L.wz[k] * (lc - lu) * (xc - xu) : 0.0;
        if (active) {
            if constexpr (NT) {
                __builtin_nontemporal_store(gE, g + o + col);
                __builtin_nontemporal_store(gN, g + fstride + o + col);
                __builtin_nontemporal_store(gU, g + 2 * fstride + o + col);
            } else {
                g[o + col] = gE;
                g[fstride + o + col] = gN;
                g[2 * fstride + o + col] = gU;
            }
        }
        lc = lu;
        xc = xu;
    }
}

// The same gradient with two columns per thread and 16-byte accesses (rows
// of whole 128-column segments, 16-byte aligned arrays): thread = (column
// pair, chunk of KC levels); the east value of the pair's second column comes
// from the next lane (one load at the segment edge).  1024^2 x 128: 1.115 vs
// 1.22 ms for one column per thread.
typedef double dbl2 __attribute__((ext_vector_type(2)));
template <int KC>
__global__ __launch_bounds__(kStreamThreads) void k_face_gradient2(Level<double> L,
                                                                   const double *__restrict__ lam,
                                                                   const double *__restrict__ x,
                                                                   double *__restrict__ g)
{
    const int nz = L.nz, plane = L.plane, n = L.n;
    const int npairs = plane >> 1, ncb = npairs / kStreamThreads;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int kc = blk / ncb, cb = blk % ncb;
    const int pr = cb * kStreamThreads + threadIdx.x;
    const int col = 2 * pr, k0 = kc * KC;
    const int i = col % n, j = col / n;
    const int ce = (i + 2 == n) ? col + 2 - n : col + 2;           // east of the second column
    const int cn = (j + 1 == n) ? col + n - plane : col + n;       // north of both
    const int lane = threadIdx.x & 63;
    const int cx = lane == 63 ? ce : col;
    const size_t fstride = (size_t)nz * plane;
    auto ld2 = [](const double *a, size_t o) { return *reinterpret_cast<const dbl2 *>(a + o); };
    dbl2 lc = ld2(lam, (size_t)k0 * plane + col), xc = ld2(x, (size_t)k0 * plane + col);
    for (int t = 0; t < KC; ++t) {
        const int k = k0 + t;
        if (k >= nz) break;
        const size_t o = (size_t)k * plane;
        const double h = L.wh[k];
        const bool up = k + 1 < nz;
        const dbl2 lu = up ? ld2(lam, o + plane + col) : dbl2{0.0, 0.0};
        const dbl2 xu = up ? ld2(x, o + plane + col) : dbl2{0.0, 0.0};
        const dbl2 ln = ld2(lam, o + cn), xn = ld2(x, o + cn);
        const double le = lane_from_next(lam[o + cx], lc.x), xe = lane_from_next(x[o + cx], xc.x);
        dbl2 gE, gN, gU;
        gE.x = -h * (lc.x - lc.y) * (xc.x - xc.y);
        gE.y = -h * (lc.y - le) * (xc.y - xe);
        gN.x = -h * (lc.x - ln.x) * (xc.x - xn.x);
        gN.y = -h * (lc.y - ln.y) * (xc.y - xn.y);
        const double wz = L.wz[k];
        gU.x = up ? -wz * (lc.x - lu.x) * (xc.x - xu.x) : 0.0;
        gU.y = up ? -wz * (lc.y - lu.y) * (xc.y - xu.y) : 0.0;
        __builtin_nontemporal_store(gE, reinterpret_cast<dbl2 *>(g + o + col));
        __builtin_nontemporal_store(gN, reinterpret_cast<dbl2 *>(g + fstride + o + col));
        __builtin_nontemporal_store(gU, reinterpret_cast<dbl2 *>(g + 2 * fstride + o + col));
        lc = lu;
        xc = xu;
    }
}

// Streaming copy with 16-byte accesses: the bandwidth reference point.
// One 16-byte element per thread, non-temporal: the fastest plain copy
// measured on MI355X (more elements per thread lowered the rate).
typedef unsigned v4u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_probe_copy(const v4u *__restrict__ s, v4u *__restrict__ d, size_t n)
{
    for (size_t g = (size_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (size_t)gridDim.x * 256)
        __builtin_nontemporal_store(__builtin_nontemporal_load(s + g), d + g);
}



// Levels of at least 2^24 cells (an FP32 vector of 64 MiB; the six arrays a
// sweep streams exceed the 256 MB last-level cache) use non-temporal hints
// for the data they read or write once.
template <typename T>
bool nt_level(const Level<T> &L)
{
    return (size_t)L.plane * L.nz >= ((size_t)1 << 24);
}

// Small FP32 levels fill few CUs and are bound by the latency of each
// thread's chain of cells along k (1024^2 x 128, V-cycle 4.24 vs 4.27 ms
// with both):
//  - below 2^24 cells (levels 2-6) the restriction walks 4-level chunks
//    instead of 16 (TPMG_SHORT_RESTRICT_CELLS overrides the bound);
//  - below 2^22 cells (levels 3-6) every sweep walks its full chunks
//    unguarded (TPMG_LAT_CELLS overrides the bound).
template <typename T>
bool small_level(const Level<T> &L, int env_cells, int log2_cells)
{
    const double bound = env_cells >= 0 ? (double)env_cells : (double)((size_t)1 << log2_cells);
    return sizeof(T) == 4 && (double)L.plane * L.nz < bound;
}
template <typename T>
bool lat_level(const Level<T> &L)
{
    static const int e = env_int("TPMG_LAT_CELLS");
    return small_level(L, e, 22);
}
template <typename T>
bool short_restrict_level(const Level<T> &L)
{
    static const int e = env_int("TPMG_SHORT_RESTRICT_CELLS");
    return small_level(L, e, 24);
}

// k-chunk of a streaming kernel: `dflt` unless TPMG_KCHUNK overrides it.
// Measured on 1024^2 x 128: longer chunks help the FP64 CG stencils (64
// cells: 1.68 vs 1.77 ms) and the finest restriction (32: 0.685 vs 0.70 ms);
// the other kernels and smaller planes (fewer workgroups) prefer 16.
int stream_kc(int dflt = 16)
{
    static const int e = env_int("TPMG_KCHUNK");
    return (e == 4 || e == 8 || e == 16 || e == 32 || e == 64) ? e : dflt;
}

template <typename T>
int stream_grid(const Level<T> &L, int kc)
{
    const int ncb = (L.plane + kStreamThreads - 1) / kStreamThreads;
    const int nkc = (L.nz + kc - 1) / kc;
    return ncb * nkc;
}

// Calls f(std::integral_constant<int, KC>) for the k-chunk length kc.
template <class F>
hipError_t with_kc(int kc, F f)
{
    switch (kc) {
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return f(std::integral_constant<int, 8>());
    case 32: return f(std::integral_constant<int, 32>());
    case 64: return f(std::integral_constant<int, 64>());
    default: return f(std::integral_constant<int, 16>());
    }
}

template <typename T, int M, int CPW, int LB>
hipError_t sweep_m(const Level<T> &L, int mode, const T *u, const T *b, T *out, const T *ec, T omega, int P,
                   hipStream_t s)
{
    // Tile order: plain row order in both precisions (measured on 1024^2 x
    // 128 with the non-temporal hints and the lane exchange: FP64 V-cycle
    // 9.58 vs 9.96 ms for blocks of 2 tiles x 32 rows, 9.87 ms for 4 x 16;
    // FP32 V-cycle 4.24 vs 4.27-4.59 ms for 1 x 4 to 4 x 2 and 2 x 16).
    // TPMG_SWEEP_BI / TPMG_SWEEP_BJ select blocks of BI tiles x BJ rows.
    static const int ebi = env_int("TPMG_SWEEP_BI"), ebj = env_int("TPMG_SWEEP_BJ");
    const int tbi = ebi >= 0 ? ebi : 0;
    const int tbj = ebj > 0 ? ebj : 1;
    const int tiles = (L.plane + 63) / 64;
    const dim3 block(64 * P);
    const size_t lds = (size_t)P * CPW * 512 * sizeof(T);
    // Row-uniform neighbour offsets where the rows are whole tiles on this
    // level (and, for the prolongation sweep, on the coarser one).  Measured
    // on 1024^2 x 128 they help the FP32 prolongation sweep (0.80 vs 0.86 ms:
    // 8 instead of 16 bytes of spill) and cost about 1 % elsewhere, so by
    // default only that sweep uses them (TPMG_SWEEP_ROWS=1: every sweep that
    // can, 0: none).
    static const int erows = env_int("TPMG_SWEEP_ROWS"), exl = env_int("TPMG_SWEEP_XL");
    const bool fits = L.n % 64 == 0 && (mode != SWEEP_PROLONG || L.n % 128 == 0);
    const bool rows = fits && (erows == 1 || (erows < 0 && sizeof(T) == 4 && mode == SWEEP_PROLONG));
    // East / west values of u by lane exchange wherever the rows are whole
    // tiles (TPMG_SWEEP_XL=0: loads as elsewhere).  Measured at 1024^2 x 128:
    // FP32 V-cycle 4.32 vs 4.36-4.39 ms; the FP32 prolongation sweep then
    // fits its 64-VGPR bound without spill.
    const bool xl = fits && mode != SWEEP_ZERO && exl != 0;
    const int rm = xl ? 2 : (rows ? 1 : 0);
    // Non-temporal accesses for b, c_U and the output on levels too large
    // for the caches (TPMG_SWEEP_NT=0: plain everywhere, 1: everywhere):
    // measured at 1024^2 x 128, FP32 V-cycle 4.36 vs 4.51 ms; on levels whose
    // data stays in the last-level cache the next kernel's reads of b are
    // hits that the hints would give away.
    static const int ent = env_int("TPMG_SWEEP_NT");
    const bool nt = ent == 1 || (ent != 0 && nt_level(L));
    // Unguarded chunks (every chunk inside the column) for the FP32 sweep from
    // zero and for every FP32 sweep on a latency-bound level.
    const bool chunks_full = L.full_chunks && L.nz % (M * CPW) == 0;
    auto go = [&](auto mc, auto rc) {
        constexpr int MC = decltype(mc)::value, RC = decltype(rc)::value;
        auto launch = [&](auto cp, auto fl) {
            hipLaunchKernelGGL((k_sweep<T, M, CPW, MC, LB, RC, decltype(cp)::value, decltype(fl)::value>),
                               dim3(tiles), block, lds, s, L, u, b, out, ec, omega, tbi, tbj);
        };
        using CNT = std::integral_constant<int, kNT>;
        using C0 = std::integral_constant<int, 0>;
        if constexpr (MC == SWEEP_ZERO && sizeof(T) == 4) {
            if (chunks_full) return nt ? launch(CNT(), std::true_type()) : launch(C0(), std::true_type());
        } else if constexpr (sizeof(T) == 4) {
            if (chunks_full && lat_level(L)) return launch(C0(), std::true_type());
        }
        nt ? launch(CNT(), std::false_type()) : launch(C0(), std::false_type());
    };
    using R0 = std::integral_constant<int, 0>;
    using R1 = std::integral_constant<int, 1>;
    using R2 = std::integral_constant<int, 2>;
    auto by_rm = [&](auto mc) {
        if (rm == 2) go(mc, R2());
        else if (rm == 1) go(mc, R1());
        else go(mc, R0());
    };
    switch (mode) {
    case SWEEP_ZERO:
        rm ? go(std::integral_constant<int, SWEEP_ZERO>(), R1()) : go(std::integral_constant<int, SWEEP_ZERO>(), R0());
        break;
    case SWEEP_GENERAL: by_rm(std::integral_constant<int, SWEEP_GENERAL>()); break;
    default: by_rm(std::integral_constant<int, SWEEP_PROLONG>()); break;
    }
    return hipGetLastError();
}

// Launch bound = the smaller of 512/1024 threads that holds the P wavefronts,
// so each shape gets the largest register budget it can.
template <typename T, int M, int CPW>
hipError_t sweep_lb(const Level<T> &L, int mode, const T *u, const T *b, T *out, const T *ec, T omega, int P,
                    hipStream_t s)
{
    if (P <= 8) return sweep_m<T, M, CPW, 512>(L, mode, u, b, out, ec, omega, P, s);
    return sweep_m<T, M, CPW, 1024>(L, mode, u, b, out, ec, omega, P, s);
}

}  // namespace

// Chunking of a column for the sweep: M cells per chunk, CPW chunks per
// wavefront, P wavefronts (P <= 16).  Default (measured on 1024^2 x 128 in
// both precisions): one chunk of 16 cells per wavefront.
bool sweep_shape(int nz, bool fp32, int mode, int *M, int *CPW, int *P)
{
    static const int fm = env_int("TPMG_SWEEP_M"), fc = env_int("TPMG_SWEEP_CPW");
    int c = (fc == 1 || fc == 2) ? fc : 1;
    // Chunk length measured on 1024^2 x 128 (tiled storage): 8 cells (16
    // wavefronts) for every FP32 sweep (general 0.66 vs 0.70 ms; the
    // prolongation sweep, held to 64 VGPRs so that two workgroups share a CU,
    // 0.86 vs 0.95 ms) and the FP64 prolongation sweep (2.19 vs 2.22 ms); 16
    // cells (8 wavefronts) for the other FP64 sweeps (general 1.57 vs 1.70 ms).
    const bool eight = fp32 || mode == SWEEP_PROLONG;
    int m = (fm == 4 || fm == 8 || fm == 16) ? fm : ((eight && (nz + 7) / 8 <= 16) ? 8 : 16);
    if (m == 16) c = 1;  // (16, 2) is not instantiated: too many registers
    // short columns: the smallest chunk that still covers them
    while (m > 4 && (m / 2) * c >= nz) m /= 2;
    const int p = (nz + m * c - 1) / (m * c);
    if (p > 16) return false;
    *M = m;
    *CPW = c;
    *P = p;
    return true;
}

template <typename T>
hipError_t launch_sweep(const Level<T> &L, int mode, const T *u, const T *b, T *out, const T *ec, T omega,
                        hipStream_t s)
{
    int M = 0, CPW = 0, P = 0;
    if (!sweep_shape(L.nz, sizeof(T) == 4, mode, &M, &CPW, &P)) return hipErrorInvalidValue;
    if (CPW == 2) {
        switch (M) {
        case 4: return sweep_lb<T, 4, 2>(L, mode, u, b, out, ec, omega, P, s);
        default: return sweep_lb<T, 8, 2>(L, mode, u, b, out, ec, omega, P, s);
        }
    }
    switch (M) {
    case 4: return sweep_lb<T, 4, 1>(L, mode, u, b, out, ec, omega, P, s);
    case 8: return sweep_lb<T, 8, 1>(L, mode, u, b, out, ec, omega, P, s);
    default: return sweep_lb<T, 16, 1>(L, mode, u, b, out, ec, omega, P, s);
    }
}

template <typename T>
hipError_t launch_apply(const Level<T> &L, const T *x, T *y, hipStream_t s)
{
    const int kc = stream_kc();
    return with_kc(kc, [&](auto KCc) {
        hipLaunchKernelGGL((k_apply<T, decltype(KCc)::value>), dim3(stream_grid(L, kc)), dim3(kStreamThreads), 0, s,
                           L, x, y);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_resid_restrict(const Level<T> &L, const T *u, const T *b, T *bc, hipStream_t s)
{
    // Rows of whole tiles, FP32: the row-tile kernel (1024^2 x 128: 0.58 vs
    // 0.69 ms).  In FP64 it was slower (1.29 vs 1.21 ms) and is not used
    // (TPMG_RESTRICT_ROWS64=1 selects it).
    static const int er64 = env_int("TPMG_RESTRICT_ROWS64");
    if ((L.n & 63) == 0 && (sizeof(T) == 4 || er64 == 1)) {
        const bool short_chunks = short_restrict_level(L);
        const int kc = short_chunks ? 4 : 16, nkc = (L.nz + kc - 1) / kc;
        const int grid = nkc * (L.n / 2) * (L.n / 64);
        // non-temporal b, c_U and output, as in the sweep (TPMG_RESTRICT_NT=0:
        // plain); east / west values of u by lane exchange (TPMG_RESTRICT_XL=0: loads)
        static const int ent = env_int("TPMG_RESTRICT_NT"), exl = env_int("TPMG_RESTRICT_XL");
        const bool nt = ent == 1 || (ent != 0 && nt_level(L)), xl = exl != 0;
        auto go = [&](auto kcc, auto cp, auto x) {
            hipLaunchKernelGGL((k_resid_restrict_rows<T, decltype(kcc)::value, decltype(cp)::value,
                                                      decltype(x)::value>),
                               dim3(grid), dim3(128), 0, s, L, u, b, bc);
        };
        using K16 = std::integral_constant<int, 16>;
        using NT = std::integral_constant<int, kNT>;
        using PL = std::integral_constant<int, 0>;
        using Y = std::true_type;
        using F = std::false_type;
        if (nt) {
            xl ? go(K16(), NT(), Y()) : go(K16(), NT(), F());
        } else if (short_chunks) {
            go(std::integral_constant<int, 4>(), PL(), Y());
        } else {
            xl ? go(K16(), PL(), Y()) : go(K16(), PL(), F());
        }
        return hipGetLastError();
    }
    const int planec = (L.n / 2) * (L.n / 2);
    const int ncb = (planec + kStreamThreads - 1) / kStreamThreads;
    const int kc = short_restrict_level(L) ? 4 : stream_kc(planec >= 512 * 512 && L.nz >= 32 ? 32 : 16);
    const int nkc = (L.nz + kc - 1) / kc;
    return with_kc(kc, [&](auto KCc) {
        hipLaunchKernelGGL((k_resid_restrict<T, decltype(KCc)::value>), dim3(ncb * nkc), dim3(kStreamThreads), 0, s,
                           L, u, b, bc);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_coarse_gemv(const T *ainv, int m, const T *b, T *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_coarse_gemv<T>, dim3((m + 255) / 256), dim3(256), 0, s, ainv, m, b, x);
    return hipGetLastError();
}

template hipError_t launch_sweep<double>(const Level<double> &, int, const double *, const double *,
                                         double *, const double *, double, hipStream_t);
template hipError_t launch_sweep<float>(const Level<float> &, int, const float *, const float *, float *,
                                        const float *, float, hipStream_t);
template hipError_t launch_apply<double>(const Level<double> &, const double *, double *, hipStream_t);
template hipError_t launch_apply<float>(const Level<float> &, const float *, float *, hipStream_t);
template hipError_t launch_resid_restrict<double>(const Level<double> &, const double *, const double *,
                                                  double *, hipStream_t);
template hipError_t launch_resid_restrict<float>(const Level<float> &, const float *, const float *,
                                                 float *, hipStream_t);
template hipError_t launch_coarse_gemv<double>(const double *, int, const double *, double *, hipStream_t);
template hipError_t launch_coarse_gemv<float>(const float *, int, const float *, float *, hipStream_t);

hipError_t launch_coarsen(const Level<double> &F, double *c_coarse, float *c_coarse32, hipStream_t s)
{
    const size_t total = (size_t)(F.n / 2) * (F.n / 2) * F.nz;
    hipLaunchKernelGGL(k_coarsen, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, F, c_coarse, c_coarse32);
    return hipGetLastError();
}

hipError_t launch_cast(const double *src, float *dst, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_copy_coeffs(const double *src, int layout, double *dst, float *dst32, int plane, int nz, int *bad,
                              hipStream_t s)
{
    const unsigned blocks = (unsigned)(((size_t)plane * nz + 255) / 256);
    hipLaunchKernelGGL(k_copy_coeffs, dim3(blocks, 3), dim3(256), 0, s, src, layout, dst, dst32, plane, nz, bad);
    return hipGetLastError();
}

hipError_t launch_fill(double *x, double v, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, x, v, n);
    return hipGetLastError();
}


static hipError_t transpose_elem(const void *src, void *dst, int R, int C, int elem, hipStream_t s, int batches = 1)
{
    const dim3 grid((unsigned)(((C + 31) / 32) * (size_t)((R + 31) / 32) * batches));
    if (elem == 8)
        hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, s, (const double *)src, (double *)dst, R, C);
    else
        hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, s, (const float *)src, (float *)dst, R, C);
    return hipGetLastError();
}

// Column-major [plane][nz] <-> tiled: each 64-column tile is a 64 x nz
// transpose; a plane that is not a multiple of 64 is one plane x nz transpose.
static hipError_t tile_transposes(const void *src, void *dst, int plane, int nz, int elem, bool to_tiled,
                                  hipStream_t s)
{
    const int W = tile_width(plane), nt = plane / W;
    return to_tiled ? transpose_elem(src, dst, W, nz, elem, s, nt) : transpose_elem(src, dst, nz, W, elem, s, nt);
}

hipError_t launch_cells_in(const void *src, int layout, void *dst, void *dst2, int plane, int nz, int elem,
                           hipStream_t s)
{
    if (layout == 1) {
        hipError_t e = tile_transposes(src, dst, plane, nz, elem, true, s);
        if (e == hipSuccess && dst2) e = hipMemcpyAsync(dst2, dst, (size_t)plane * nz * elem, hipMemcpyDeviceToDevice, s);
        return e;
    }
    const unsigned blocks = (unsigned)(((size_t)plane * nz + 255) / 256);
    if (elem == 8)
        hipLaunchKernelGGL(k_level_to_tiled<double>, dim3(blocks), dim3(256), 0, s, (const double *)src, (double *)dst,
                           (double *)dst2, plane, nz);
    else
        hipLaunchKernelGGL(k_level_to_tiled<float>, dim3(blocks), dim3(256), 0, s, (const float *)src, (float *)dst,
                           (float *)dst2, plane, nz);
    return hipGetLastError();
}

hipError_t launch_cells_out(const void *src, void *dst, int layout, int plane, int nz, int elem, hipStream_t s)
{
    if (layout == 1) return tile_transposes(src, dst, plane, nz, elem, false, s);
    const unsigned blocks = (unsigned)(((size_t)plane * nz + 255) / 256);
    if (elem == 8)
        hipLaunchKernelGGL(k_tiled_to_level<double>, dim3(blocks), dim3(256), 0, s, (const double *)src, (double *)dst,
                           plane, nz);
    else
        hipLaunchKernelGGL(k_tiled_to_level<float>, dim3(blocks), dim3(256), 0, s, (const float *)src, (float *)dst,
                           plane, nz);
    return hipGetLastError();
}

hipError_t launch_solve_start(const double *bsrc, double *b, double *r, float *r32, double *x, int plane, int nz,
                              double *partials, int *nblocks_out, hipStream_t s)
{
    const int G = grid_for((size_t)plane * nz);
    *nblocks_out = G;
    hipLaunchKernelGGL(k_solve_start, dim3(G), dim3(256), 0, s, bsrc, b, r, r32, x, plane, nz, partials);
    return hipGetLastError();
}

hipError_t launch_cells_to_level(const void *src, void *dst, int plane, int nz, int elem, hipStream_t s)
{
    return transpose_elem(src, dst, plane, nz, elem, s);  // [plane][nz] -> [nz][plane]
}


hipError_t launch_faces_to_column(const double *src, double *dst, int plane, int nz, hipStream_t s)
{
    hipLaunchKernelGGL(k_faces_to_column, dim3(grid_for(3 * (size_t)plane * nz)), dim3(256), 0, s, src, dst,
                       plane, nz);
    return hipGetLastError();
}

hipError_t launch_pcg_apply(const Level<double> &L, const double *z, const float *z32, const double *p_old,
                            double *p_new, double *q, const Scalars *sc, int first, double *partials,
                            int *nblocks_out, hipStream_t s)
{
    // 16-level chunks (1024^2 x 128, FP32 z: 1.45 ms vs 1.47 at 32; at 64 the
    // two levels in flight need 92 VGPRs)
    const int kc = stream_kc(16);
    const int G = stream_grid(L, kc);
    *nblocks_out = G;
    // Non-temporal c_U and p, q stores on levels larger than the caches
    // (TPMG_CG_NT=0: never, 1: always): 1.39 vs 1.45 ms at 1024^2 x 128.
    // East / west neighbours by lane exchange where the rows are whole tiles
    // (16-level chunks only; TPMG_CG_XL=0: loads).
    static const int ent = env_int("TPMG_CG_NT"), exl = env_int("TPMG_CG_XL"), er4 = env_int("TPMG_CG_ROWS4");
    const bool nt = ent == 1 || (ent != 0 && nt_level(L));
    const bool xl = exl != 0 && (L.n & 63) == 0;
    // four rows per workgroup with the lane exchange (TPMG_CG_ROWS4=0: one
    // row); the same grid, n being a multiple of 64
    const int rw = (xl && er4 != 0) ? 4 : 0;
    return with_kc(kc, [&](auto KCc) {
        constexpr int K = decltype(KCc)::value;
        auto go = [&](auto cp, auto x, auto rr) {
            constexpr int CP = decltype(cp)::value, RR = decltype(rr)::value;
            constexpr bool XL = decltype(x)::value;
            if (z32)
                hipLaunchKernelGGL((k_pcg_apply<K, float, CP, XL, RR>), dim3(G), dim3(kStreamThreads), 0, s, L,
                                   z32, p_old, p_new, q, sc, first, partials);
            else
                hipLaunchKernelGGL((k_pcg_apply<K, double, CP, XL, RR>), dim3(G), dim3(kStreamThreads), 0, s, L,
                                   z, p_old, p_new, q, sc, first, partials);
        };
        using R0 = std::integral_constant<int, 0>;
        auto by_xl = [&](auto cp) {
            if constexpr (K == 16) {
                if (rw == 4) return go(cp, std::true_type(), std::integral_constant<int, 4>());
                if (xl) return go(cp, std::true_type(), R0());
            }
            go(cp, std::false_type(), R0());
        };
        if (nt) by_xl(std::integral_constant<int, kNT>());
        else by_xl(std::integral_constant<int, 0>());
        return hipGetLastError();
    });
}

hipError_t launch_residual(const Level<double> &L, const double *x, const double *b, int b_level, double *r,
                           double *xout, double *partials, int *nblocks_out, hipStream_t s)
{
    const int kc = stream_kc(L.nz >= 64 && L.plane >= 256 * 256 ? 64 : 16);
    const int G = stream_grid(L, kc);
    *nblocks_out = G;
    // lane exchange where the rows are whole tiles (TPMG_CG_XL=0: loads)
    static const int exl = env_int("TPMG_CG_XL");
    const bool xl = exl != 0 && (L.n & 63) == 0;
    return with_kc(kc, [&](auto KCc) {
        constexpr int K = decltype(KCc)::value;
        auto go = [&](auto xlc) {
            hipLaunchKernelGGL((k_residual<K, decltype(xlc)::value>), dim3(G), dim3(kStreamThreads), 0, s, L, x, b,
                               b_level, r, xout, partials);
        };
        bool done = false;
        if constexpr (K == 16 || K == 64) {
            if (xl) go(std::true_type()), done = true;
        }
        if (!done) go(std::false_type());
        return hipGetLastError();
    });
}

// Elements per thread of the elementwise CG kernels (TPMG_EPT overrides).
// Measured on 1024^2 x 128: the x/r update streams fastest at one (1.23 vs
// 1.38 ms at four), the dot, with less work per element, at four (0.28 vs
// 0.41 ms at one).
int cg_ept(int dflt)
{
    static const int e = env_int("TPMG_EPT");
    return (e == 1 || e == 2 || e == 4 || e == 8) ? e : dflt;
}

hipError_t launch_pcg_update(size_t n, double *x, const double *p, double *r, const double *q, float *r32,
                             const Scalars *sc, double *partials, int x_first, int *nblocks_out, hipStream_t s)
{
    const int G = grid_for(n, cg_ept(1), kCgThreads);
    *nblocks_out = G;
    hipLaunchKernelGGL(k_pcg_update, dim3(G), dim3(kCgThreads), 0, s, n, x, p, r, q, r32, sc, partials, x_first);
    return hipGetLastError();
}

hipError_t launch_dot(size_t n, const double *a, const double *b, const float *b32, double *partials,
                      int *nblocks_out, hipStream_t s, const double *c)
{
    const int G = grid_for(n, cg_ept(4), kCgThreads);
    *nblocks_out = G;
    hipLaunchKernelGGL(k_dot, dim3(G), dim3(kCgThreads), 0, s, n, a, b, b32, c, partials);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nblocks, int nvals, Scalars *sc, int stage, int flexible,
                           double *stage_buf, hipStream_t s)
{
    if (nblocks > 8 * kReduceSegs) {
        hipLaunchKernelGGL(k_reduce_partials, dim3(kReduceSegs, nvals), dim3(256), 0, s, partials, nblocks,
                           stage_buf);
        partials = stage_buf;
        nblocks = kReduceSegs;
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s, partials, nblocks, nvals, sc, stage, flexible);
    return hipGetLastError();
}

hipError_t launch_face_gradient(const Level<double> &L, const double *lam, const double *x, double *g,
                                hipStream_t s)
{
    // Measured at 1024^2 x 128 (one column per thread): non-temporal stores
    // and 64-cell chunks 1.218 ms, plain stores 1.266 ms (64) / 1.328 ms (16
    // cells); TPMG_FG_NT=0 restores plain stores.  Planes below 512^2 keep
    // 16-cell chunks (more workgroups).  Two columns per thread where the
    // rows and the arrays allow it (TPMG_FG_WIDE=0: one).
    const int kc = stream_kc(L.plane >= (1 << 18) ? 64 : 16);
    static const int nt = env_int("TPMG_FG_NT"), ew = env_int("TPMG_FG_WIDE");
    const bool aligned = ((uintptr_t)lam | (uintptr_t)x | (uintptr_t)g) % 16 == 0;
    if (ew != 0 && nt != 0 && aligned && L.n % 128 == 0 && (L.plane / 2) % kStreamThreads == 0) {
        const int nkc = (L.nz + kc - 1) / kc;
        const int grid = nkc * (L.plane / 2 / kStreamThreads);
        return with_kc(kc, [&](auto KCc) {
            hipLaunchKernelGGL((k_face_gradient2<decltype(KCc)::value>), dim3(grid), dim3(kStreamThreads), 0, s, L,
                               lam, x, g);
            return hipGetLastError();
        });
    }
    return with_kc(kc, [&](auto KCc) {
        if (nt != 0)
            hipLaunchKernelGGL((k_face_gradient<decltype(KCc)::value, true>), dim3(stream_grid(L, kc)),
                               dim3(kStreamThreads), 0, s, L, lam, x, g);
        else
            hipLaunchKernelGGL((k_face_gradient<decltype(KCc)::value, false>), dim3(stream_grid(L, kc)),
                               dim3(kStreamThreads), 0, s, L, lam, x, g);
        return hipGetLastError();
    });
}

hipError_t launch_probe_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    size_t g = (n + 255) / 256;
    if (g > (1u << 30)) g = 1u << 30;
    hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)g), dim3(256), 0, s, (const v4u *)src, (v4u *)dst, n);
    return hipGetLastError();
}

}  // namespace tpmg
