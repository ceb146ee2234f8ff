// HIP kernels for gfx950 (MI355X): the next-to-lowest-order pressure level
// of Mitchell & Mueller (Tab. FiniteElements: DG_1 pressure, six unknowns per
// cell), its vertical line smoother by a banded LU that is factorised once and
// applied per sweep (Sec. 4.3.1: dgbtrf at setup, dgbtrs per application),
// and the p-transfers to the lowest-order DG0 level by the natural embedding
// (Sec. 4.2.1).
//
// Operator (the reading this library implements; it is stated in full in
// tpmg.h).  Basis of a cell: u = sum_{v,h} u_{3v+h} l_v(zeta) psi_h(xi, eta)
// with psi = (1, xi, eta) and l_0, l_1 the bottom / top values of a linear
// function in the vertical.  H1 is the broken form of -div(K grad p) + p with
// K = diag(a_h c, a_h c, a_z c) (cell coefficients: means of the cell's face
// coefficients) plus a penalty of the jumps across every face with the
// lowest-order face weights w_f.  Written out for cell P with neighbours
// E, W, N, S (horizontal) and the cells below / above:
//   cell term   y_{3v+h} += alpha_h (P_v/3 + P_o/6) + beta_h (P_v - P_o)/4
//               (P_v = u_{3v+h}, P_o = u_{3(1-v)+h}; alpha_0 = s_k,
//               alpha_1 = s_k/3 + 4 a_h s_k c^x, alpha_2 = s_k/3 + 4 a_h s_k c^y,
//               beta_h = 4 a_z c^z / s_k * (1, 1/3, 1/3)_h);
//   east face   jump modes per vertical value w: J0 = (P_0 + P_1) - (E_0 - E_1),
//               J1 = P_2 - E_2 (subscripts h of level w), face mass
//               (1/3, 1/6 ; 1/6, 1/3) in v and 1, 1/3 for the two modes;
//               the cell on the face's low side receives +T^T F, the high
//               side -T^T F (T: the traces, signs of xi = +-1);
//   north face  the same with eta for xi (modes (P_0 + P_2) - (N_0 - N_2) and
//               P_1 - N_1);
//   upper face  J_h = P_{3+h} - U_h with weight w_f (1, 1/3, 1/3)_h.
// The column block H1_z (cell terms, self parts of the four horizontal faces,
// both vertical faces) is banded with 5 sub- and 5 super-diagonals in the row
// order r = 6k + a.
//
// Layout.  DG1 vectors use the tiled storage of the lowest-order levels with
// 6 nz rows per column, row p = a nz + k (so the caller's level-major
// (6, nz, n, n) arrays convert with the same kernels).  Band factors of a
// 64-column tile are stored [row r][entry e][lane]: one entry of one row of
// a tile is a 512-byte segment, read by one wavefront load.  Entry e of row
// r is L(r, r - 5 + e) for e < 5, 1 / U(r, r) for e = 5 and U(r, r + e - 5)
// for e > 5 (the reciprocal saves a division per row and sweep).
//
// Every kernel gives one lane one column and streams k; the band solve is a
// forward pass (residual, forward substitution, y stored in the output
// vector) and a backward pass (back substitution from y, the update).
#include "tpmg_device.h"

namespace tpmg {

namespace {

constexpr int kNb = 6;                    // unknowns per cell
constexpr int kNf = 11;                   // band entries per factor row (5 + 1 + 5)
constexpr double kMh[3] = {1.0, 1.0 / 3.0, 1.0 / 3.0};
constexpr double kThird = 1.0 / 3.0, kSixth = 1.0 / 6.0;

// Addresses of one lane (= one column) in the DG1 vectors, the face arrays
// and the band factors.
struct Dg1Lane {
    bool active;
    unsigned ov;                 // byte offset of row 0 of this column in a DG1 vector
    unsigned oe, ow, on, os;     // the same for the four horizontal neighbours
    unsigned oc, ocw, ocs;       // byte offset of level 0 in a face array: own, west, south column
    unsigned row;                // bytes between storage rows (W values)
    unsigned of;                 // byte offset of this lane within a factor row
    unsigned frow;               // bytes between factor rows (W factor values)
    Rsrc rE, rN, rU, rF;         // faces E, N, U; this tile's band factors
};

// cb: the workgroup's block of 256 consecutive columns; FT: the type the
// band factors are stored in.
template <typename FT = double>
__device__ __forceinline__ Dg1Lane dg1_lane(const Dg1Level &G, const FT *fac, int cb)
{
    Dg1Lane q;
    const int plane = G.plane, nz = G.nz, W = tile_width(plane);
    int col = cb * 256 + (int)threadIdx.x;
    q.active = col < plane;
    if (!q.active) col = 0;
    const Nbr nb = neighbours(col, G.n, plane);
    const int rows = kNb * nz;
    q.ov = (unsigned)(cell_base(col, plane, rows) * 8);
    q.oe = (unsigned)(cell_base(nb.e, plane, rows) * 8);
    q.ow = (unsigned)(cell_base(nb.w, plane, rows) * 8);
    q.on = (unsigned)(cell_base(nb.n, plane, rows) * 8);
    q.os = (unsigned)(cell_base(nb.s, plane, rows) * 8);
    q.oc = (unsigned)(cell_base(col, plane, nz) * 8);
    q.ocw = (unsigned)(cell_base(nb.w, plane, nz) * 8);
    q.ocs = (unsigned)(cell_base(nb.s, plane, nz) * 8);
    q.row = (unsigned)W * 8u;
    // a wavefront is one tile (W = 64) or lies in the single tile (W = plane)
    const unsigned tile = __builtin_amdgcn_readfirstlane((unsigned)(col / W));
    q.of = (unsigned)(col - (int)tile * W) * (unsigned)sizeof(FT);
    q.frow = (unsigned)W * (unsigned)sizeof(FT);
    const size_t fstride = (size_t)nz * plane;
    q.rE = make_rsrc(G.c, fstride * 8);
    q.rN = make_rsrc(G.c + fstride, fstride * 8);
    q.rU = make_rsrc(G.c + 2 * fstride, fstride * 8);
    const size_t tile_vals = (size_t)rows * kNf * W;
    q.rF = fac ? make_rsrc(fac + tile * tile_vals, tile_vals * sizeof(FT)) : make_rsrc(G.c, 0);
    return q;
}

// Coefficients of cell k of a column: face weights and the cell term's scalars.
struct Dg1Coef {
    double wE, wW, wN, wS, wT, wB;
    double al[3], be[3];
};

// Face coefficients the cell term and the face weights of cell k need
// (cU below is the previous cell's, carried by the caller).
struct Dg1Faces {
    double cE, cW, cN, cS, cU;
};

__device__ __forceinline__ Dg1Faces dg1_faces(const Dg1Lane &q, unsigned k)
{
    const unsigned sk = k * q.row;
    Dg1Faces f;
    f.cE = bload(double(), q.rE, q.oc, sk);
    f.cW = bload(double(), q.rE, q.ocw, sk);
    f.cN = bload(double(), q.rN, q.oc, sk);
    f.cS = bload(double(), q.rN, q.ocs, sk);
    f.cU = bload(double(), q.rU, q.oc, sk);  // 0 in the top cell's slot
    return f;
}

__device__ __forceinline__ Dg1Coef dg1_coef(const Dg1Level &G, int k, const Dg1Faces &f, double cUm)
{
    const int nz = G.nz;
    const double mu = G.tab[k], wh = G.tab[nz + k], wh4 = G.tab[2 * nz + k], kz4 = G.tab[3 * nz + k];
    const double wz = G.tab[4 * nz + k];
    Dg1Coef c;
    c.wE = wh * f.cE;
    c.wW = wh * f.cW;
    c.wN = wh * f.cN;
    c.wS = wh * f.cS;
    c.wT = wz * f.cU;  // wz = 0 at the top
    c.wB = (k > 0) ? G.tab[4 * nz + k - 1] * cUm : 0.0;
    const double cx = 0.5 * (f.cE + f.cW), cy = 0.5 * (f.cN + f.cS);
    const double cz = (k == 0) ? f.cU : ((k == nz - 1) ? cUm : 0.5 * (f.cU + cUm));
    c.al[0] = mu;
    c.al[1] = mu * kThird + wh4 * cx;
    c.al[2] = mu * kThird + wh4 * cy;
#pragma unroll
    for (int h = 0; h < 3; ++h) c.be[h] = kz4 * cz * kMh[h];
    return c;
}

// y = (H1 x) on the six rows of one cell: P the cell, E W N S its horizontal
// neighbours, Dn the top values of the cell below and Up the bottom values of
// the cell above (zero where there is no such cell: their weights are 0).
__device__ __forceinline__ void dg1_cell_apply(const double (&P)[6], const double (&E)[6], const double (&Wc)[6],
                                               const double (&N)[6], const double (&S)[6], const double (&Dn)[3],
                                               const double (&Up)[3], const Dg1Coef &c, double (&y)[6])
{
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int h = 0; h < 3; ++h) {
            const double pv = P[3 * v + h], po = P[3 * (1 - v) + h];
            y[3 * v + h] = c.al[h] * (pv * kThird + po * kSixth) + c.be[h] * 0.25 * (pv - po);
        }
    double J0[2], J1[2];
    // east face: this cell on its low side
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        J0[w] = (P[3 * w] + P[3 * w + 1]) - (E[3 * w] - E[3 * w + 1]);
        J1[w] = P[3 * w + 2] - E[3 * w + 2];
    }
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const double F0 = c.wE * (J0[v] * kThird + J0[1 - v] * kSixth);
        const double F1 = c.wE * (J1[v] * kThird + J1[1 - v] * kSixth) * kThird;
        y[3 * v] += F0;
        y[3 * v + 1] += F0;
        y[3 * v + 2] += F1;
    }
    // west face: this cell on its high side
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        J0[w] = (Wc[3 * w] + Wc[3 * w + 1]) - (P[3 * w] - P[3 * w + 1]);
        J1[w] = Wc[3 * w + 2] - P[3 * w + 2];
    }
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const double F0 = c.wW * (J0[v] * kThird + J0[1 - v] * kSixth);
        const double F1 = c.wW * (J1[v] * kThird + J1[1 - v] * kSixth) * kThird;
        y[3 * v] -= F0;
        y[3 * v + 1] += F0;
        y[3 * v + 2] -= F1;
    }
    // north face
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        J0[w] = (P[3 * w] + P[3 * w + 2]) - (N[3 * w] - N[3 * w + 2]);
        J1[w] = P[3 * w + 1] - N[3 * w + 1];
    }
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const double F0 = c.wN * (J0[v] * kThird + J0[1 - v] * kSixth);
        const double F1 = c.wN * (J1[v] * kThird + J1[1 - v] * kSixth) * kThird;
        y[3 * v] += F0;
        y[3 * v + 2] += F0;
        y[3 * v + 1] += F1;
    }
    // south face
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        J0[w] = (S[3 * w] + S[3 * w + 2]) - (P[3 * w] - P[3 * w + 2]);
        J1[w] = S[3 * w + 1] - P[3 * w + 1];
    }
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const double F0 = c.wS * (J0[v] * kThird + J0[1 - v] * kSixth);
        const double F1 = c.wS * (J1[v] * kThird + J1[1 - v] * kSixth) * kThird;
        y[3 * v] -= F0;
        y[3 * v + 2] += F0;
        y[3 * v + 1] -= F1;
    }
    // upper and lower faces
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        y[3 + h] += c.wT * kMh[h] * (P[3 + h] - Up[h]);
        y[h] -= c.wB * kMh[h] * (Dn[h] - P[h]);
    }
}

// Entry (a, b) of the cell's own 6 x 6 block of H1_z: cell term, self parts
// of the four horizontal faces and of the two vertical faces.
__device__ __forceinline__ double dg1_block(const Dg1Coef &c, int a, int b)
{
    const int v = a / 3, h = a % 3, w = b / 3, g = b % 3;
    const double mv = (v == w) ? kThird : kSixth;
    const double kv = (v == w) ? 0.25 : -0.25;
    const double sx = c.wE + c.wW, sy = c.wN + c.wS;
    if (h == g) {
        const double hs = (h == 0) ? sx + sy : ((h == 1) ? sx + sy * kThird : sx * kThird + sy);
        double val = (c.al[h] + hs) * mv + c.be[h] * kv;
        if (v == w) val += (v == 1 ? c.wT : c.wB) * kMh[h];
        return val;
    }
    if ((h == 0 && g == 1) || (h == 1 && g == 0)) return (c.wE - c.wW) * mv;
    if ((h == 0 && g == 2) || (h == 2 && g == 0)) return (c.wN - c.wS) * mv;
    return 0.0;
}

__device__ __forceinline__ void ld6(double (&v)[6], Rsrc r, unsigned voff, unsigned k, unsigned nz, unsigned row)
{
#pragma unroll
    for (int a = 0; a < kNb; ++a) v[a] = bload(double(), r, voff, (a * nz + k) * row);
}

// ---------------------------------------------------------------------------
// Band LU of every column block (setup): one lane per column streams its rows
// r = 6k + a, assembles row r of H1_z from the cell's coefficients and forms
// L(r, r-5..r-1) and U(r, r..r+5) from the five previous rows of U
// (Doolittle order; the same sums, in the same order, as Gaussian
// elimination restricted to the band).  No pivoting: H1_z is symmetric
// positive definite.  A non-positive or non-finite pivot counts into *bad.
// ---------------------------------------------------------------------------
template <typename FT>
__global__ __launch_bounds__(256) void k_dg1_factor(Dg1Level G, FT *__restrict__ fac, int *__restrict__ bad)
{
    const Dg1Lane q = dg1_lane<FT>(G, fac, xcd_remap(blockIdx.x, gridDim.x));
    const int nz = G.nz;
    const unsigned oo = q.active ? q.of : 0xFFFFFFFFu;
    double Uw[5][6], Iw[5];  // rows r-1 .. r-5: U(q, q..q+5), 1/U(q, q)
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        Iw[d] = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) Uw[d][j] = 0.0;
    }
    int nbad = 0;
    double cUm = 0.0;
    for (int k = 0; k < nz; ++k) {
        const Dg1Faces f = dg1_faces(q, (unsigned)k);
        const Dg1Coef c = dg1_coef(G, k, f, cUm);
        cUm = f.cU;
#pragma unroll
        for (int a = 0; a < kNb; ++a) {
            // row r = 6k + a of H1_z: band[e] = H1_z(r, r - 5 + e)
            double band[kNf];
#pragma unroll
            for (int e = 0; e < kNf; ++e) {
                const int b = a + e - 5;
                band[e] = (b >= 0 && b < kNb) ? dg1_block(c, a, b) : 0.0;
            }
            if (a < 3) band[2] = -c.wB * kMh[a];          // bottom value -> top value of the cell below
            else band[8] = -c.wT * kMh[a - 3];             // top value -> bottom value of the cell above
            double l[6];  // l[d] = L(r, r - d), d = 1..5
#pragma unroll
            for (int d = 5; d >= 1; --d) {
                double s = band[5 - d];
#pragma unroll
                for (int dd = 5; dd > d; --dd) s -= l[dd] * Uw[dd - 1][dd - d];
                l[d] = s * Iw[d - 1];
            }
            double u[6];  // u[j] = U(r, r + j)
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                double s = band[5 + j];
#pragma unroll
                for (int d = 5 - j; d >= 1; --d) s -= l[d] * Uw[d - 1][j + d];
                u[j] = s;
            }
            const bool ok = u[0] > 0.0 && u[0] <= kDblMax;
            if (!ok) ++nbad;
            const double iu = ok ? 1.0 / u[0] : 0.0;
#pragma unroll
            for (int d = 4; d > 0; --d) {
                Iw[d] = Iw[d - 1];
#pragma unroll
                for (int j = 0; j < 6; ++j) Uw[d][j] = Uw[d - 1][j];
            }
            Iw[0] = iu;
#pragma unroll
            for (int j = 0; j < 6; ++j) Uw[0][j] = u[j];
            const unsigned rr = (unsigned)(kNb * k + a) * kNf;
#pragma unroll
            for (int e = 0; e < 5; ++e) bstore((FT)l[5 - e], q.rF, oo, (rr + e) * q.frow);
            bstore((FT)iu, q.rF, oo, (rr + 5) * q.frow);
#pragma unroll
            for (int j = 1; j < 6; ++j) bstore((FT)u[j], q.rF, oo, (rr + 5 + j) * q.frow);
        }
    }
    if (q.active && nbad) atomicAdd(bad, nbad);
}

// ---------------------------------------------------------------------------
// Line sweep (Sec. 4.2 smoother with the DG1 column blocks):
//   ZERO:     out = omega H1_z^{-1} b
//   GENERAL:  out = u + omega H1_z^{-1} (b - H1 u)
//   SOLVE:    out = H1_z^{-1} b
// Forward pass over the rows: right-hand side, y = L^{-1} rhs, y written to
// out; backward pass: x = U^{-1} y read back from out, then the update.
// ---------------------------------------------------------------------------
enum Dg1SweepMode : int { DG1_ZERO = 0, DG1_GENERAL = 1, DG1_SOLVE = 2 };

// Loads of one cell's rows for the forward pass: the right-hand side and
// L(r, r-5..r-1) of its six rows.
struct Dg1Fwd {
    double b[6], l[6][5];
};
// ... and for the backward pass: y (read back from the output), 1/U(r, r)
// and U(r, r+1..r+5), and u for the update.
struct Dg1Bwd {
    double y[6], u[6][6], uo[6];
};

// All loads of a cell are issued before any of its arithmetic and stores
// (the stores go through the same kind of buffer access, so the compiler
// keeps loads that follow a store in program order behind it); with PF the
// forward loads of cell k + 1 are issued before the stores of cell k.
// CP: cache policy of the data the sweep reads or writes once (the band
// factors, b, the final output); y, written in the forward pass and read back
// in the backward pass, and u keep the default policy.
template <int MODE, bool PF, int CP, typename FT>
__global__ __launch_bounds__(256) void k_dg1_sweep(Dg1Level G, const FT *__restrict__ fac,
                                                   const double *__restrict__ u, const double *__restrict__ b,
                                                   double *__restrict__ out, double omega)
{
    const Dg1Lane q = dg1_lane<FT>(G, fac, xcd_remap(blockIdx.x, gridDim.x));
    const unsigned nz = (unsigned)G.nz;
    const size_t vbytes = (size_t)kNb * nz * G.plane * 8;
    const Rsrc ru = make_rsrc(u ? u : b, vbytes), rb = make_rsrc(b, vbytes), ro = make_rsrc(out, vbytes);
    const unsigned oo = q.active ? q.ov : 0xFFFFFFFFu;
    auto load_fwd = [&](Dg1Fwd &F, unsigned k) {
#pragma unroll
        for (int a = 0; a < kNb; ++a) F.b[a] = bload<CP>(double(), rb, q.ov, (a * nz + k) * q.row);
#pragma unroll
        for (int a = 0; a < kNb; ++a)
#pragma unroll
            for (int e = 0; e < 5; ++e)
                F.l[a][e] = (double)bload<CP>(FT(), q.rF, q.of, ((kNb * k + a) * kNf + e) * q.frow);
    };
    auto load_bwd = [&](Dg1Bwd &B, unsigned k) {
        ld6(B.y, ro, q.ov, k, nz, q.row);
        if constexpr (MODE == DG1_GENERAL) ld6(B.uo, ru, q.ov, k, nz, q.row);
#pragma unroll
        for (int a = 0; a < kNb; ++a)
#pragma unroll
            for (int e = 0; e < 6; ++e)
                B.u[a][e] = (double)bload<CP>(FT(), q.rF, q.of, ((kNb * k + a) * kNf + 5 + e) * q.frow);
    };

    double yw[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // y(r-1) .. y(r-5)
    double cur[6], dn[3] = {0.0, 0.0, 0.0};
    if constexpr (MODE == DG1_GENERAL) ld6(cur, ru, q.ov, 0, nz, q.row);
    double cUm = 0.0;
    Dg1Fwd F;
    load_fwd(F, 0);
    for (unsigned k = 0; k < nz; ++k) {
        Dg1Fwd Fn;
        if constexpr (PF) {
            if (k + 1 < nz) load_fwd(Fn, k + 1);
        }
        double rhs[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) rhs[a] = F.b[a];
        if constexpr (MODE == DG1_GENERAL) {
            const Dg1Faces f = dg1_faces(q, k);
            double nxt[6], E[6], Wc[6], N[6], S[6];
            if (k + 1 < nz) ld6(nxt, ru, q.ov, k + 1, nz, q.row);
            else
#pragma unroll
                for (int a = 0; a < 6; ++a) nxt[a] = 0.0;
            ld6(E, ru, q.oe, k, nz, q.row);
            ld6(Wc, ru, q.ow, k, nz, q.row);
            ld6(N, ru, q.on, k, nz, q.row);
            ld6(S, ru, q.os, k, nz, q.row);
            const Dg1Coef c = dg1_coef(G, (int)k, f, cUm);
            cUm = f.cU;
            const double up[3] = {nxt[0], nxt[1], nxt[2]};
            double hy[6];
            dg1_cell_apply(cur, E, Wc, N, S, dn, up, c, hy);
#pragma unroll
            for (int a = 0; a < 6; ++a) rhs[a] -= hy[a];
#pragma unroll
            for (int h = 0; h < 3; ++h) dn[h] = cur[3 + h];
#pragma unroll
            for (int a = 0; a < 6; ++a) cur[a] = nxt[a];
        }
        double y[6];
#pragma unroll
        for (int a = 0; a < kNb; ++a) {
            double s = rhs[a];
#pragma unroll
            for (int d = 1; d <= 5; ++d) s -= F.l[a][5 - d] * yw[d - 1];
#pragma unroll
            for (int d = 4; d > 0; --d) yw[d] = yw[d - 1];
            yw[0] = s;
            y[a] = s;
        }
#pragma unroll
        for (int a = 0; a < kNb; ++a) bstore(y[a], ro, oo, (a * nz + k) * q.row);
        if (k + 1 < nz) {
            if constexpr (PF) F = Fn;
            else load_fwd(F, k + 1);
        }
    }
    double xw[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // x(r+1) .. x(r+5)
    Dg1Bwd B;
    load_bwd(B, nz - 1);
    for (int k = (int)nz - 1; k >= 0; --k) {
        Dg1Bwd Bn;
        if constexpr (PF) {
            if (k > 0) load_bwd(Bn, (unsigned)k - 1);
        }
        double o[6];
#pragma unroll
        for (int a = kNb - 1; a >= 0; --a) {
            double s = B.y[a];
#pragma unroll
            for (int d = 1; d <= 5; ++d) s -= B.u[a][d] * xw[d - 1];
            const double x = s * B.u[a][0];
#pragma unroll
            for (int d = 4; d > 0; --d) xw[d] = xw[d - 1];
            xw[0] = x;
            if constexpr (MODE == DG1_GENERAL) o[a] = B.uo[a] + omega * x;
            else if constexpr (MODE == DG1_ZERO) o[a] = omega * x;
            else o[a] = x;
        }
#pragma unroll
        for (int a = 0; a < kNb; ++a) bstore<CP>(o[a], ro, oo, ((unsigned)a * nz + (unsigned)k) * q.row);
        if (k > 0) {
            if constexpr (PF) B = Bn;
            else load_bwd(B, (unsigned)k - 1);
        }
    }
}

// ---------------------------------------------------------------------------
// Operator kernels (one lane per column, streaming k):
//   APPLY:  y = H1 x
//   RESID:  y = b - H1 x (y may be null) and partial sums of (y, y)
//   PCG:    p = z + beta p_old (p = z on the first iteration), q = H1 p,
//           partial sums of (p, q); beta from the CG scalars
// ---------------------------------------------------------------------------
enum Dg1OpMode : int { DG1_APPLY = 0, DG1_RESID = 1, DG1_PCG = 2 };

// Workgroup -> (chunk of kc cells along k, block of 256 columns), the
// chunks outermost, XCD-aware.
__device__ __forceinline__ void dg1_chunk(const Dg1Level &G, int kc, int &cb, unsigned &k0, unsigned &k1)
{
    const int ncb = (G.plane + 255) / 256;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int c = blk / ncb;
    cb = blk - c * ncb;
    k0 = (unsigned)(c * kc);
    k1 = (unsigned)min(G.nz, (c + 1) * kc);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_dg1_op(Dg1Level G, int kc, const double *__restrict__ x,
                                                const double *__restrict__ x2, const double *__restrict__ b,
                                                double *__restrict__ y, double *__restrict__ pout,
                                                const Scalars *__restrict__ sc, int first,
                                                double *__restrict__ partials)
{
    int cb;
    unsigned k0, k1;
    dg1_chunk(G, kc, cb, k0, k1);
    const Dg1Lane q = dg1_lane<double>(G, nullptr, cb);
    const unsigned nz = (unsigned)G.nz;
    const size_t vbytes = (size_t)kNb * nz * G.plane * 8;
    const Rsrc rx = make_rsrc(x, vbytes), rx2 = make_rsrc(x2 ? x2 : x, vbytes);
    const Rsrc rb = make_rsrc(b ? b : x, vbytes), ry = make_rsrc(y ? y : x, y ? vbytes : 0);
    const Rsrc rp = make_rsrc(pout ? pout : x, pout ? vbytes : 0);
    const unsigned oo = q.active ? q.ov : 0xFFFFFFFFu;
    double beta = 0.0;
    if constexpr (MODE == DG1_PCG) beta = first ? 0.0 : sc->beta;
    // operand value of a cell: x, or z + beta p_old
    auto load6 = [&](double (&v)[6], unsigned off, unsigned k) {
        ld6(v, rx, off, k, nz, q.row);
        if constexpr (MODE == DG1_PCG) {
            if (!first) {
                double p[6];
                ld6(p, rx2, off, k, nz, q.row);
#pragma unroll
                for (int a = 0; a < 6; ++a) v[a] += beta * p[a];
            }
        }
    };
    double acc = 0.0;
    double cur[6], nxt[6], dn[3] = {0.0, 0.0, 0.0};
    load6(cur, q.ov, k0);
    double cUm = 0.0;
    if (k0 > 0) {
        double below[6];
        load6(below, q.ov, k0 - 1);
#pragma unroll
        for (int h = 0; h < 3; ++h) dn[h] = below[3 + h];
        cUm = bload(double(), q.rU, q.oc, (k0 - 1) * q.row);
    }
    for (unsigned k = k0; k < k1; ++k) {
        const Dg1Faces f = dg1_faces(q, k);
        const Dg1Coef c = dg1_coef(G, (int)k, f, cUm);
        cUm = f.cU;
        double E[6], Wc[6], N[6], S[6];
        if (k + 1 < nz) load6(nxt, q.ov, k + 1);
        else
#pragma unroll
            for (int a = 0; a < 6; ++a) nxt[a] = 0.0;
        load6(E, q.oe, k);
        load6(Wc, q.ow, k);
        load6(N, q.on, k);
        load6(S, q.os, k);
        const double up[3] = {nxt[0], nxt[1], nxt[2]};
        double hy[6];
        dg1_cell_apply(cur, E, Wc, N, S, dn, up, c, hy);
        if constexpr (MODE == DG1_RESID) {
            double bb[6];
            ld6(bb, rb, q.ov, k, nz, q.row);
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                const double r = bb[a] - hy[a];
                if (y) bstore(r, ry, oo, (a * nz + k) * q.row);
                if (q.active) acc += r * r;
            }
        } else {
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                bstore(hy[a], ry, oo, (a * nz + k) * q.row);
                if constexpr (MODE == DG1_PCG) {
                    bstore(cur[a], rp, oo, (a * nz + k) * q.row);
                    if (q.active) acc += cur[a] * hy[a];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 3; ++h) dn[h] = cur[3 + h];
#pragma unroll
        for (int a = 0; a < 6; ++a) cur[a] = nxt[a];
    }
    if constexpr (MODE != DG1_APPLY) {
        double v[1] = {acc};
        block_partials<1>(v, partials, gridDim.x, blockIdx.x);
    }
}

// ---------------------------------------------------------------------------
// p-restriction of the residual (Sec. 4.2.1, transpose of the embedding):
//   b0(col, k) = r_0 + r_3,  r = b - H1 u  of the cell (bottom and top values
//   of the constant mode), into a lowest-order level-0 vector of type T.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_dg1_resid_restrict(Dg1Level G, int kc, const double *__restrict__ u,
                                                            const double *__restrict__ b, T *__restrict__ b0)
{
    int cb;
    unsigned k0, k1;
    dg1_chunk(G, kc, cb, k0, k1);
    const Dg1Lane q = dg1_lane<double>(G, nullptr, cb);
    const unsigned nz = (unsigned)G.nz;
    const size_t vbytes = (size_t)kNb * nz * G.plane * 8;
    const Rsrc ru = make_rsrc(u, vbytes), rb = make_rsrc(b, vbytes);
    const Rsrc r0 = make_rsrc(b0, (size_t)nz * G.plane * sizeof(T));
    const unsigned oo = q.active ? q.oc / (8 / sizeof(T)) : 0xFFFFFFFFu;
    const unsigned row0 = q.row / (8 / sizeof(T));
    double cur[6], nxt[6], dn[3] = {0.0, 0.0, 0.0};
    ld6(cur, ru, q.ov, k0, nz, q.row);
    double cUm = 0.0;
    if (k0 > 0) {
#pragma unroll
        for (int h = 0; h < 3; ++h) dn[h] = bload(double(), ru, q.ov, ((3 + h) * nz + k0 - 1) * q.row);
        cUm = bload(double(), q.rU, q.oc, (k0 - 1) * q.row);
    }
    for (unsigned k = k0; k < k1; ++k) {
        const Dg1Faces f = dg1_faces(q, k);
        const Dg1Coef c = dg1_coef(G, (int)k, f, cUm);
        cUm = f.cU;
        double E[6], Wc[6], N[6], S[6];
        if (k + 1 < nz) ld6(nxt, ru, q.ov, k + 1, nz, q.row);
        else
#pragma unroll
            for (int a = 0; a < 6; ++a) nxt[a] = 0.0;
        ld6(E, ru, q.oe, k, nz, q.row);
        ld6(Wc, ru, q.ow, k, nz, q.row);
        ld6(N, ru, q.on, k, nz, q.row);
        ld6(S, ru, q.os, k, nz, q.row);
        const double up[3] = {nxt[0], nxt[1], nxt[2]};
        double hy[6];
        dg1_cell_apply(cur, E, Wc, N, S, dn, up, c, hy);
        const double r0v = bload(double(), rb, q.ov, k * q.row) - hy[0];
        const double r3v = bload(double(), rb, q.ov, (3 * nz + k) * q.row) - hy[3];
        bstore((T)(r0v + r3v), r0, oo, k * row0);
#pragma unroll
        for (int h = 0; h < 3; ++h) dn[h] = cur[3 + h];
#pragma unroll
        for (int a = 0; a < 6; ++a) cur[a] = nxt[a];
    }
}

// u += P e0: the lowest-order correction added to the bottom and top values
// of the constant mode (natural embedding).  Thread = one (column, k).
template <typename T>
__global__ __launch_bounds__(256) void k_dg1_prolong(int plane, int nz, const T *__restrict__ e0,
                                                     double *__restrict__ u)
{
    const size_t g = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (size_t)plane * nz) return;
    const int W = tile_width(plane);
    // g enumerates the lowest-order storage: (col, k) at cell_base(col, nz) + k W
    size_t col;
    int k;
    if (W == 64) {
        const size_t tile = g / ((size_t)nz * 64);
        const size_t rem = g - tile * nz * 64;
        k = (int)(rem / 64);
        col = tile * 64 + (rem & 63);
    } else {
        k = (int)(g / plane);
        col = g - (size_t)k * plane;
    }
    const double e = (double)e0[g];
    const size_t base = cell_base(col, plane, kNb * nz);
    u[base + (size_t)k * W] += e;
    u[base + (size_t)(3 * nz + k) * W] += e;
}

// Band factors in the order [col][row][entry] with U(r, r) itself in entry 5.
template <typename FT>
__global__ __launch_bounds__(256) void k_dg1_factors_out(int plane, int nz, const FT *__restrict__ fac,
                                                         double *__restrict__ dst)
{
    const size_t g = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t rows = (size_t)kNb * nz, total = (size_t)plane * rows * kNf;
    if (g >= total) return;
    const size_t col = g / (rows * kNf), rem = g - col * rows * kNf;
    const size_t r = rem / kNf, e = rem - r * kNf;
    const int W = tile_width(plane);
    const size_t tile = col / W, lane = col - tile * W;
    const double v = (double)fac[tile * rows * kNf * W + (r * kNf + e) * W + lane];
    dst[g] = (e == 5) ? 1.0 / v : v;
}

inline unsigned dg1_blocks(int plane) { return (unsigned)((plane + 255) / 256); }

// Cells along k per workgroup of the operator kernels: TPMG_DG1_KC, else 64.
// Measured at 256^2 x 64 (CG direction update + apply): 8: 263, 16: 270,
// 32: 258, 64: 251 us; shorter chunks add workgroups but not speed.
inline int dg1_kc(int nz)
{
    static const int e = env_int("TPMG_DG1_KC");
    const int kc = (e >= 1) ? e : 64;
    return kc < nz ? kc : nz;
}
inline unsigned dg1_chunk_blocks(const Dg1Level &G, int kc)
{
    return dg1_blocks(G.plane) * (unsigned)((G.nz + kc - 1) / kc);
}

}  // namespace

// ---- launchers ------------------------------------------------------------------

hipError_t launch_dg1_factor(const Dg1Level &G, void *fac, int *bad, hipStream_t s)
{
    if (G.fac32)
        hipLaunchKernelGGL(k_dg1_factor<float>, dim3(dg1_blocks(G.plane)), dim3(256), 0, s, G, (float *)fac, bad);
    else
        hipLaunchKernelGGL(k_dg1_factor<double>, dim3(dg1_blocks(G.plane)), dim3(256), 0, s, G, (double *)fac,
                           bad);
    return hipGetLastError();
}

template <bool PF, int CP, typename FT>
void dg1_sweep_ft(const Dg1Level &G, const FT *fac, int mode, const double *u, const double *b, double *out,
                  double omega, hipStream_t s)
{
    const dim3 grid(dg1_blocks(G.plane)), block(256);
    if (mode == DG1_SWEEP_GENERAL)
        hipLaunchKernelGGL((k_dg1_sweep<DG1_GENERAL, PF, CP, FT>), grid, block, 0, s, G, fac, u, b, out, omega);
    else if (mode == DG1_SWEEP_ZERO)
        hipLaunchKernelGGL((k_dg1_sweep<DG1_ZERO, PF, CP, FT>), grid, block, 0, s, G, fac, nullptr, b, out, omega);
    else
        hipLaunchKernelGGL((k_dg1_sweep<DG1_SOLVE, PF, CP, FT>), grid, block, 0, s, G, fac, nullptr, b, out, 1.0);
}

template <bool PF, int CP>
void dg1_sweep_pf(const Dg1Level &G, const void *fac, int mode, const double *u, const double *b, double *out,
                  double omega, hipStream_t s)
{
    if (G.fac32)
        dg1_sweep_ft<PF, CP>(G, (const float *)fac, mode, u, b, out, omega, s);
    else
        dg1_sweep_ft<PF, CP>(G, (const double *)fac, mode, u, b, out, omega, s);
}

hipError_t launch_dg1_sweep(const Dg1Level &G, const void *fac, int mode, const double *u, const double *b,
                            double *out, double omega, hipStream_t s)
{
    // TPMG_DG1_PF = 1: the next cell's forward / backward loads issued ahead
    // of this cell's stores (256 VGPRs in the general form); measured at
    // 256^2 x 64 it ran as fast as the default (0.717 vs 0.713 ms)
    static const int pf = env_int("TPMG_DG1_PF");
    // Non-temporal factors, b and output when the factors exceed the 256 MB
    // last-level cache (TPMG_DG1_NT=0: never, 1: always): measured at
    // 256^2 x 64 (2.2 GB of factors), general sweep 0.646 vs 0.715 ms.
    static const int nt = env_int("TPMG_DG1_NT");
    const bool big = (size_t)G.plane * kNb * G.nz * kNf * (G.fac32 ? 4 : 8) >= ((size_t)1 << 28);
    if (pf == 1)
        dg1_sweep_pf<true, 0>(G, fac, mode, u, b, out, omega, s);
    else if (nt == 1 || (nt != 0 && big))
        dg1_sweep_pf<false, kNT>(G, fac, mode, u, b, out, omega, s);
    else
        dg1_sweep_pf<false, 0>(G, fac, mode, u, b, out, omega, s);
    return hipGetLastError();
}

hipError_t launch_dg1_apply(const Dg1Level &G, const double *x, double *y, hipStream_t s)
{
    const int kc = dg1_kc(G.nz);
    hipLaunchKernelGGL(k_dg1_op<DG1_APPLY>, dim3(dg1_chunk_blocks(G, kc)), dim3(256), 0, s, G, kc, x, nullptr,
                       nullptr, y, nullptr, nullptr, 0, nullptr);
    return hipGetLastError();
}

hipError_t launch_dg1_residual(const Dg1Level &G, const double *x, const double *b, double *r, double *partials,
                               int *nblocks_out, hipStream_t s)
{
    const int kc = dg1_kc(G.nz);
    const unsigned G0 = dg1_chunk_blocks(G, kc);
    if (G0 > (unsigned)kMaxPartials) return hipErrorInvalidValue;
    *nblocks_out = (int)G0;
    hipLaunchKernelGGL(k_dg1_op<DG1_RESID>, dim3(G0), dim3(256), 0, s, G, kc, x, nullptr, b, r, nullptr, nullptr, 0,
                       partials);
    return hipGetLastError();
}

hipError_t launch_dg1_pcg_apply(const Dg1Level &G, const double *z, const double *p_old, double *p_new, double *q,
                                const Scalars *sc, int first, double *partials, int *nblocks_out, hipStream_t s)
{
    const int kc = dg1_kc(G.nz);
    const unsigned G0 = dg1_chunk_blocks(G, kc);
    if (G0 > (unsigned)kMaxPartials) return hipErrorInvalidValue;
    *nblocks_out = (int)G0;
    hipLaunchKernelGGL(k_dg1_op<DG1_PCG>, dim3(G0), dim3(256), 0, s, G, kc, z, p_old, nullptr, q, p_new, sc, first,
                       partials);
    return hipGetLastError();
}

hipError_t launch_dg1_resid_restrict(const Dg1Level &G, const double *u, const double *b, void *b0, int fp32,
                                     hipStream_t s)
{
    const int kc = dg1_kc(G.nz);
    const dim3 grid(dg1_chunk_blocks(G, kc)), block(256);
    if (fp32)
        hipLaunchKernelGGL(k_dg1_resid_restrict<float>, grid, block, 0, s, G, kc, u, b, (float *)b0);
    else
        hipLaunchKernelGGL(k_dg1_resid_restrict<double>, grid, block, 0, s, G, kc, u, b, (double *)b0);
    return hipGetLastError();
}

hipError_t launch_dg1_prolong(const Dg1Level &G, const void *e0, int fp32, double *u, hipStream_t s)
{
    const unsigned blocks = (unsigned)(((size_t)G.plane * G.nz + 255) / 256);
    if (fp32)
        hipLaunchKernelGGL(k_dg1_prolong<float>, dim3(blocks), dim3(256), 0, s, G.plane, G.nz, (const float *)e0, u);
    else
        hipLaunchKernelGGL(k_dg1_prolong<double>, dim3(blocks), dim3(256), 0, s, G.plane, G.nz, (const double *)e0,
                           u);
    return hipGetLastError();
}

hipError_t launch_dg1_factors_out(const Dg1Level &G, const void *fac, double *dst, hipStream_t s)
{
    const size_t total = (size_t)G.plane * kNb * G.nz * kNf;
    const dim3 grid((unsigned)((total + 255) / 256));
    if (G.fac32)
        hipLaunchKernelGGL(k_dg1_factors_out<float>, grid, dim3(256), 0, s, G.plane, G.nz, (const float *)fac, dst);
    else
        hipLaunchKernelGGL(k_dg1_factors_out<double>, grid, dim3(256), 0, s, G.plane, G.nz, (const double *)fac,
                           dst);
    return hipGetLastError();
}

}  // namespace tpmg
