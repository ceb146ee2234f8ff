"""Independent constructions used to pin the oracle (test helpers).

Everything here is built from the problem definition by a different route
than the oracle takes (sparse incidence matrices, dense numpy algebra,
Fourier/cosine transforms), so a slip in the oracle's index arithmetic,
signs or scalings shows up as a mismatch.
"""
import numpy as np
import scipy.fft as sfft


def cell_index(n, nz, i, j, k):
    return (k * n + (j % n)) * n + (i % n)


def vertical_metrics(nz, dz=None):
    dz = np.ones(nz) if dz is None else np.asarray(dz, dtype=np.float64)
    s = dz / dz.mean()
    t = 0.5 * (s[:-1] + s[1:])
    return s, t


def incidence_operator(c, a_h, a_z, dz=None, level=0):
    """H = M + B diag(w) B^T from the cell-face incidence matrix B.

    c: (3, nz, n, n) coefficients at this level.  Faces: E of (i,j,k) joins
    (i+1,j,k); N joins (i,j+1,k); U joins (i,j,k+1) for k < nz-1."""
    _, nz, n, _ = c.shape
    s, t = vertical_metrics(nz, dz)
    m = n * n * nz
    rows, weights = [], []
    for k in range(nz):
        for j in range(n):
            for i in range(n):
                p = cell_index(n, nz, i, j, k)
                rows.append((p, cell_index(n, nz, i + 1, j, k), a_h * s[k] * c[0, k, j, i]))
                rows.append((p, cell_index(n, nz, i, j + 1, k), a_h * s[k] * c[1, k, j, i]))
                if k + 1 < nz:
                    rows.append((p, cell_index(n, nz, i, j, k + 1),
                                 4.0 ** level * a_z * c[2, k, j, i] / t[k]))
    B = np.zeros((m, len(rows)))
    w = np.zeros(len(rows))
    for f, (p, q, wf) in enumerate(rows):
        B[p, f] += 1.0
        B[q, f] -= 1.0
        w[f] = wf
    mass = np.repeat(4.0 ** level * s, n * n)
    return np.diag(mass) + (B * w) @ B.T


def prolongation(n, nz):
    """Dense natural-embedding matrix from the (n/2)^2 x nz level to n^2 x nz."""
    nc = n // 2
    P = np.zeros((n * n * nz, nc * nc * nz))
    for k in range(nz):
        for j in range(n):
            for i in range(n):
                P[cell_index(n, nz, i, j, k), cell_index(nc, nz, i // 2, j // 2, k)] = 1.0
    return P


def column_block(A, n, nz):
    """Keep only couplings inside a vertical column (the H_z of the paper)."""
    idx = np.arange(n * n * nz)
    col = idx % (n * n)
    return np.where(col[:, None] == col[None, :], A, 0.0)


def closed_form_eigs(n, nz, a_h, a_z, c0, level=0):
    l1 = np.arange(n)
    th = 2 * np.pi * l1 / n
    m = np.arange(nz)
    lam = (4.0 ** level
           + 2 * a_h * c0 * (2 - np.cos(th)[None, :, None] - np.cos(th)[None, None, :])
           + 4.0 ** level * 2 * a_z * c0 * (1 - np.cos(np.pi * m / nz))[:, None, None])
    return lam  # shape (nz, n, n): index (m, ly, lx)


def closed_form_solve(b, a_h, a_z, c0):
    """Uniform coefficients and spacing: diagonalised by FFT in i, j and DCT-II in k."""
    nz, n, _ = b.shape
    lam = closed_form_eigs(n, nz, a_h, a_z, c0)
    bh = sfft.dct(b, type=2, axis=0, norm="ortho")
    bh = np.fft.fft2(bh, axes=(1, 2))
    xh = bh / lam
    x = np.fft.ifft2(xh, axes=(1, 2)).real
    return sfft.idct(x, type=2, axis=0, norm="ortho")


def random_coeffs(rng, n, nz, lo=1.0, hi=1.5):
    return rng.uniform(lo, hi, size=(3, nz, n, n))


def patch(field, i, j, size=3, lo=1):
    """The periodic size x size block of columns starting at (i - lo, j - lo)
    of a (..., nz, n, n) field.  With size 3 (lo 1) the block holds every
    stencil input of column (i, j): its four neighbours and the faces between;
    with size 4 (lo 1) at (2I, 2J) it holds every input of the residual of
    the four children of coarse column (I, J)."""
    n = field.shape[-1]
    ii = (np.arange(size) + i - lo) % n
    jj = (np.arange(size) + j - lo) % n
    return field[..., jj[:, None], ii[None, :]]


# -- DG1 (next-to-lowest order) pressure: an independent quadrature route ------------
_GAUSS2 = np.array([-1.0, 1.0]) / np.sqrt(3.0)   # 2-point Gauss on [-1, 1], weights 1 each


def _dg1_eval(Ucell, xi, eta, zeta):
    """Value and reference derivatives (d/dxi, d/deta, d/dzeta) at one point of
    u = sum U[3v+h] l_v(zeta) psi_h(xi, eta), psi = (1, xi, eta), l = ((1-zeta)/2, (1+zeta)/2)."""
    psi = np.array([1.0, xi, eta])
    dpsi_xi = np.array([0.0, 1.0, 0.0])
    dpsi_eta = np.array([0.0, 0.0, 1.0])
    lv = np.array([(1 - zeta) / 2, (1 + zeta) / 2])
    dlv = np.array([-0.5, 0.5])
    Uv = Ucell.reshape(2, 3)
    return (lv @ Uv @ psi, lv @ Uv @ dpsi_xi, lv @ Uv @ dpsi_eta, dlv @ Uv @ psi)


def dg1_quadrature_form(c, a_h, a_z, dz, U, W):
    """a(U, W) of the DG1 form evaluated by Gauss quadrature in physical
    coordinates: cell (i, j, k) is [i, i+1] x [j, j+1] x [z_k, z_k + s_k]
    (s = dz / mean dz), density-1 mass, K = diag(a_h c^x, a_h c^y, a_z c^z)
    with the cell coefficients of the definition, and the jump penalty with
    density w_f / |f| on every interior face (a_h c_f on x / y faces of area
    s_k, a_z c_f / t_{k+1/2} on z faces of area 1).  U, W: (6, nz, n, n)."""
    _, nz, n, _ = c.shape
    s, t = vertical_metrics(nz, dz)
    cell = lambda A, i, j, k: A[:, k, j % n, i % n]
    total = 0.0
    for k in range(nz):
        cz = c[2, 0] if k == 0 else (c[2, nz - 2] if k == nz - 1 else 0.5 * (c[2, k] + c[2, k - 1]))
        for j in range(n):
            for i in range(n):
                cx = 0.5 * (c[0, k, j, i] + c[0, k, j, (i - 1) % n])
                cy = 0.5 * (c[1, k, j, i] + c[1, k, (j - 1) % n, i])
                Kx, Ky, Kz = a_h * cx, a_h * cy, a_z * cz[j, i]
                u, w = cell(U, i, j, k), cell(W, i, j, k)
                vol = s[k]                     # volume 1 x 1 x s_k; quadrature weight vol / 8
                for xi in _GAUSS2:
                    for eta in _GAUSS2:
                        for ze in _GAUSS2:
                            fu = _dg1_eval(u, xi, eta, ze)
                            fw = _dg1_eval(w, xi, eta, ze)
                            # physical derivatives: d/dx = 2 d/dxi, d/dy = 2 d/deta, d/dz = (2 / s_k) d/dzeta
                            grad = (Kx * 4 * fu[1] * fw[1] + Ky * 4 * fu[2] * fw[2] +
                                    Kz * (2 / s[k]) ** 2 * fu[3] * fw[3])
                            total += vol / 8 * (fu[0] * fw[0] + grad)
                # x face at the east end: cells (i, j, k) | (i+1, j, k), area s_k
                for d in (0, 1):
                    ul, wl = cell(U, i, j, k), cell(W, i, j, k)
                    ur = cell(U, i + 1, j, k) if d == 0 else cell(U, i, j + 1, k)
                    wr = cell(W, i + 1, j, k) if d == 0 else cell(W, i, j + 1, k)
                    dens = a_h * c[d, k, j, i]
                    for p in _GAUSS2:
                        for ze in _GAUSS2:
                            if d == 0:
                                jl = _dg1_eval(ul, 1.0, p, ze)[0] - _dg1_eval(ur, -1.0, p, ze)[0]
                                jw = _dg1_eval(wl, 1.0, p, ze)[0] - _dg1_eval(wr, -1.0, p, ze)[0]
                            else:
                                jl = _dg1_eval(ul, p, 1.0, ze)[0] - _dg1_eval(ur, p, -1.0, ze)[0]
                                jw = _dg1_eval(wl, p, 1.0, ze)[0] - _dg1_eval(wr, p, -1.0, ze)[0]
                            total += s[k] / 4 * dens * jl * jw
                if k + 1 < nz:   # z face at the top: cells k | k+1, area 1
                    ul, wl = cell(U, i, j, k), cell(W, i, j, k)
                    ur, wr = cell(U, i, j, k + 1), cell(W, i, j, k + 1)
                    dens = a_z * c[2, k, j, i] / t[k]
                    for xi in _GAUSS2:
                        for eta in _GAUSS2:
                            jl = _dg1_eval(ul, xi, eta, 1.0)[0] - _dg1_eval(ur, xi, eta, -1.0)[0]
                            jw = _dg1_eval(wl, xi, eta, 1.0)[0] - _dg1_eval(wr, xi, eta, -1.0)[0]
                            total += 1.0 / 4 * dens * jl * jw
    return total


def dg1_embedding(n, nz):
    """Dense natural embedding DG0 -> DG1 on the same grid (logical orders):
    a cellwise constant is the DG1 function with bottom and top values c."""
    m0 = n * n * nz
    P = np.zeros((6 * m0, m0))
    for q in range(m0):
        P[0 * m0 + q, q] = 1.0   # a = 3 v + h with v = 0 (bottom), h = 0 (constant)
        P[3 * m0 + q, q] = 1.0   # v = 1 (top), h = 0
    return P
