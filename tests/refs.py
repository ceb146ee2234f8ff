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
