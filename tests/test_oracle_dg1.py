"""Pins for the oracle's next-to-lowest-order (DG1) pressure level: the
operator against Gauss quadrature of its defining bilinear form in physical
coordinates, the exact Galerkin relation to the lowest-order operator under
the natural embedding (Sec. 4.2.1), the banded column block and its LU
(Sec. 4.3.1) against dense algebra, the NLO V-cycle against a dense
brute-force cycle, and PCG against a dense solve."""
import numpy as np
import pytest

import oracle
import refs


def _case(n=4, nz=3, levels=2, a_h=1.3, a_z=50.0, graded=True, seed=3, **kw):
    rng = np.random.default_rng(seed)
    dz = 1.05 ** np.arange(nz) if graded else None
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=a_h, a_z=a_z, dz=dz, levels=levels, **kw)
    return rng, c, dz, P, oracle.DG1(P)


@pytest.mark.parametrize("n,nz,graded", [(4, 3, True), (3, 2, False), (2, 4, True)])
def test_operator_equals_quadrature_of_the_form(n, nz, graded):
    """w^T H1 u equals the bilinear form integrated by Gauss quadrature in
    physical coordinates (cell heights s_k, K grad . grad with the cell
    coefficients, jump penalty with density w_f / |f|): pins the mode
    weights, the 4 and 1/s_k scalings, the trace signs and the face weights."""
    rng, c, dz, P, G = _case(n=n, nz=nz, graded=graded, levels=1)
    for _ in range(3):
        U = rng.standard_normal((6, nz, n, n))
        W = rng.standard_normal((6, nz, n, n))
        got = float(np.sum(W * G.apply(U)))
        ref = refs.dg1_quadrature_form(c, 1.3, 50.0, dz, U, W)
        assert abs(got - ref) <= 1e-12 * abs(ref) + 1e-12, (got, ref)


def test_symmetric_positive_definite():
    _, _, _, P, G = _case()
    A = G.dense()
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)
    # every other term is positive semidefinite, so the cell mass s_k (Mv x Mh)
    # bounds the spectrum from below: its smallest eigenvalue is s_k (1/6)(1/3)
    lam = np.linalg.eigvalsh(A)
    s, _ = refs.vertical_metrics(3, 1.05 ** np.arange(3))
    assert lam.min() >= s.min() * (1.0 / 6.0) * (1.0 / 3.0) * (1 - 1e-12)


@pytest.mark.parametrize("graded", [True, False])
def test_galerkin_with_the_embedding_is_the_lowest_order_operator(graded):
    """P^T H1 P = H for the natural embedding P of DG0 in DG1: for cellwise
    constants the DG1 form is the lowest-order operator (assembled here from
    the incidence matrix, independently of the oracle)."""
    _, c, dz, P, G = _case(graded=graded)
    Pm = refs.dg1_embedding(4, 3)
    H0 = refs.incidence_operator(c, 1.3, 50.0, dz)
    got = Pm.T @ G.dense() @ Pm
    assert np.abs(got - H0).max() <= 1e-13 * np.abs(H0).max()


def test_transfers_are_the_embedding_and_its_transpose():
    rng, c, dz, P, G = _case()
    Pm = refs.dg1_embedding(4, 3)
    r = rng.standard_normal((6, 3, 4, 4))
    e = rng.standard_normal((3, 4, 4))
    u = rng.standard_normal((6, 3, 4, 4))
    np.testing.assert_array_equal(G.restrict(r).reshape(-1), Pm.T @ r.reshape(-1))
    np.testing.assert_allclose(G.prolong_add(e, u).reshape(-1), u.reshape(-1) + Pm @ e.reshape(-1), rtol=0,
                               atol=1e-15)
    # the embedded constant 1 is the function 1 at every point of every cell
    one = (Pm @ np.ones(48)).reshape(6, 3, 4, 4)
    for (xi, eta, ze) in [(-1, -1, -1), (0.3, -0.7, 0.2), (1, 1, 1)]:
        assert refs._dg1_eval(one[:, 1, 2, 3], xi, eta, ze)[0] == pytest.approx(1.0, abs=1e-15)


def test_column_block_is_the_in_column_part_of_H1():
    """The oracle's column assembly equals the dense H1 restricted to one
    column, and every coupling lies within the band (5 below, 5 above) in
    the row order r = 6 k + a."""
    _, _, _, P, G = _case()
    A = G.dense()
    n, nz = 4, 3
    for (i, j) in [(0, 0), (3, 1), (2, 3)]:
        idx = [a * nz * n * n + k * n * n + j * n + i for k in range(nz) for a in range(6)]
        ref = A[np.ix_(idx, idx)]
        # the horizontal couplings' self parts belong to the block, their cross parts do not:
        # ref holds only in-column entries of H1, which is exactly the block
        blk = G.column_block(i, j)
        np.testing.assert_allclose(blk, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        r, q = np.nonzero(blk)
        assert np.abs(r - q).max() <= 5


def test_band_lu_factors_and_line_solve():
    """L U rebuilt from the band factors is the column block; the line solve
    equals a dense solve of every column block; a_h = 0 decouples the
    columns, so one undamped sweep is then exact."""
    rng, _, _, P, G = _case()
    F = G.factors()
    nz, m = 3, 18
    for (i, j) in [(0, 0), (1, 3)]:
        f = F[j, i]
        Lm, Um = np.eye(m), np.zeros((m, m))
        for r in range(m):
            for d in range(1, 6):
                if r - d >= 0:
                    Lm[r, r - d] = f[r, 5 - d]
            for d in range(0, 6):
                if r + d < m:
                    Um[r, r + d] = f[r, 5 + d]
        blk = G.column_block(i, j)
        np.testing.assert_allclose(Lm @ Um, blk, rtol=0, atol=1e-13 * np.abs(blk).max())
    r = rng.standard_normal((6, nz, 4, 4))
    x = G.line_solve(r)
    for (i, j) in [(0, 0), (2, 1), (3, 3)]:
        blk = G.column_block(i, j)
        rc = np.array([r[a, k, j, i] for k in range(nz) for a in range(6)])
        xc = np.array([x[a, k, j, i] for k in range(nz) for a in range(6)])
        np.testing.assert_allclose(xc, np.linalg.solve(blk, rc), rtol=1e-13, atol=1e-15)
    _, _, _, P0, G0 = _case(a_h=0.0, omega=1.0)
    b = rng.standard_normal((6, nz, 4, 4))
    u = G0.smooth(None, b)
    ref = np.linalg.solve(G0.dense(), b.reshape(-1))
    np.testing.assert_allclose(u.reshape(-1), ref, rtol=1e-12, atol=1e-14)


def _dense_lowest_order_vcycle(P, m0, n, nz):
    """The lowest-order V-cycle as a dense matrix (columns V e_q; that cycle
    is pinned by its own brute-force test)."""
    V = np.empty((m0, m0))
    e = np.zeros(m0)
    for q in range(m0):
        e[q] = 1.0
        V[:, q] = P.vcycle(e.reshape(nz, n, n)).reshape(-1)
        e[q] = 0.0
    return V


@pytest.mark.parametrize("nu", [(1, 1), (2, 2), (2, 1)])
def test_vcycle_equals_dense_brute_force(nu):
    """The NLO V-cycle: nu_pre block-Jacobi sweeps with the column blocks, the
    residual restricted by P^T, the lowest-order V-cycle, the correction
    embedded by P, nu_post sweeps; all as dense linear algebra."""
    rng, c, dz, P, G = _case(nu=nu, levels=2)
    n, nz = 4, 3
    A = G.dense()
    M, m0 = A.shape[0], n * n * nz
    # block-diagonal H1_z: keep the couplings inside each column
    colid = np.array([(q % (n * n)) for q in range(m0)])
    colid = np.concatenate([colid] * 6)
    Az = np.where(colid[:, None] == colid[None, :], A, 0.0)
    Zinv = np.linalg.inv(Az)
    Pm = refs.dg1_embedding(n, nz)
    V0 = _dense_lowest_order_vcycle(P, m0, n, nz)
    b = rng.standard_normal(M)
    u = np.zeros(M)
    for _ in range(nu[0]):
        u = u + 0.8 * Zinv @ (b - A @ u)
    u = u + Pm @ (V0 @ (Pm.T @ (b - A @ u)))
    for _ in range(nu[1]):
        u = u + 0.8 * Zinv @ (b - A @ u)
    got = G.vcycle(b.reshape(6, nz, n, n)).reshape(-1)
    np.testing.assert_allclose(got, u, rtol=1e-12, atol=1e-13 * np.abs(u).max())


def test_vcycle_symmetric_positive():
    rng, _, _, P, G = _case(n=8, nz=5, levels=3)
    u = rng.standard_normal((6, 5, 8, 8))
    v = rng.standard_normal((6, 5, 8, 8))
    a, b = np.sum(u * G.vcycle(v)), np.sum(v * G.vcycle(u))
    assert abs(a - b) <= 1e-13 * np.sqrt(np.sum(u * G.vcycle(u)) * np.sum(v * G.vcycle(v)))
    assert np.sum(v * G.vcycle(v)) > 0


def test_pcg_matches_dense_solve():
    rng, _, _, P, G = _case()
    b = rng.standard_normal((6, 3, 4, 4))
    x, info = G.pcg(b, rtol=1e-13, maxit=100)
    ref = np.linalg.solve(G.dense(), b.reshape(-1))
    assert info["converged"]
    assert np.linalg.norm(x.reshape(-1) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_nlo_multigrid_beats_single_level():
    """Multigrid with the p step and horizontal coarsening down to 4 x 4
    needs far fewer iterations than the p step alone (one DG0 level smoothed
    twice), Sec. 5.1's comparison on the NLO level."""
    rng = np.random.default_rng(5)
    n, nz = 32, 8
    dz = 1.05 ** np.arange(nz)
    c = refs.random_coeffs(rng, n, nz)
    b = rng.standard_normal((6, nz, n, n))
    its = {}
    for levels in (1, 4):
        P = oracle.Problem(c, a_h=16.0, a_z=1e4, dz=dz, levels=levels, coarse="smooth", n_coarse=2)
        _, info = oracle.DG1(P).pcg(b, rtol=1e-8, maxit=500)
        assert info["converged"]
        its[levels] = info["iterations"]
    assert 2 * its[4] <= its[1], its
