"""Pins for the column solve H_z^{-1} and the line smoother (no GPU)."""
import numpy as np
import pytest

import oracle
import refs


@pytest.mark.parametrize("graded", [False, True])
def test_line_solve_equals_column_block_solve(graded):
    rng = np.random.default_rng(11)
    n, nz = 4, 12
    dz = 1.05 ** np.arange(nz) if graded else None
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=1.0, a_z=1e4, dz=dz, levels=2)
    for lev in range(2):
        nl = P.n_at(lev)
        Hz = refs.column_block(P.dense(lev), nl, nz)
        r = rng.standard_normal((nz, nl, nl))
        x = P.line_solve(r, level=lev)
        ref = np.linalg.solve(Hz, r.reshape(-1)).reshape(r.shape)
        np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_no_horizontal_coupling_one_sweep_is_exact():
    """a_h = 0: H = H_z, so one undamped sweep from zero solves H u = b."""
    rng = np.random.default_rng(12)
    n, nz = 4, 8
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=0.0, a_z=300.0, levels=1, omega=1.0)
    b = rng.standard_normal((nz, n, n))
    u = P.smooth(np.zeros_like(b), b)
    ref = np.linalg.solve(refs.incidence_operator(c, 0.0, 300.0), b.reshape(-1)).reshape(b.shape)
    np.testing.assert_allclose(u, ref, rtol=1e-12, atol=1e-14)


def test_smoother_is_damped_block_jacobi():
    rng = np.random.default_rng(13)
    n, nz = 4, 6
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=1.0, a_z=80.0, levels=1, omega=0.8)
    A = refs.incidence_operator(c, 1.0, 80.0)
    Hz = refs.column_block(A, n, nz)
    u, b = rng.standard_normal((2, nz, n, n))
    ref = u.reshape(-1) + 0.8 * np.linalg.solve(Hz, b.reshape(-1) - A @ u.reshape(-1))
    np.testing.assert_allclose(P.smooth(u, b).reshape(-1), ref, rtol=1e-12, atol=1e-13)


def test_float_line_solve_accuracy_graded():
    """Float Thomas on a strongly graded column stays within a loose bound of double."""
    rng = np.random.default_rng(14)
    n, nz = 4, 64
    dz = 1.05 ** np.arange(nz)
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=1.0, a_z=1e4, dz=dz, levels=1)
    r = rng.standard_normal((nz, n, n))
    x64 = P.line_solve(r)
    x32 = P.line_solve(r.astype(np.float32), fp32=True)
    err = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    assert err < 1e-3, err
