"""Pins for the oracle's operator H and its coarse versions (no GPU).

H is the lumped approximate Helmholtz operator of Sec. 4.2; the pins are
invariants, an independent incidence-matrix assembly, closed-form spectra and
the exact Galerkin relations of the rediscretised coarse operators."""
import numpy as np
import pytest

import oracle
import refs
import synthetic as syn


def make(c, **kw):
    return oracle.Problem(c, **kw)


@pytest.mark.parametrize("graded", [False, True])
def test_constant_vector_gives_mass(graded):
    rng = np.random.default_rng(1)
    n, nz = 8, 6
    dz = 1.05 ** np.arange(nz) if graded else None
    P = make(refs.random_coeffs(rng, n, nz), a_h=1.3, a_z=50.0, dz=dz, levels=3)
    s, _ = refs.vertical_metrics(nz, dz)
    for lev in range(3):
        nl = P.n_at(lev)
        y = P.apply(np.ones((nz, nl, nl)), level=lev)
        expect = np.broadcast_to((4.0 ** lev * s)[:, None, None], y.shape)
        np.testing.assert_allclose(y, expect, rtol=1e-13, atol=0)


@pytest.mark.parametrize("graded", [False, True])
def test_matches_incidence_assembly(graded):
    rng = np.random.default_rng(2)
    n, nz = 4, 5
    dz = 1.05 ** np.arange(nz) if graded else None
    c = refs.random_coeffs(rng, n, nz)
    P = make(c, a_h=0.7, a_z=30.0, dz=dz, levels=1)
    A = P.dense(0)
    R = refs.incidence_operator(c, 0.7, 30.0, dz)
    np.testing.assert_allclose(A, R, rtol=1e-13, atol=1e-12)


def test_symmetric_positive_definite():
    rng = np.random.default_rng(3)
    n, nz = 8, 6
    dz = 1.05 ** np.arange(nz)
    P = make(refs.random_coeffs(rng, n, nz), a_h=1.0, a_z=100.0, dz=dz, levels=2)
    s, _ = refs.vertical_metrics(nz, dz)
    for lev in range(2):
        A = P.dense(lev)
        assert np.abs(A - A.T).max() == 0.0
        ev = np.linalg.eigvalsh(A)
        assert ev.min() >= (4.0 ** lev) * s.min() * (1 - 1e-12)
        np.linalg.cholesky(A)
    x, y = rng.standard_normal((2, nz, n, n))
    lhs = np.vdot(y, P.apply(x))
    rhs = np.vdot(x, P.apply(y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("level", [0, 1])
def test_closed_form_spectrum(level):
    n, nz, a_h, a_z, c0 = 8, 6, 1.0, 100.0, 1.3
    c = np.full((3, nz, n, n), c0)
    P = make(c, a_h=a_h, a_z=a_z, levels=2)
    ev = np.sort(np.linalg.eigvalsh(P.dense(level)))
    nl = n >> level
    ref = np.sort(refs.closed_form_eigs(nl, nz, a_h, a_z, c0, level=level).reshape(-1))
    np.testing.assert_allclose(ev, ref, rtol=1e-12, atol=1e-10)


def test_closed_form_apply_large():
    """H applied to a Fourier x cosine mode is that mode times its eigenvalue."""
    n, nz, a_h, a_z, c0 = 64, 16, 1.0, 1e3, 1.25
    c = np.full((3, nz, n, n), c0)
    P = make(c, a_h=a_h, a_z=a_z, levels=1)
    lx, ly, m = 5, 11, 3
    i = np.arange(n)
    k = np.arange(nz)
    mode = (np.cos(np.pi * m * (k + 0.5) / nz)[:, None, None]
            * np.cos(2 * np.pi * ly * i / n)[None, :, None]
            * np.cos(2 * np.pi * lx * i / n)[None, None, :])
    lam = refs.closed_form_eigs(n, nz, a_h, a_z, c0)[m, ly, lx]
    np.testing.assert_allclose(P.apply(mode), lam * mode, rtol=0, atol=1e-10 * lam)


@pytest.mark.parametrize("graded", [False, True])
def test_coarse_operator_galerkin_relations(graded):
    """Rediscretised coarse operator vs P^T H P: mass and vertical parts equal,
    horizontal part exactly one half (piecewise-constant embedding)."""
    rng = np.random.default_rng(4)
    n, nz = 8, 4
    dz = 1.05 ** np.arange(nz) if graded else None
    c = refs.random_coeffs(rng, n, nz, 0.5, 2.0)
    full = make(c, a_h=1.7, a_z=40.0, dz=dz, levels=3)
    noh = make(c, a_h=0.0, a_z=40.0, dz=dz, levels=3)
    for lev in range(2):
        nl = full.n_at(lev)
        Pm = refs.prolongation(nl, nz)
        A0, A1 = full.dense(lev), full.dense(lev + 1)
        V0, V1 = noh.dense(lev), noh.dense(lev + 1)
        np.testing.assert_allclose(V1, Pm.T @ V0 @ Pm, rtol=1e-13, atol=1e-10)
        np.testing.assert_allclose(A1 - V1, 0.5 * Pm.T @ (A0 - V0) @ Pm, rtol=1e-13, atol=1e-10)


def test_coarse_coefficients_are_face_means():
    rng = np.random.default_rng(5)
    n, nz = 8, 3
    c = refs.random_coeffs(rng, n, nz)
    P = make(c, levels=2)
    c1 = P.coeffs(1)
    I, J = 1, 2
    assert np.allclose(c1[0, :, J, I], 0.5 * (c[0, :, 2 * J, 2 * I + 1] + c[0, :, 2 * J + 1, 2 * I + 1]))
    assert np.allclose(c1[1, :, J, I], 0.5 * (c[1, :, 2 * J + 1, 2 * I] + c[1, :, 2 * J + 1, 2 * I + 1]))
    assert np.allclose(c1[2, :, J, I], c[2, :, 2 * J:2 * J + 2, 2 * I:2 * I + 2].mean(axis=(1, 2)))


def test_workload_generator_shapes():
    w = syn.CONFIGS["fp64_ref_32x32x16"]
    c = w.coefficients()
    assert c.shape == (3, 16, 32, 32) and c.min() >= 1.0 and c.max() < 1.5
    b = w.rhs()
    assert b.shape == (16, 32, 32)
    assert abs(b.mean()) < 0.05 and abs(b.std() - 1) < 0.05
    w4 = syn.CONFIGS["adjoint_256x256x32"]
    faces = w4.fd_faces(32)
    assert len(faces) == 32 and len({tuple(f) for f in faces}) == 32
    assert all(not (f == 2 and k == w4.nz - 1) for f, k, _, _ in faces)


def _graded_grid(nz):
    """An irregular graded column: cell widths s_k (mean 1) and centres z_k."""
    dz = 1.05 ** np.arange(nz) * (1.0 + 0.3 * np.sin(np.arange(nz)))
    s = dz / dz.mean()
    return dz, s, np.cumsum(s) - 0.5 * s


@pytest.mark.parametrize("level", [0, 1, 2])
def test_graded_scaling_exact_for_linear_profiles(level):
    """Finite-volume reading of the graded scaling (Sec. 4.2, Eq. Preconditioner
    on cells of height s_k): the mass is the cell volume 4^l s_k and the vertical
    flux through a face is a_z 4^l (p_{k+1} - p_k) / (distance between the
    centres), which is exact for a linear profile p = z.  So H z = 4^l s_k z_k
    in interior cells, and only the missing bottom / top faces leave a flux
    imbalance of -/+ 4^l a_z.  A wrong mass scaling or a face distance other
    than (s_k + s_{k+1}) / 2 breaks this identity."""
    nz, n, a_h, a_z = 12, 8, 2.5, 40.0
    dz, s, zc = _graded_grid(nz)
    P = oracle.Problem(np.ones((3, nz, n, n)), a_h=a_h, a_z=a_z, dz=dz, levels=3)
    nl = n >> level
    x = np.broadcast_to(zc[:, None, None], (nz, nl, nl)).copy()
    y = P.apply(x, level=level)
    f = 4.0 ** level
    expect = f * s * zc
    expect[0] -= f * a_z
    expect[-1] += f * a_z
    np.testing.assert_allclose(y, np.broadcast_to(expect[:, None, None], y.shape), rtol=0, atol=1e-13 * f * a_z)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_graded_scaling_horizontal_mode(level):
    """Horizontal faces of a graded cell have area proportional to s_k, so a
    horizontal Fourier mode cos(2 pi i / n_l), constant in j and k, is an
    eigenvector with eigenvalue s_k (4^l + 2 a_h (1 - cos(2 pi / n_l))) on every
    level (coefficients 1; the coarse ones are means of ones)."""
    nz, n, a_h, a_z = 12, 8, 2.5, 40.0
    dz, s, _ = _graded_grid(nz)
    P = oracle.Problem(np.ones((3, nz, n, n)), a_h=a_h, a_z=a_z, dz=dz, levels=3)
    nl = n >> level
    th = 2.0 * np.pi / nl
    x = np.broadcast_to(np.cos(th * np.arange(nl))[None, None, :], (nz, nl, nl)).copy()
    y = P.apply(x, level=level)
    lam = s * (4.0 ** level + 2.0 * a_h * (1.0 - np.cos(th)))
    np.testing.assert_allclose(y, lam[:, None, None] * x, rtol=0, atol=1e-13 * lam.max())

