"""Pins for restriction and prolongation (natural embedding, R = P^T)."""
import numpy as np

import oracle
import refs


def _problem(n=8, nz=3, levels=3):
    rng = np.random.default_rng(21)
    return oracle.Problem(refs.random_coeffs(rng, n, nz), levels=levels), rng


def test_restriction_is_adjoint_of_prolongation():
    P, rng = _problem()
    for lev in range(2):
        nf, nc = P.n_at(lev), P.n_at(lev + 1)
        r = rng.standard_normal((P.nz, nf, nf))
        e = rng.standard_normal((P.nz, nc, nc))
        lhs = np.vdot(P.restrict(r, lev), e)
        rhs = np.vdot(r, P.prolong_add(e, np.zeros_like(r), lev))
        assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def test_transfer_of_constants():
    P, _ = _problem()
    nf, nc = P.n_at(0), P.n_at(1)
    assert np.array_equal(P.prolong_add(np.ones((P.nz, nc, nc)), np.zeros((P.nz, nf, nf))),
                          np.ones((P.nz, nf, nf)))
    assert np.array_equal(P.restrict(np.ones((P.nz, nf, nf))), 4 * np.ones((P.nz, nc, nc)))


def test_matches_dense_embedding():
    P, rng = _problem(n=4, nz=2, levels=2)
    Pm = refs.prolongation(4, 2)
    r = rng.standard_normal((2, 4, 4))
    np.testing.assert_allclose(P.restrict(r).reshape(-1), Pm.T @ r.reshape(-1), rtol=1e-15)
    e = rng.standard_normal((2, 2, 2))
    np.testing.assert_allclose(P.prolong_add(e, np.zeros((2, 4, 4))).reshape(-1),
                               Pm @ e.reshape(-1), rtol=1e-15)
