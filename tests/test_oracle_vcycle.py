"""Pins for the oracle's V-cycle (no GPU): a dense brute-force run of the same
cycle on independently assembled matrices, symmetry and positivity (needed by
CG), the single-level special case, and grid-independent contraction."""
import numpy as np
import pytest

import oracle
import refs


def dense_vcycle(As, Ps, Hzs, b, nu, omega, coarse, n_coarse):
    """Brute force: the correction-scheme V-cycle with dense matrices."""
    def smooth(l, u, rhs):
        return u + omega * np.linalg.solve(Hzs[l], rhs - As[l] @ u)

    def V(l, rhs):
        if l == len(As) - 1:
            if coarse == "direct":
                return np.linalg.solve(As[l], rhs)
            u = np.zeros_like(rhs)
            for _ in range(n_coarse):
                u = smooth(l, u, rhs)
            return u
        u = np.zeros_like(rhs)
        for _ in range(nu[0]):
            u = smooth(l, u, rhs)
        e = V(l + 1, Ps[l].T @ (rhs - As[l] @ u))
        u = u + Ps[l] @ e
        for _ in range(nu[1]):
            u = smooth(l, u, rhs)
        return u
    return V(0, b)


def hierarchy(c, a_h, a_z, dz, levels):
    """Dense level matrices: level 0 by incidence assembly, coarse levels from the
    Galerkin relations (mass/vertical exact, horizontal halved) pinned elsewhere."""
    _, nz, n, _ = c.shape
    A0 = refs.incidence_operator(c, a_h, a_z, dz)
    V0 = refs.incidence_operator(c, 0.0, a_z, dz)
    As, Ps, Hzs = [A0], [], [refs.column_block(A0, n, nz)]
    A, Vm, nl = A0, V0, n
    for _ in range(1, levels):
        Pm = refs.prolongation(nl, nz)
        Vc = Pm.T @ Vm @ Pm
        A = Vc + 0.5 * Pm.T @ (A - Vm) @ Pm
        Vm, nl = Vc, nl // 2
        Ps.append(Pm)
        As.append(A)
        Hzs.append(refs.column_block(A, nl, nz))
    return As, Ps, Hzs


@pytest.mark.parametrize("coarse", ["direct", "smooth"])
@pytest.mark.parametrize("nu", [(2, 2), (1, 1), (1, 2)])
def test_matches_dense_brute_force(coarse, nu):
    rng = np.random.default_rng(31)
    n, nz, levels = 8, 4, 3
    dz = 1.05 ** np.arange(nz)
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=1.0, a_z=100.0, dz=dz, levels=levels, nu=nu, coarse=coarse)
    As, Ps, Hzs = hierarchy(c, 1.0, 100.0, dz, levels)
    b = rng.standard_normal((nz, n, n))
    ref = dense_vcycle(As, Ps, Hzs, b.reshape(-1), nu, 0.8, coarse, 2)
    np.testing.assert_allclose(P.vcycle(b).reshape(-1), ref, rtol=1e-11, atol=1e-13)


def test_single_level_is_two_line_jacobi_sweeps():
    """One level with two coarse sweeps = the single-level method of Sec. 5."""
    rng = np.random.default_rng(32)
    n, nz = 4, 6
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=1.0, a_z=100.0, levels=1, coarse="smooth", n_coarse=2)
    A = refs.incidence_operator(c, 1.0, 100.0)
    Hz = refs.column_block(A, n, nz)
    b = rng.standard_normal((nz, n, n)).reshape(-1)
    u = 0.8 * np.linalg.solve(Hz, b)
    u = u + 0.8 * np.linalg.solve(Hz, b - A @ u)
    np.testing.assert_allclose(P.vcycle(b.reshape(nz, n, n)).reshape(-1), u, rtol=1e-12)


@pytest.mark.parametrize("coarse", ["direct", "smooth"])
def test_symmetric_positive(coarse):
    rng = np.random.default_rng(33)
    n, nz = 16, 8
    dz = 1.05 ** np.arange(nz)
    P = oracle.Problem(refs.random_coeffs(rng, n, nz), a_h=1.0, a_z=1e4, dz=dz, levels=3,
                       coarse=coarse)
    for _ in range(3):
        u, v = rng.standard_normal((2, nz, n, n))
        a, b = np.vdot(u, P.vcycle(v)), np.vdot(v, P.vcycle(u))
        assert abs(a - b) <= 1e-13 * max(abs(a), np.linalg.norm(u) * np.linalg.norm(P.vcycle(u)))
        assert np.vdot(v, P.vcycle(v)) > 0


def contraction(P, rng, iters=25):
    """A-norm contraction of I - V H by power iteration."""
    shape = (P.nz, P.n, P.n)
    e = rng.standard_normal(shape)
    rho = 0.0
    for _ in range(iters):
        He = P.apply(e)
        norm = np.sqrt(np.vdot(e, He))
        e = e / norm
        e = e - P.vcycle(P.apply(e))
        rho = np.sqrt(np.vdot(e, P.apply(e)))
    return rho


def test_grid_independent_contraction():
    """Robustness claim of Sec. 4.2.1 / Sec. 5.2: contraction flat in the grid size."""
    rng = np.random.default_rng(34)
    nz = 16
    dz = 1.05 ** np.arange(nz)
    rhos = []
    for n, levels in [(32, 2), (64, 3), (128, 4)]:
        c = refs.random_coeffs(rng, n, nz)
        P = oracle.Problem(c, a_h=1.0, a_z=1e4, dz=dz, levels=levels)
        rhos.append(contraction(P, rng))
    assert max(rhos) < 0.3, rhos
    assert abs(rhos[1] - rhos[2]) <= 0.02, rhos
