"""Pins for the oracle's velocity-pressure system (no GPU): the block structure
of Eq. PressureVelocitySystem, the diagonal lumping that turns its Schur
complement into the pressure operator H, the Raviart-Thomas mass in the
uniform limit, the Schur-complement factorisation (Eq. SchurComplement), and
the flexible GMRES against dense solves and the paper's single-level claim."""
import numpy as np
import pytest

import oracle
import refs
import synthetic as syn


def real_dofs(n, nz):
    """Logical (4, nz, n, n) positions of the real unknowns: every E and N face,
    U faces below the top cell, every cell."""
    mask = np.ones((4, nz, n, n), dtype=bool)
    mask[2, nz - 1] = False
    return np.flatnonzero(mask.reshape(-1))


def densify(fn, n, nz):
    idx = real_dofs(n, nz)
    A = np.zeros((idx.size, idx.size))
    e = np.zeros(4 * nz * n * n)
    for col, q in enumerate(idx):
        e[:] = 0.0
        e[q] = 1.0
        A[:, col] = fn(e.reshape(4, nz, n, n)).reshape(-1)[idx]
    return A, idx


def small_problem(levels=1, coarse="smooth", n=4, nz=3, graded=True, seed=61):
    rng = np.random.default_rng(seed)
    c = refs.random_coeffs(rng, n, nz)
    dz = 1.05 ** np.arange(nz) if graded else None
    P = oracle.Problem(c, a_h=2.0, a_z=50.0, dz=dz, levels=levels, coarse=coarse)
    return P, c, dz


def blocks(A, n, nz):
    nu = 3 * n * n * nz - n * n  # real face unknowns
    return A[:nu, :nu], A[:nu, nu:], A[nu:, :nu], A[nu:, nu:]


def test_top_slot_is_inert():
    P, _, _ = small_problem()
    n, nz = 4, 3
    x = np.random.default_rng(1).standard_normal((4, nz, n, n))
    y = P.mixed_apply(x)
    assert np.all(y[2, -1] == 0.0)
    x2 = x.copy()
    x2[2, -1] = 1e6
    assert np.array_equal(P.mixed_apply(x2), y)


@pytest.mark.parametrize("graded", [False, True])
def test_lumped_schur_complement_is_the_pressure_operator(graded):
    """Block structure A = [M, -D^T; D, M3], and M3 + D diag(M)^{-1} D^T = H."""
    n, nz = 4, 3
    P, c, dz = small_problem(graded=graded)
    A, _ = densify(P.mixed_apply, n, nz)
    Muu, Aup, Apu, App = blocks(A, n, nz)
    np.testing.assert_array_equal(Apu, -Aup.T)
    assert np.allclose(App, np.diag(np.diag(App))) and np.all(np.diag(App) > 0)
    H = App + Apu @ np.diag(1.0 / np.diag(Muu)) @ (-Aup)
    ref = refs.incidence_operator(c, 2.0, 50.0, dz)
    np.testing.assert_allclose(H, ref, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(H, P.dense(0), rtol=1e-13, atol=1e-12)


def test_velocity_mass_spd_and_normalised():
    n, nz = 4, 3
    P, _, _ = small_problem()
    A, _ = densify(P.mixed_apply, n, nz)
    Muu = blocks(A, n, nz)[0]
    np.testing.assert_allclose(Muu, Muu.T, rtol=1e-14, atol=0)
    d = np.sqrt(np.diag(Muu))
    T = Muu / np.outer(d, d)
    ev = np.linalg.eigvalsh(T)
    assert np.allclose(np.diag(T), 1.0) and ev.min() >= 0.5 - 1e-12 and ev.max() <= 1.5 + 1e-12, ev


def rt0_mass_1d(ncells, periodic):
    """Lowest-order Raviart-Thomas mass on unit cells in 1-D, assembled from
    the element matrix [1/3 1/6; 1/6 1/3]; without periodicity the two
    boundary faces are removed (zero normal flux)."""
    nf = ncells if periodic else ncells + 1
    Mf = np.zeros((nf, nf))
    for cell in range(ncells):
        a, b = cell, (cell + 1) % nf if periodic else cell + 1
        Mf[np.ix_([a, b], [a, b])] += np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])
    return Mf if periodic else Mf[1:-1, 1:-1]


def test_uniform_limit_is_raviart_thomas_mass():
    """Uniform coefficients and spacing: each directional block of M is the
    1-D lowest-order Raviart-Thomas mass (scaled by 3/(2 w))."""
    n, nz = 4, 5
    c = np.full((3, nz, n, n), 1.0)
    P = oracle.Problem(c, a_h=1.0, a_z=1.0, levels=1)
    x = np.zeros((4, nz, n, n))
    # E faces along one row: (i, j=1, k=2)
    row = np.zeros((n, n))
    for i in range(n):
        x[:] = 0
        x[0, 2, 1, i] = 1.0
        row[:, i] = P.mixed_apply(x)[0, 2, 1, :]
    np.testing.assert_allclose(row * 2.0 / 3.0, rt0_mass_1d(n, True), rtol=1e-14)
    # U faces along one column (i=1, j=2): nz - 1 interior faces
    col = np.zeros((nz - 1, nz - 1))
    for k in range(nz - 1):
        x[:] = 0
        x[2, k, 2, 1] = 1.0
        col[:, k] = P.mixed_apply(x)[2, : nz - 1, 2, 1]
    np.testing.assert_allclose(col * 2.0 / 3.0, rt0_mass_1d(nz, False), rtol=1e-14)


def test_schur_factorisation_is_the_inverse():
    """Eq. SchurComplement with exact inverses reproduces A^{-1} (pure algebra on
    the oracle's blocks)."""
    n, nz = 4, 3
    P, _, _ = small_problem()
    A, _ = densify(P.mixed_apply, n, nz)
    Muu, Aup, Apu, App = blocks(A, n, nz)
    Dt, D = -Aup, Apu
    Mi = np.linalg.inv(Muu)
    Hi = np.linalg.inv(App + D @ Mi @ Dt)
    nu, npr = Muu.shape[0], App.shape[0]
    L = np.block([[np.eye(nu), np.zeros((nu, npr))], [-D @ Mi, np.eye(npr)]])
    Dg = np.block([[Mi, np.zeros((nu, npr))], [np.zeros((npr, nu)), Hi]])
    U = np.block([[np.eye(nu), Mi @ Dt], [np.zeros((npr, nu)), np.eye(npr)]])
    np.testing.assert_allclose(U @ Dg @ L @ A, np.eye(nu + npr), atol=1e-10)


@pytest.mark.parametrize("levels,coarse", [(1, "direct"), (2, "smooth")])
def test_preconditioner_is_the_lumped_factorisation(levels, coarse):
    """The oracle's preconditioner equals Eq. SchurComplement with diag(M)^{-1}
    for M^{-1} and the (dense) V-cycle for H^{-1}."""
    n, nz = 4, 3
    P, _, _ = small_problem(levels=levels, coarse=coarse)
    A, idx = densify(P.mixed_apply, n, nz)
    Muu, Aup, Apu, _ = blocks(A, n, nz)
    Dt, D = -Aup, Apu
    W = np.diag(1.0 / np.diag(Muu))
    m = n * n * nz
    V = np.zeros((m, m))
    for q in range(m):
        e = np.zeros(m)
        e[q] = 1.0
        V[:, q] = P.vcycle(e.reshape(nz, n, n)).reshape(-1)
    nu = Muu.shape[0]
    L = np.block([[np.eye(nu), np.zeros((nu, m))], [-D @ W, np.eye(m)]])
    Dg = np.block([[W, np.zeros((nu, m))], [np.zeros((m, nu)), V]])
    U = np.block([[np.eye(nu), W @ Dt], [np.zeros((m, nu)), np.eye(m)]])
    Pd, _ = densify(P.mixed_precondition, n, nz)
    np.testing.assert_allclose(Pd, U @ Dg @ L, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("restart", [30, 3])
def test_fgmres_matches_dense_solve(restart):
    n, nz = 4, 3
    P, _, _ = small_problem(levels=2)
    A, idx = densify(P.mixed_apply, n, nz)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((4, nz, n, n))
    b[2, -1] = 0.0
    x, info = P.mixed_fgmres(b, rtol=1e-13, restart=restart, maxit=200)
    ref = np.linalg.solve(A, b.reshape(-1)[idx])
    assert info["converged"], info
    err = np.linalg.norm(x.reshape(-1)[idx] - ref) / np.linalg.norm(ref)
    assert err < 1e-11, err
    assert np.all(x[2, -1] == 0.0)
    assert np.all(np.diff(info["history"][: restart + 1]) <= 1e-15), info["history"]


def test_multigrid_beats_single_level_on_the_mixed_system():
    """Sec. 5.1: with the multigrid preconditioner the outer GMRES converges in
    about ten iterations, the single-level method needs several times more."""
    w = syn.Workload("mixed64x64x32", 64, 32, 3, 16.0, 1e4, True, "uniform")
    c = w.coefficients()
    b = w.mixed_rhs()
    mg = oracle.Problem(c, a_h=w.a_h, a_z=w.a_z, dz=w.dz(), levels=3)
    single = oracle.Problem(c, a_h=w.a_h, a_z=w.a_z, dz=w.dz(), levels=1)
    _, i_mg = mg.mixed_fgmres(b, rtol=1e-5)
    _, i_1 = single.mixed_fgmres(b, rtol=1e-5)
    assert i_mg["converged"] and i_1["converged"]
    assert i_mg["true_rel_residual"] <= 1.01e-5
    assert i_mg["iterations"] <= 12, i_mg["iterations"]
    assert i_1["iterations"] >= 3 * i_mg["iterations"], (i_mg["iterations"], i_1["iterations"])
    _, i_32 = mg.mixed_fgmres(b, rtol=1e-5, fp32=True)
    assert i_32["converged"] and abs(i_32["iterations"] - i_mg["iterations"]) <= 1
