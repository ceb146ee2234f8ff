"""Pins for the adjoint face gradient (no GPU): a tangent-linear directional
derivative on independently assembled dense matrices, central finite
differences with converged solves, and symmetry of the solve operator."""
import numpy as np

import oracle
import refs


def test_tangent_linear_directional_derivative():
    rng = np.random.default_rng(51)
    n, nz, a_h, a_z = 4, 5, 1.0, 200.0
    dz = 1.05 ** np.arange(nz)
    c = np.exp(0.3 * rng.standard_normal((3, nz, n, n)))
    dc = rng.standard_normal(c.shape)
    dc[2, nz - 1] = 0.0
    A = refs.incidence_operator(c, a_h, a_z, dz)
    dA = refs.incidence_operator(c + dc, a_h, a_z, dz) - A      # linear in c
    b, xt = rng.standard_normal((2, nz * n * n))
    x = np.linalg.solve(A, b)
    dx = -np.linalg.solve(A, dA @ x)
    dJ_tl = np.dot(x - xt, dx)                                  # J = 0.5 |x - x_t|^2
    lam = np.linalg.solve(A, x - xt)
    P = oracle.Problem(c, a_h=a_h, a_z=a_z, dz=dz, levels=1)
    g = P.face_gradient(lam.reshape(nz, n, n), x.reshape(nz, n, n))
    assert np.all(g[2, nz - 1] == 0.0)
    dJ_adj = np.sum(g * dc)
    assert abs(dJ_adj - dJ_tl) <= 1e-10 * abs(dJ_tl)


def test_central_finite_differences():
    rng = np.random.default_rng(52)
    n, nz, a_h, a_z, h = 16, 8, 1.0, 1e3, 1e-6
    c = np.exp(0.3 * rng.standard_normal((3, nz, n, n)))
    b, xt = rng.standard_normal((2, nz, n, n))
    kw = dict(a_h=a_h, a_z=a_z, levels=3)
    P = oracle.Problem(c, **kw)
    x, _ = P.pcg(b, rtol=1e-14, maxit=100)
    lam, _ = P.pcg(x - xt, rtol=1e-14, maxit=100)
    g = P.face_gradient(lam, x)
    gmax = np.abs(g).max()
    picks = [(0, 3, 5, 7), (1, 0, 2, 9), (2, 4, 11, 1), (2, 0, 0, 0), (0, 7, 15, 15),
             (1, 6, 8, 3), (2, 6, 3, 12), (0, 2, 9, 4)]
    for f, k, j, i in picks:
        ds = []
        for sgn in (1.0, -1.0):
            cc = c.copy()
            cc[f, k, j, i] += sgn * h
            Q = oracle.Problem(cc, **kw)
            # x_pm = x + d_pm, H_pm d_pm = b - H_pm x: no solver floor in the difference
            d, _ = Q.pcg(b - Q.apply(x), rtol=1e-12, maxit=100)
            ds.append(d)
        # J+ - J- = 0.5 sum (x+ - x-)(x+ + x- - 2 x_t): no difference of large sums
        fd = 0.5 * np.sum((ds[0] - ds[1]) * (2 * (x - xt) + ds[0] + ds[1])) / (2 * h)
        ga = g[f, k, j, i]
        assert abs(fd - ga) <= 1e-6 * gmax + 1e-4 * abs(ga), (f, k, j, i, fd, ga)


def test_solve_operator_symmetric():
    rng = np.random.default_rng(53)
    n, nz = 16, 8
    P = oracle.Problem(np.exp(0.3 * rng.standard_normal((3, nz, n, n))), a_h=1.0, a_z=1e3,
                       levels=3)
    u, v = rng.standard_normal((2, nz, n, n))
    xu, _ = P.pcg(u, rtol=1e-13)
    xv, _ = P.pcg(v, rtol=1e-13)
    assert abs(np.vdot(xu, v) - np.vdot(u, xv)) <= 1e-11 * abs(np.vdot(xu, v))
