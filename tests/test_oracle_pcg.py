"""Pins for the oracle's preconditioned CG (no GPU): dense direct solves on tiny
grids, the Fourier/cosine closed form for uniform coefficients, the
mixed-precision form's residual, and the paper's qualitative claims."""
import numpy as np
import pytest

import oracle
import refs
import synthetic as syn


@pytest.mark.parametrize("coarse", ["direct", "smooth"])
@pytest.mark.parametrize("mixed", [False, True])
def test_matches_dense_solve(coarse, mixed):
    rng = np.random.default_rng(41)
    n, nz = 8, 6
    dz = 1.05 ** np.arange(nz)
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=1.0, a_z=100.0, dz=dz, levels=2, coarse=coarse)
    b = rng.standard_normal((nz, n, n))
    x, info = P.pcg(b, rtol=1e-14, maxit=60, mixed=mixed, flexible=mixed)
    ref = np.linalg.solve(refs.incidence_operator(c, 1.0, 100.0, dz), b.reshape(-1))
    err = np.linalg.norm(x.reshape(-1) - ref) / np.linalg.norm(ref)
    assert info["converged"] and err < 1e-12, (info, err)


def test_matches_closed_form_uniform():
    n, nz, a_h, a_z, c0 = 64, 16, 1.0, 1e3, 1.2
    c = np.full((3, nz, n, n), c0)
    P = oracle.Problem(c, a_h=a_h, a_z=a_z, levels=3)
    b = syn.normal(syn.SEED, syn.STREAM_TEST, n * n * nz).reshape(nz, n, n)
    x, info = P.pcg(b, rtol=1e-13, maxit=60)
    ref = refs.closed_form_solve(b, a_h, a_z, c0)
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert info["converged"] and err < 1e-11, (info, err)


def test_reference_config_converges_and_beats_single_level():
    w = syn.CONFIGS["fp64_ref_32x32x16"]
    P = oracle.problem_for(w)
    b = w.rhs()
    x, info = P.pcg(b, rtol=w.rtol, maxit=100)
    assert info["converged"] and info["true_rel_residual"] <= 1.01e-8
    hist = info["history"]
    assert np.all(np.diff(hist) < 0)
    single = oracle.problem_for(w, levels=1, coarse="smooth")
    _, info1 = single.pcg(b, rtol=w.rtol, maxit=200)
    # Sec. 5.1: the single-level method needs several times more iterations
    assert info1["iterations"] >= 2 * info["iterations"], (info["iterations"], info1["iterations"])


@pytest.mark.parametrize("flexible", [False, True])
def test_mixed_precision_reaches_fp64_accuracy(flexible):
    w = syn.scaled(syn.CONFIGS["fp64_512x512x64"], 64, nz=32, levels=3)
    P = oracle.problem_for(w)
    b = w.rhs()
    x_ref, _ = P.pcg(b, rtol=1e-13, maxit=100)
    x64, i64 = P.pcg(b, rtol=1e-8, maxit=100)
    x32, i32 = P.pcg(b, rtol=1e-8, maxit=100, mixed=True, flexible=flexible)
    assert i32["converged"] and i32["true_rel_residual"] <= 1.05e-8
    e64 = np.linalg.norm(x64 - x_ref) / np.linalg.norm(x_ref)
    e32 = np.linalg.norm(x32 - x_ref) / np.linalg.norm(x_ref)
    assert e32 < 1e-7 and e64 < 1e-7, (e32, e64)
    assert abs(i32["iterations"] - i64["iterations"]) <= 1


def test_nonzero_initial_guess_and_zero_rhs():
    rng = np.random.default_rng(42)
    n, nz = 8, 4
    c = refs.random_coeffs(rng, n, nz)
    P = oracle.Problem(c, a_h=1.0, a_z=10.0, levels=2)
    b = rng.standard_normal((nz, n, n))
    x, _ = P.pcg(b, rtol=1e-12)
    x2, info = P.pcg(b, rtol=1e-12, x0=x)
    assert info["iterations"] <= 1
    z, infoz = P.pcg(np.zeros_like(b), rtol=1e-8)
    assert infoz["converged"] and infoz["iterations"] == 0 and not z.any()


def _iterations(c, b, dz, a_h, **kw):
    P = oracle.Problem(c, a_h=a_h, a_z=1e4, dz=dz, **kw)
    _, info = P.pcg(b, rtol=1e-8, maxit=400)
    assert info["converged"]
    return info["iterations"]


def test_courant_number_robustness():
    """Sec. 5.2 (robustness in the Courant number, a_h = (nu_CFL / 2)^2): the
    single-level method degrades sharply as nu_CFL grows; multigrid with a
    fixed coarsest grid (16 x 16, two sweeps) degrades mildly; a stronger
    coarse solve (more sweeps, or coarsening to one column with an exact
    solve) removes most of the growth."""
    n, nz = 64, 16
    w = syn.Workload("cfl64x64x16", n, nz, 3, 1.0, 1e4, True, "uniform")
    c, b, dz = w.coefficients(), w.rhs(), w.dz()
    it = {}
    for nu in (2, 8, 64):
        a_h = (nu / 2.0) ** 2
        it[nu] = dict(
            single=_iterations(c, b, dz, a_h, levels=1, coarse="smooth", n_coarse=2),
            mg=_iterations(c, b, dz, a_h, levels=3, coarse="smooth", n_coarse=2),
            mg16=_iterations(c, b, dz, a_h, levels=3, coarse="smooth", n_coarse=16),
            deep=_iterations(c, b, dz, a_h, levels=7, coarse="direct"))
    assert it[64]["single"] >= 4 * it[2]["single"], it
    for nu in (8, 64):
        assert 3 * it[nu]["mg"] <= it[nu]["single"], it
        assert it[nu]["mg16"] < it[nu]["mg"], it
    assert it[64]["mg16"] <= 0.6 * it[64]["mg"], it
    assert it[64]["deep"] - it[2]["deep"] <= 2, it


def test_resolution_independence_fixed_courant():
    """Sec. 5.2: at fixed nu_CFL = 8 the multigrid iteration count does not grow
    with the horizontal resolution (coarsest grid 16 x 16 throughout)."""
    its = []
    for n, levels in [(32, 2), (64, 3), (128, 4)]:
        w = syn.Workload(f"res{n}", n, 16, levels, 16.0, 1e4, True, "uniform")
        its.append(_iterations(w.coefficients(), w.rhs(), w.dz(), 16.0, levels=levels))
    assert its[2] <= its[1] <= its[0], its


def _variable_preconditioner_case():
    rng = np.random.default_rng(7)
    n, nz = 16, 8
    dz = 1.05 ** np.arange(nz)
    c = refs.random_coeffs(rng, n, nz)
    A = refs.incidence_operator(c, 1.0, 1e3, dz)   # assembled independently of the oracle
    P = oracle.Problem(c, a_h=1.0, a_z=1e3, dz=dz, levels=3)
    b = rng.standard_normal((nz, n, n))
    return A, P, b


def _conjugacy(A, info):
    """Largest H-cosine between consecutive directions, and largest cosine
    between each direction and the residual after its update."""
    D = info["directions"].reshape(info["iterations"], -1)
    R = info["residuals"].reshape(info["iterations"], -1)
    conj = max(abs(D[k + 1] @ A @ D[k]) / np.sqrt((D[k + 1] @ A @ D[k + 1]) * (D[k] @ A @ D[k]))
               for k in range(len(D) - 1))
    orth = max(abs(R[k] @ D[k]) / (np.linalg.norm(R[k]) * np.linalg.norm(D[k])) for k in range(len(D)))
    return conj, orth


@pytest.mark.parametrize("omega_alt", [0.3, 0.5])
def test_flexible_beta_keeps_local_conjugacy(omega_alt):
    """Flexible CG with one stored direction (the reading of Sec. 5's call
    for a flexible Krylov method): whatever the preconditioner does between
    iterations, each new direction is H-conjugate to the previous one and the
    residual after an update is orthogonal to the direction just used.  With
    every other V-cycle damped differently (an SPD preconditioner that
    changes between iterations) the standard beta loses the conjugacy by
    O(1) and needs more iterations, so this check tells the two apart; a
    flipped or dropped term in the flexible beta fails it."""
    A, P, b = _variable_preconditioner_case()
    _, fx = P.pcg(b, rtol=1e-10, maxit=80, flexible=True, omega_alt=omega_alt, trace=True)
    _, st = P.pcg(b, rtol=1e-10, maxit=80, flexible=False, omega_alt=omega_alt, trace=True)
    assert fx["converged"] and st["converged"]
    conj_f, orth_f = _conjugacy(A, fx)
    conj_s, orth_s = _conjugacy(A, st)
    assert conj_f <= 1e-12 and orth_f <= 1e-12, (conj_f, orth_f)
    assert conj_s >= 1e-2, conj_s            # the variable preconditioner really matters
    assert orth_s <= 1e-12, orth_s           # (the residual property comes from alpha)
    assert fx["iterations"] < st["iterations"], (fx["iterations"], st["iterations"])


def test_flexible_equals_standard_for_a_fixed_preconditioner():
    """With a fixed SPD preconditioner both betas agree in exact arithmetic:
    same iterations, iterates equal to rounding."""
    A, P, b = _variable_preconditioner_case()
    xf, fx = P.pcg(b, rtol=1e-10, maxit=80, flexible=True, trace=True)
    xs, st = P.pcg(b, rtol=1e-10, maxit=80, flexible=False, trace=True)
    assert fx["iterations"] == st["iterations"]
    assert np.linalg.norm(xf - xs) / np.linalg.norm(xs) <= 1e-10
    conj, orth = _conjugacy(A, fx)
    assert conj <= 1e-12 and orth <= 1e-12
