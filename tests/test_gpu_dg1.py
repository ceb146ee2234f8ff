"""The next-to-lowest-order (DG1) level on the GPU against the oracle: band
factors of the column blocks (Sec. 4.3.1), the operator, the line solve,
the damped sweeps, the p-transfers to the lowest-order level (Sec. 4.2.1),
the NLO V-cycle and CG, on grids that span several 64-column tiles with a
ragged tail in k and on planes that are not a multiple of 64 (untiled
storage)."""
import numpy as np
import pytest

import oracle
import paper_1605_00492_amd as tp
from gpu_util import device, host, max_rel, rel_err, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# name: n, nz, levels, a_z, graded, coarse
CASES = {
    "2x2x2_single_level": (2, 2, 1, 30.0, False, "direct"),
    "4x4x3_graded": (4, 3, 2, 50.0, True, "direct"),
    "12x12x5_untiled": (12, 5, 3, 1e3, True, "smooth"),
    "32x32x16": (32, 16, 3, 100.0, False, "direct"),
    "64x64x37_graded": (64, 37, 3, 1e4, True, "smooth"),
    "96x96x24_ragged": (96, 24, 4, 1e3, True, "smooth"),
}


def _coeffs(n, nz, seed):
    rng = np.random.default_rng(seed)
    c = 1.0 + 0.5 * rng.random((3, nz, n, n))
    c[2, nz - 1] = 0.0
    return c


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    dev = device()
    n, nz, levels, a_z, graded, coarse = CASES[request.param]
    print(f"[gpu] DG1 case {request.param}", flush=True)
    c = _coeffs(n, nz, 7 + n + nz)
    dz = 1.05 ** np.arange(nz) if graded else None
    kw = dict(a_h=1.0, a_z=a_z, dz=dz, levels=levels, nu=(2, 2), omega=0.8, coarse=coarse, n_coarse=2)
    P = oracle.Problem(c, **kw)
    G = oracle.DG1(P)
    ct = to_dev(c)
    H = {p: tp.Hierarchy(ct, precision=p, **kw) for p in ("fp64", "mixed")}
    D = {p: tp.binding.DG1Level(H[p]) for p in H}
    rng = np.random.default_rng(100 + n)
    yield dict(name=request.param, n=n, nz=nz, P=P, G=G, H=H, D=D, rng=rng, dev=dev)
    for d in D.values():
        d.close()
    for h in H.values():
        h.close()


def _rand(case):
    return case["rng"].standard_normal((6, case["nz"], case["n"], case["n"]))


def test_factors_match_oracle(case):
    got = host(case["D"]["fp64"].factors())
    ref = case["G"].factors()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"[gpu] {case['name']} factors: {err:.2e}", flush=True)
    assert err <= 1e-13, err


def test_apply_matches_oracle(case):
    x = _rand(case)
    got = host(case["D"]["fp64"].apply(to_dev(x)))
    err = max_rel(got, case["G"].apply(x))
    assert err <= 1e-13, err


def test_line_solve_matches_oracle(case):
    r = _rand(case)
    got = host(case["D"]["fp64"].line_solve(to_dev(r)))
    err = rel_err(got, case["G"].line_solve(r))
    print(f"[gpu] {case['name']} line solve: {err:.2e}", flush=True)
    assert err <= 1e-12, err


@pytest.mark.parametrize("zero", [True, False])
def test_smooth_matches_oracle(case, zero):
    b, u = _rand(case), _rand(case)
    D = case["D"]["fp64"]
    got = host(D.smooth(to_dev(b), None if zero else to_dev(u)))
    ref = case["G"].smooth(None if zero else u, b)
    err = rel_err(got, ref)
    assert err <= 1e-12, err


def test_p_transfers_match_oracle(case):
    b, u = _rand(case), _rand(case)
    D, G = case["D"]["fp64"], case["G"]
    got = host(D.residual_restrict(to_dev(u), to_dev(b)))
    ref = G.restrict(b - G.apply(u))
    assert rel_err(got, ref) <= 1e-13
    e0 = case["rng"].standard_normal((case["nz"], case["n"], case["n"]))
    got = host(D.prolong_add(to_dev(e0), to_dev(u)))
    assert np.array_equal(got, G.prolong_add(e0, u))


def test_vcycle_matches_oracle(case):
    b = _rand(case)
    got = host(case["D"]["fp64"].vcycle(to_dev(b)))
    err = rel_err(got, case["G"].vcycle(b))
    print(f"[gpu] {case['name']} V-cycle: {err:.2e}", flush=True)
    assert err <= 1e-11, err


def test_fp64_solve_matches_oracle_iterate(case):
    b = _rand(case)
    x_or, info_or = case["G"].pcg(b, rtol=1e-8, maxit=100)
    it = info_or["iterations"]
    x, info = case["D"]["fp64"].solve(to_dev(b), rtol=1e-8, maxit=it, flexible=False, history=True)
    err = rel_err(host(x), x_or)
    print(f"[gpu] {case['name']} DG1 FP64 solve: {info['iterations']} it (oracle {it}), error {err:.2e}", flush=True)
    assert info["converged"] and info["iterations"] == it and err <= 1e-10, (info, err)
    np.testing.assert_allclose(info["history"], info_or["history"], rtol=1e-5)
    assert info["true_rel_residual"] <= 1.05e-8


def _stored_fp32(ref):
    """The oracle's band factors as a mixed hierarchy stores them: every entry
    rounded to FP32, the diagonal entry as the FP32 value of 1 / U(r, r)."""
    f = ref.astype(np.float32).astype(np.float64)
    with np.errstate(divide="ignore"):
        f[..., 5] = (1.0 / ref[..., 5]).astype(np.float32).astype(np.float64)
    return f


def _band_solve(F, r, n, nz):
    """x = (L U)^{-1} r column by column with stored factors F ([j, i, row,
    entry], entry 5 the reciprocal of U(row, row)): forward and back
    substitution in FP64, r and x in the (6, nz, n, n) layout."""
    m = 6 * nz
    rc = oracle.dg1_to_columns(r).reshape(n, n, m)
    y = np.zeros_like(rc)
    for row in range(m):
        acc = rc[..., row].copy()
        for d in range(1, 6):
            if row - d >= 0:
                acc -= F[..., row, 5 - d] * y[..., row - d]
        y[..., row] = acc
    x = np.zeros_like(rc)
    for row in range(m - 1, -1, -1):
        acc = y[..., row].copy()
        for d in range(1, 6):
            if row + d < m:
                acc -= F[..., row, 5 + d] * x[..., row + d]
        x[..., row] = acc * F[..., row, 5]
    return oracle.dg1_from_columns(x.reshape(-1), n, nz)


def test_mixed_factors_are_fp32_roundings(case):
    """A mixed hierarchy stores the FP64 factors rounded to FP32: equal to the
    oracle's factors rounded the same way (both FP64 factorisations agree to
    1e-13, so at most a value sitting on a rounding boundary could differ, by
    one FP32 unit in the last place)."""
    got = host(case["D"]["mixed"].factors())
    stored = _stored_fp32(case["G"].factors())
    expect = stored.copy()
    nz_ = stored[..., 5] != 0
    expect[..., 5][nz_] = 1.0 / stored[..., 5][nz_]
    scale = np.maximum(np.abs(expect), np.finfo(np.float64).tiny)
    err = np.abs(got - expect) / scale
    exact = np.count_nonzero(got == expect)
    print(f"[gpu] {case['name']} mixed factors: {exact} of {got.size} equal, max rel diff {err.max():.2e}",
          flush=True)
    assert err.max() <= 2.0 ** -23, err.max()


def test_mixed_line_solve_and_sweeps_use_the_fp32_factors(case):
    """The mixed level's line solve and sweeps are the FP64 substitutions
    with the FP32-rounded factors (emulated here from the oracle's factors and
    operator); against the FP64 oracle they differ by the factor rounding."""
    n, nz = case["n"], case["nz"]
    ref = case["G"].factors()
    F = _stored_fp32(ref)
    D, G = case["D"]["mixed"], case["G"]
    omega = 0.8
    r, u, b = _rand(case), _rand(case), _rand(case)
    # the emulation itself: with the FP64 factors it is the oracle's line solve
    F64 = ref.copy()
    nzd = ref[..., 5] != 0
    F64[..., 5][nzd] = 1.0 / ref[..., 5][nzd]
    assert rel_err(_band_solve(F64, r, n, nz), G.line_solve(r)) <= 1e-12
    got = host(D.line_solve(to_dev(r)))
    emu = _band_solve(F, r, n, nz)
    err, err64 = rel_err(got, emu), rel_err(got, G.line_solve(r))
    print(f"[gpu] {case['name']} mixed line solve: {err:.2e} vs FP32-factor emulation, "
          f"{err64:.2e} vs FP64 factors", flush=True)
    assert err <= 1e-10, err
    got0 = host(D.smooth(to_dev(b), None))
    err0 = rel_err(got0, omega * _band_solve(F, b, n, nz))
    got1 = host(D.smooth(to_dev(b), to_dev(u)))
    err1 = rel_err(got1, u + omega * _band_solve(F, b - G.apply(u), n, nz))
    print(f"[gpu] {case['name']} mixed sweeps: zero {err0:.2e}, general {err1:.2e}", flush=True)
    assert err0 <= 1e-10 and err1 <= 1e-10, (err0, err1)


def test_mixed_solve_matches_oracle(case):
    """FP32 lowest-order V-cycle inside the FP64 DG1 sweeps and CG
    (flexible beta): the solution to 1e-8 against the oracle's FP64 one."""
    b = _rand(case)
    x_or, info_or = case["G"].pcg(b, rtol=1e-8, maxit=100)
    x, info = case["D"]["mixed"].solve(to_dev(b), rtol=1e-8, maxit=100)
    err = rel_err(host(x), x_or)
    print(f"[gpu] {case['name']} DG1 mixed solve: {info['iterations']} it (oracle FP64 {info_or['iterations']}), "
          f"true rel residual {info['true_rel_residual']:.2e}, error vs oracle {err:.2e}", flush=True)
    assert info["converged"] and info["true_rel_residual"] <= 1.05e-8
    assert err <= 1e-8, err


def test_dg1_argument_errors(case):
    D = case["D"]["fp64"]
    if case["name"] != "32x32x16":
        pytest.skip("one case suffices")
    L = tp.lib()
    import ctypes as C
    x = torch.zeros(D.shape, dtype=torch.float64, device=case["dev"])
    assert L.tpmg_dg1_apply(None, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), None) == -1
    assert L.tpmg_dg1_apply(D.handle, None, C.c_void_p(x.data_ptr()), None) == -1
    assert L.tpmg_dg1_vcycle(D.handle, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), None) == -1


def test_nlo_workload_matches_oracle():
    """The benchmark's NLO workload in full (256 x 256 x 64 graded, 25.2 M DG1
    unknowns, five lowest-order levels): band factors of sampled columns, one
    NLO V-cycle, the FP64 CG at the oracle's iteration count and the mixed CG
    against the oracle's FP64 solution."""
    import synthetic as syn
    dev = device()
    w = syn.NLO_WORKLOADS["nlo_dg1_256x256x64"]
    print(f"[gpu] DG1 at full size: {w.name}", flush=True)
    c, b = w.coefficients(), w.dg1_rhs()
    kw = dict(dz=w.dz(), a_h=w.a_h, a_z=w.a_z, levels=w.levels, nu=w.nu, omega=w.omega, coarse=w.coarse,
              n_coarse=w.n_coarse)
    P = oracle.problem_for(w, c)
    G = oracle.DG1(P)
    ct, bt = to_dev(c), to_dev(b)
    H = tp.Hierarchy(ct, precision="fp64", **kw)
    D = tp.DG1Level(H)
    F = D.factors()
    rng = np.random.default_rng(11)
    cols = [(0, 0), (255, 255), (0, 255), (255, 0)] + [tuple(v) for v in rng.integers(0, 256, size=(28, 2))]
    Fo = G.factors()
    for (j, i) in cols:
        got = F[j, i].cpu().numpy()
        ref = Fo[j, i]
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (j, i)
    del Fo, F
    e = rel_err(host(D.vcycle(bt)), G.vcycle(b))
    print(f"[gpu] {w.name} NLO V-cycle: {e:.2e}", flush=True)
    assert e <= 1e-11, e
    x_or, info_or = G.pcg(b, rtol=w.rtol, maxit=100)
    x, info = D.solve(bt, rtol=w.rtol, maxit=info_or["iterations"], flexible=False)
    err = rel_err(host(x), x_or)
    print(f"[gpu] {w.name} FP64 CG: {info['iterations']} it (oracle {info_or['iterations']}), error {err:.2e}",
          flush=True)
    assert info["converged"] and info["iterations"] == info_or["iterations"] and err <= 1e-10, (info, err)
    D.close()
    H.close()
    Hm = tp.Hierarchy(ct, precision="mixed", **kw)
    Dm = tp.DG1Level(Hm)
    x, info = Dm.solve(bt, rtol=w.rtol, maxit=100)
    err = rel_err(host(x), x_or)
    print(f"[gpu] {w.name} mixed CG: {info['iterations']} it, error vs oracle {err:.2e}", flush=True)
    assert info["converged"] and err <= 1e-8, (info, err)
    Dm.close()
    Hm.close()
