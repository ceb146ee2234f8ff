"""GPU parity of the velocity-pressure system (mixed operator, Schur-complement
preconditioner, flexible GMRES) against the CPU oracle.

Operator: the GPU and the oracle evaluate the same sums in a different order,
1e-13 max-relative.  Preconditioner: one V-cycle inside, so the V-cycle bounds
of the component tests apply (FP64 1e-12 raised to 8 kappa u64; FP32 within 2x
of the oracle's own FP32 error, floor 2e-5).  GMRES in FP64: the GPU runs the
oracle's iteration count (classical Gram-Schmidt twice on the GPU, modified
Gram-Schmidt in the oracle: equal in exact arithmetic) and its iterate must
match within 1e-10 relative.  With the FP32 V-cycle the flexible GMRES must
reach the same tolerance in FP64 residuals within one iteration of the oracle.
"""
import zlib

import numpy as np
import pytest

import oracle
import paper_1605_00492_amd as tp
import synthetic as syn
from gpu_util import device, host, max_rel, rel_err, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    # name: (n, nz, levels, a_h, a_z, graded, coarse)
    "ref32x16": (32, 16, 3, 1.0, 100.0, False, "direct"),
    "ragged24x13": (24, 13, 3, 4.0, 1e4, True, "smooth"),
    "graded64x32_cfl8": (64, 32, 3, 16.0, 1e4, True, "smooth"),
    "single_level32x16": (32, 16, 1, 16.0, 1e4, True, "smooth"),
    "tiny2x3": (2, 3, 1, 1.0, 10.0, False, "smooth"),
    "graded256x32_cfl8": (256, 32, 5, 16.0, 1e4, True, "smooth"),
}


class Case:
    def __init__(self, name):
        n, nz, levels, a_h, a_z, graded, coarse = CASES[name]
        self.name = name
        self.w = syn.Workload(name, n, nz, levels, a_h, a_z, graded, "uniform", coarse=coarse)
        self.c = self.w.coefficients()
        self.P = oracle.problem_for(self.w, self.c)
        kw = dict(dz=self.w.dz(), a_h=a_h, a_z=a_z, levels=levels, nu=self.w.nu, omega=self.w.omega,
                  coarse=coarse, n_coarse=self.w.n_coarse)
        ct = to_dev(self.c)
        self.H = {p: tp.Hierarchy(ct, precision=p, **kw) for p in ("fp64", "mixed")}
        self.rng = np.random.default_rng(zlib.crc32(name.encode()))
        self.b = self.w.mixed_rhs()

    def vec(self):
        v = self.rng.standard_normal((4, self.w.nz, self.w.n, self.w.n))
        v[2, -1] = 0.0
        return v


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    device()
    print(f"[gpu] mixed-system case {request.param}", flush=True)
    cs = Case(request.param)
    yield cs
    for h in cs.H.values():
        h.close()


def test_mixed_apply(case):
    x = case.vec()
    ref = case.P.mixed_apply(x)
    for p in ("fp64", "mixed"):
        got = host(case.H[p].mixed_apply(to_dev(x)))
        assert np.all(got[2, -1] == 0.0)
        e = max_rel(got, ref)
        assert e <= 1e-13, (case.name, p, e)


def test_mixed_precondition(case):
    r = case.vec()
    ref = case.P.mixed_precondition(r)
    got = host(case.H["fp64"].mixed_precondition(to_dev(r)))
    e64 = rel_err(got, ref)
    ref32o = case.P.mixed_precondition(r, fp32=True)
    e32o = rel_err(ref32o, ref)
    got32 = host(case.H["mixed"].mixed_precondition(to_dev(r), fp32=True))
    e32 = rel_err(got32, ref)
    bound64 = max(1e-12, 8.0 * (e32o / 2.0 ** -24) * 2.0 ** -53)
    bound32 = max(2e-5, 2.0 * e32o)
    print(f"[gpu] {case.name} preconditioner: fp64 {e64:.2e} (bound {bound64:.1e}), fp32 {e32:.2e} "
          f"(oracle fp32 {e32o:.2e})", flush=True)
    assert e64 <= bound64 and e32 <= bound32


def test_fgmres_fp64_matches_oracle(case):
    xo, io = case.P.mixed_fgmres(case.b, rtol=1e-8, restart=30, maxit=300)
    assert io["converged"]
    it = io["iterations"]
    x, info = case.H["fp64"].mixed_solve(to_dev(case.b), rtol=1e-8, restart=30, maxit=it, history=True)
    print(f"[gpu] {case.name} GMRES fp64: {info['iterations']} it (oracle {it}), true residual "
          f"{info['true_rel_residual']:.2e}", flush=True)
    assert info["converged"] and info["iterations"] == it, (info, io)
    err = rel_err(host(x), xo)
    assert err <= 1e-10, err
    np.testing.assert_allclose(info["history"], io["history"], rtol=1e-6, atol=1e-14)
    assert info["true_rel_residual"] <= 1.01e-8


def test_fgmres_mixed_precision(case):
    xo, io = case.P.mixed_fgmres(case.b, rtol=1e-10, restart=30, maxit=300)
    x, info = case.H["mixed"].mixed_solve(to_dev(case.b), rtol=1e-10, restart=30, maxit=300)
    err = rel_err(host(x), xo)
    print(f"[gpu] {case.name} GMRES mixed: {info['iterations']} it (oracle fp64 {io['iterations']}), "
          f"true residual {info['true_rel_residual']:.2e}, vs oracle {err:.2e}", flush=True)
    assert info["converged"] and info["true_rel_residual"] <= 1.05e-10
    assert abs(info["iterations"] - io["iterations"]) <= max(1, io["iterations"] // 10)
    assert err <= 1e-8


def test_fgmres_restart_and_determinism(case):
    b = to_dev(case.b)
    H = case.H["fp64"]
    x1, i1 = H.mixed_solve(b, rtol=1e-8, restart=4, maxit=400)
    x2, i2 = H.mixed_solve(b, rtol=1e-8, restart=4, maxit=400)
    assert i1["converged"] and i1["true_rel_residual"] <= 1.01e-8
    assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]
    xo, io = case.P.mixed_fgmres(case.b, rtol=1e-8, restart=4, maxit=400)
    assert i1["iterations"] == io["iterations"]


def test_edge_cases_and_errors():
    device()
    cs = Case("ref32x16")
    H = cs.H["fp64"]
    z = torch.zeros((4, cs.w.nz, cs.w.n, cs.w.n), dtype=torch.float64, device="cuda")
    x, info = H.mixed_solve(z, rtol=1e-8)
    assert info["converged"] and info["iterations"] == 0 and float(x.abs().max()) == 0.0
    x, info = H.mixed_solve(to_dev(cs.b), rtol=1e-14, maxit=3)
    assert not info["converged"] and info["iterations"] == 3 and info["status"] == 1
    bad = to_dev(cs.b)
    bad[2, -1, 3, 5] = 1.0                          # no face above the top cell
    with pytest.raises(tp.TpmgError) as ei:
        H.mixed_solve(bad, rtol=1e-8)
    assert ei.value.status == -1
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(tp.TpmgError) as ei:
        _raw_solve(H, to_dev(cs.b), small)
    assert ei.value.status == -4
    with pytest.raises(tp.TpmgError):
        H.mixed_precondition(to_dev(cs.b), fp32=True)   # fp32 needs a mixed hierarchy
    with pytest.raises(tp.TpmgError):
        H.mixed_workspace_bytes(0)
    for h in cs.H.values():
        h.close()


def _raw_solve(H, b, ws):
    """Call tpmg_mixed_solve with a workspace that is too small."""
    import ctypes as C
    from paper_1605_00492_amd.binding import MixedOpts, SolveInfo, _check, _ptr, _stream, lib
    x = torch.empty_like(b)
    opts = MixedOpts()
    opts.rtol, opts.restart, opts.maxit, opts.history = 1e-8, 30, 10, None
    info = SolveInfo()
    st = lib().tpmg_mixed_solve(H.handle, _ptr(b), _ptr(x), _ptr(ws), ws.numel(), C.byref(opts), C.byref(info),
                                _stream(H.device))
    _check(st, "tpmg_mixed_solve", H.handle)
