"""GPU parity of each V-cycle component against the CPU oracle.

Every kernel of the path is called through the C interface (via the ctypes
binding) and compared element by element with the oracle on the same seeded
inputs: operator apply on every level, the line-relaxation sweep (zero guess
and general), residual + restriction, prolongation + sweep, the coarsest
solve, the coarse coefficients and the whole V-cycle, in FP64 and FP32.

Tolerances.  FP64: the GPU and the oracle differ only in rounding order
(fused multiply-adds, partitioned vs textbook column elimination), so the
results agree to a few hundred ulps: 1e-12 relative (sweeps and V-cycles,
whose column solves amplify rounding by the column condition number) and
1e-13 for the operator.  FP32: the GPU works on FP32 copies of the
coefficients and is compared with the FP64 oracle on the same (FP32-rounded)
inputs.  The attainable FP32 accuracy depends on the conditioning of the
computation (b - H u with vertical couplings up to ~1e6 loses digits in any
FP32 arithmetic), so the bound is the error of the oracle's own textbook
FP32 computation of the same step: the GPU must be within 2x of it, and
never required below 2e-5 (a few hundred FP32 ulps, eps = 6e-8).  The same
measurement gives the condition number of the step, kappa ~ e32 / u32, and
the FP64 bound is raised to 8 kappa u64 where that exceeds the fixed bound.
"""
import zlib

import numpy as np
import pytest

import oracle
import synthetic as syn
from gpu_util import device, host, max_rel, rel_err, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    # name: (n, nz, levels, a_z, graded, coarse)
    "ref32x16_direct": (32, 16, 3, 100.0, False, "direct"),
    "ragged24x13": (24, 13, 3, 1e4, True, "smooth"),
    "tall16x64": (16, 64, 4, 1e4, True, "smooth"),
    "flat8x1": (8, 1, 2, 10.0, False, "smooth"),
    "deep64x128": (64, 128, 3, 1e4, True, "smooth"),
    "deep32x256": (32, 256, 2, 1e4, True, "smooth"),
    # rows of whole 64-column tiles on level 0 and its parent level: the
    # FP32 prolongation sweep's row-uniform addressing (two tiles per row,
    # periodic wrap, a ragged last chunk)
    "rows128x13": (128, 13, 3, 1e4, True, "smooth"),
}

TOL64_OP, TOL64, TOL32 = 1e-13, 1e-12, 2e-5


class Case:
    def __init__(self, name):
        n, nz, levels, a_z, graded, coarse = CASES[name]
        self.name = name
        self.w = syn.Workload(name, n, nz, levels, 1.0, a_z, graded, "uniform", coarse=coarse)
        self.c = self.w.coefficients()
        self.P = oracle.problem_for(self.w, self.c)
        kw = dict(dz=self.w.dz(), a_h=1.0, a_z=a_z, levels=levels, nu=self.w.nu,
                  omega=self.w.omega, coarse=coarse, n_coarse=self.w.n_coarse)
        ct = to_dev(self.c)
        self.H = {p: __import__("paper_1605_00492_amd").Hierarchy(ct, precision=p, **kw)
                  for p in ("fp64", "mixed")}
        self.rng = np.random.default_rng(zlib.crc32(name.encode()))

    def vec(self, level):
        nl = self.P.n_at(level)
        return self.rng.standard_normal((self.w.nz, nl, nl))


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    device()
    print(f"[gpu] components case {request.param}", flush=True)
    return Case(request.param)


def _both(case, fn_gpu, fn_or, level, inputs, tol64, tol32, metric=rel_err):
    """Run the GPU component in FP64 and FP32 and compare with the FP64 oracle.

    fn_or(*inputs, fp32) evaluates the oracle in double or in float."""
    ref = fn_or(*inputs, fp32=False)
    got64 = host(fn_gpu(case.H["fp64"], *[to_dev(a) for a in inputs]))
    e64 = metric(got64, ref)
    inputs32 = [a.astype(np.float32) for a in inputs]
    ref32 = fn_or(*[a.astype(np.float64) for a in inputs32], fp32=False)
    got32 = host(fn_gpu(case.H["mixed"], *[to_dev(a) for a in inputs32]))
    e32 = metric(got32, ref32)
    e32_oracle = metric(fn_or(*inputs32, fp32=True), ref32)
    bound32 = max(tol32, 2.0 * e32_oracle)
    kappa = e32_oracle / 2.0 ** -24
    bound64 = max(tol64, 8.0 * kappa * 2.0 ** -53)
    print(f"[gpu] {case.name} level {level}: fp64 {e64:.2e} (bound {bound64:.1e})  fp32 {e32:.2e} "
          f"(oracle fp32 {e32_oracle:.2e})", flush=True)
    assert e64 <= bound64 and e32 <= bound32, (case.name, level, e64, e32, e32_oracle)


def test_level_coefficients_exact(case):
    for lev in range(case.w.levels):
        ref = case.P.coeffs(lev)
        ref[2, -1] = 0.0  # the U slot above the top cell holds no face
        got = host(case.H["fp64"].level_coefficients(lev))
        assert np.array_equal(got, ref), (case.name, lev)
        got32 = host(case.H["mixed"].level_coefficients(lev, fp32=True))
        assert np.array_equal(got32, ref.astype(np.float32)), (case.name, lev)


def test_apply_every_level(case):
    for lev in range(case.w.levels):
        x = case.vec(lev)
        _both(case, lambda H, xx: H.apply(xx, level=lev),
              lambda xx, fp32: case.P.apply(xx, lev, fp32=fp32), lev,
              [x], TOL64_OP, TOL32, metric=max_rel)


def test_smooth_zero_guess(case):
    for lev in range(case.w.levels):
        b = case.vec(lev)
        _both(case, lambda H, bb: H.smooth(bb, None, level=lev),
              lambda bb, fp32: case.P.smooth(np.zeros_like(bb), bb, lev, fp32=fp32), lev, [b], TOL64,
              TOL32)


def test_smooth_general(case):
    for lev in range(case.w.levels):
        u, b = case.vec(lev), case.vec(lev)
        _both(case, lambda H, uu, bb: H.smooth(bb, uu, level=lev),
              lambda uu, bb, fp32: case.P.smooth(uu, bb, lev, fp32=fp32), lev, [u, b], TOL64, TOL32)


def test_residual_restrict(case):
    for lev in range(case.w.levels - 1):
        u, b = case.vec(lev), case.vec(lev)
        _both(case, lambda H, uu, bb: H.residual_restrict(uu, bb, level=lev),
              lambda uu, bb, fp32: case.P.restrict(bb - case.P.apply(uu, lev, fp32=fp32), lev, fp32=fp32),
              lev, [u, b],
              TOL64_OP * 10, TOL32)


def test_prolong_smooth(case):
    for lev in range(case.w.levels - 1):
        u, b, e = case.vec(lev), case.vec(lev), case.vec(lev + 1)
        _both(case, lambda H, uu, ee, bb: H.prolong_smooth(uu, ee, bb, level=lev),
              lambda uu, ee, bb, fp32: case.P.smooth(case.P.prolong_add(ee, uu, lev, fp32=fp32), bb, lev,
                                                     fp32=fp32), lev,
              [u, e, b], TOL64, TOL32)


def test_coarse_solve(case):
    b = case.vec(case.w.levels - 1)
    _both(case, lambda H, bb: H.coarse_solve(bb), lambda bb, fp32: case.P.coarse_solve(bb, fp32=fp32),
          case.w.levels - 1, [b], TOL64 * 10, TOL32 * 5)


def test_vcycle(case):
    b = case.vec(0)
    _both(case, lambda H, bb: H.vcycle(bb), lambda bb, fp32: case.P.vcycle(bb, fp32=fp32), 0, [b],
          TOL64 * 10, TOL32 * 5)


def test_vcycle_column_major_layout(case):
    """The paper's column-contiguous ordering at the boundary runs the same
    kernels between two transposes: results equal the level-major ones bit for bit."""
    import paper_1605_00492_amd as tp
    cc = np.ascontiguousarray(np.transpose(case.c, (2, 3, 1, 0)))   # c[j][i][k][f]
    w = case.w
    H = tp.Hierarchy(to_dev(cc), dz=w.dz(), a_h=w.a_h, a_z=w.a_z, levels=w.levels, nu=w.nu,
                     omega=w.omega, coarse=w.coarse, n_coarse=w.n_coarse, layout="column")
    b = case.vec(0)
    bcol = to_dev(np.ascontiguousarray(np.transpose(b, (1, 2, 0))))
    z = np.transpose(host(H.vcycle(bcol)), (2, 0, 1))
    assert np.array_equal(z, host(case.H["fp64"].vcycle(to_dev(b))))
    y = np.transpose(host(H.apply(bcol)), (2, 0, 1))
    assert np.array_equal(y, host(case.H["fp64"].apply(to_dev(b))))
    H.close()


def test_vcycle_deterministic(case):
    b = to_dev(case.vec(0))
    for p in ("fp64", "mixed"):
        bb = b if p == "fp64" else b.float()
        z1 = host(case.H[p].vcycle(bb))
        z2 = host(case.H[p].vcycle(bb))
        assert np.array_equal(z1, z2)
