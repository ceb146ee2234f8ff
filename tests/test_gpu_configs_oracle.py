"""GPU against the oracle at the stated sizes of the graded workloads.

512 x 512 x 64 (6 levels; FP64 and mixed) and 1024 x 1024 x 128 (7 levels,
the benchmark's launch configuration) are run in full by the oracle (plain C,
OpenMP over columns) once per module:
  * one V-cycle in each precision against the oracle's V-cycle (FP64 to the
    component bound, FP32 within 2x of the oracle's own float V-cycle error);
  * the FP64 solve at the oracle's iteration count: iterate within 1e-10;
  * the mixed solve to 1e-8: within 1e-8 of the oracle's FP64 iterate;
  * at 1024 x 1024 x 128, the adjoint gradient of J = 0.5 ||x||^2 (mixed
    forward and adjoint solves) against the oracle's gradient from its own
    FP64 solves, within 1e-6 norm-wise.
"""
import numpy as np
import pytest

import oracle
import paper_1605_00492_amd as tp
import synthetic as syn
from gpu_util import device, host, rel_err, to_dev

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

NAMES = ["fp64_512x512x64", "large_1024x1024x128"]


@pytest.fixture(scope="module", params=NAMES)
def cfg(request):
    dev = device()
    w = syn.CONFIGS[request.param]
    print(f"[gpu] oracle at full size: {w.name} ({w.dof} DOF)", flush=True)
    c, b = w.coefficients(), w.rhs()
    P = oracle.problem_for(w, c)
    x_or, info_or = P.pcg(b, rtol=w.rtol, maxit=100)
    print(f"[gpu] {w.name}: oracle FP64 PCG {info_or['iterations']} it, "
          f"true rel residual {info_or['true_rel_residual']:.2e}", flush=True)
    ct = to_dev(c)
    kw = dict(dz=w.dz(), a_h=w.a_h, a_z=w.a_z, levels=w.levels, nu=w.nu, omega=w.omega,
              coarse=w.coarse, n_coarse=w.n_coarse)
    H = {p: tp.Hierarchy(ct, precision=p, **kw) for p in ("fp64", "mixed")}
    yield dict(w=w, c=c, b=b, P=P, x_or=x_or, info_or=info_or, H=H, bt=to_dev(b), dev=dev)
    for h in H.values():
        h.close()
    del ct
    torch.cuda.empty_cache()


def test_vcycle_matches_oracle(cfg):
    w, P, b = cfg["w"], cfg["P"], cfg["b"]
    ref = P.vcycle(b)
    got64 = host(cfg["H"]["fp64"].vcycle(cfg["bt"]))
    e64 = rel_err(got64, ref)
    b32 = b.astype(np.float32)
    ref32 = P.vcycle(b32.astype(np.float64))
    e32_oracle = rel_err(P.vcycle(b32, fp32=True), ref32)
    got32 = host(cfg["H"]["mixed"].vcycle(to_dev(b32)))
    e32 = rel_err(got32, ref32)
    bound64 = max(1e-11, 8.0 * (e32_oracle / 2.0 ** -24) * 2.0 ** -53)
    bound32 = max(1e-4, 2.0 * e32_oracle)
    print(f"[gpu] {w.name} V-cycle: fp64 {e64:.2e} (bound {bound64:.1e}), fp32 {e32:.2e} "
          f"(oracle float {e32_oracle:.2e})", flush=True)
    assert e64 <= bound64 and e32 <= bound32, (e64, e32, e32_oracle)


def test_fp64_solve_matches_oracle_iterate(cfg):
    w = cfg["w"]
    it = cfg["info_or"]["iterations"]
    x, info = cfg["H"]["fp64"].solve(cfg["bt"], rtol=w.rtol, maxit=it, history=True)
    err = rel_err(host(x), cfg["x_or"])
    print(f"[gpu] {w.name} FP64 solve: {info['iterations']} it (oracle {it}), error vs oracle {err:.2e}",
          flush=True)
    assert info["converged"] and info["iterations"] == it and err <= 1e-10, (info, err)
    np.testing.assert_allclose(info["history"], cfg["info_or"]["history"], rtol=1e-5)


def test_mixed_solve_matches_oracle(cfg):
    w = cfg["w"]
    x, info = cfg["H"]["mixed"].solve(cfg["bt"], rtol=w.rtol, maxit=100)
    err = rel_err(host(x), cfg["x_or"])
    print(f"[gpu] {w.name} mixed solve: {info['iterations']} it (oracle FP64 {cfg['info_or']['iterations']}), "
          f"true rel residual {info['true_rel_residual']:.2e}, error vs oracle FP64 iterate {err:.2e}", flush=True)
    assert info["converged"] and info["true_rel_residual"] <= 1.05 * w.rtol
    assert err <= 1e-8, err


def test_adjoint_gradient_matches_oracle(cfg):
    """J = 0.5 ||x||^2: dJ/dx = x, lambda = H^{-1} x, dJ/dc on every face."""
    w = cfg["w"]
    if w.name != "large_1024x1024x128":
        pytest.skip("the adjoint of the large mixed-precision workload")
    P = cfg["P"]
    lam_or, info_l = P.pcg(cfg["x_or"], rtol=w.rtol, maxit=100)
    g_or = P.face_gradient(lam_or, cfg["x_or"])
    H = cfg["H"]["mixed"]
    x, _ = H.solve(cfg["bt"], rtol=w.rtol, maxit=100)
    lam, _ = H.solve(x, rtol=w.rtol, maxit=100)
    g = host(H.face_gradient(lam, x))
    err = rel_err(g, g_or)
    print(f"[gpu] {w.name} adjoint gradient (mixed GPU vs FP64 oracle): error {err:.2e}", flush=True)
    assert err <= 1e-6, err
