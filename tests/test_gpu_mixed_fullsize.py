"""The velocity-pressure system at the benchmark's full size, checked with the
oracle's own operator.

1024 x 1024 x 128 (535,822,336 unknowns: three face components and the
pressure of 134 M cells), 7 levels, a_h = 16 (nu_CFL = 8), restarted flexible
GMRES(20) to rtol 1e-5 with the FP32 V-cycle: the configuration that
`bench.py --mixed-system` times.  The oracle's GMRES does not fit at this
size (its Krylov basis alone would take 86 GB of host memory and hours of one
core), so the oracle checks what defines the answer:
  * the operator: A v for a random v, GPU against the oracle, within the
    1e-13 max-relative bound of the smaller parity cases (the same sums in
    another order);
  * the solution: b - A y formed by the oracle for the GPU's y has relative
    norm below the solve's tolerance and equals the true residual the GPU
    reports (to 1e-6 of itself).
"""
import numpy as np
import pytest

import oracle
import paper_1605_00492_amd as tp
import synthetic as syn
from gpu_util import device, host, max_rel, to_dev

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

A_H = 16.0
RTOL = 1e-5
RESTART = 20


def test_full_size_velocity_pressure_against_oracle_operator():
    device()
    w = syn.CONFIGS["large_1024x1024x128"]
    print(f"[gpu] velocity-pressure system at {w.n}x{w.n}x{w.nz}, a_h {A_H}: inputs and oracle set-up", flush=True)
    c, b = w.coefficients(), w.mixed_rhs()
    P = oracle.problem_for(w, c, a_h=A_H)
    H = tp.Hierarchy(to_dev(c), dz=w.dz(), a_h=A_H, a_z=w.a_z, levels=w.levels, nu=w.nu, omega=w.omega,
                     coarse=w.coarse, n_coarse=w.n_coarse, precision="mixed")
    try:
        rng = np.random.default_rng(1605)
        v = rng.standard_normal(b.shape)
        v[2, w.nz - 1] = 0.0  # no face above the top cell
        print("[gpu] operator apply on a random vector", flush=True)
        got = host(H.mixed_apply(to_dev(v)))
        torch.cuda.empty_cache()
        ref = P.mixed_apply(v)
        e_op = max_rel(got, ref)
        del got, ref, v
        print(f"[gpu] operator: max-relative difference {e_op:.2e}", flush=True)
        assert e_op <= 1e-13, e_op

        print(f"[gpu] GMRES({RESTART}) to {RTOL:.0e} with the FP32 V-cycle", flush=True)
        y, info = H.mixed_solve(to_dev(b), rtol=RTOL, restart=RESTART, maxit=300)
        yh = host(y)
        del y
        torch.cuda.empty_cache()
        r = b - P.mixed_apply(yh)
        rel = float(np.linalg.norm(r) / np.linalg.norm(b))
        print(f"[gpu] solve: {info['iterations']} iterations, residual by the oracle's operator {rel:.4e}, "
              f"reported {info['true_rel_residual']:.4e}", flush=True)
        assert info["converged"] and rel <= RTOL, (info, rel)
        assert abs(rel - info["true_rel_residual"]) <= 1e-6 * rel, (rel, info["true_rel_residual"])
    finally:
        H.close()
        torch.cuda.empty_cache()
