"""GPU adjoint: the fused face-gradient kernel against the oracle, the full
autograd gradient against the oracle's gradient (norm-wise 1e-6 relative
with forward and adjoint solves at 1e-10), and central finite differences
(h = 1e-6) on 32 seeded faces with the tolerance of the FD truncation and
rounding error: |g_FD - g| <= 1e-6 max|g| + 1e-4 |g|.  The perturbed
solutions are formed as x + d with d solved from the perturbed residual, so
the difference is not limited by the solver's floor relative to ||b||."""
import numpy as np
import pytest

import oracle
import paper_1605_00492_amd as tp
import synthetic as syn
from gpu_util import device, host, max_rel, rel_err, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W4 = syn.CONFIGS["adjoint_256x256x32"]


def hkw(w):
    return dict(dz=w.dz(), a_h=w.a_h, a_z=w.a_z, levels=w.levels, nu=w.nu, omega=w.omega,
                coarse=w.coarse, n_coarse=w.n_coarse)


@pytest.fixture(scope="module")
def adj():
    device()
    print("[gpu] adjoint workload", W4.name, flush=True)
    w = W4
    c, b, xt = w.coefficients(), w.rhs(), w.target()
    P = oracle.problem_for(w, c)
    x, _ = P.pcg(b, rtol=1e-12, maxit=100)
    lam, _ = P.pcg(x - xt, rtol=1e-12, maxit=100)
    g = P.face_gradient(lam, x)
    return dict(w=w, c=c, b=b, xt=xt, P=P, x=x, lam=lam, g=g)


def test_face_gradient_kernel(adj):
    H = tp.Hierarchy(to_dev(adj["c"]), **hkw(adj["w"]))
    g = host(H.face_gradient(to_dev(adj["lam"]), to_dev(adj["x"])))
    assert max_rel(g, adj["g"]) <= 1e-12
    assert np.all(g[2, -1] == 0.0)
    # column-major layout gives the same gradient
    Hc = tp.Hierarchy(to_dev(np.ascontiguousarray(np.transpose(adj["c"], (2, 3, 1, 0)))),
                      layout="column", **hkw(adj["w"]))
    gc = host(Hc.face_gradient(to_dev(np.ascontiguousarray(np.transpose(adj["lam"], (1, 2, 0)))),
                               to_dev(np.ascontiguousarray(np.transpose(adj["x"], (1, 2, 0))))))
    assert max_rel(np.transpose(gc, (3, 2, 0, 1)), adj["g"]) <= 1e-12
    H.close()
    Hc.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autograd_matches_oracle_gradient(adj, precision):
    w = adj["w"]
    c = to_dev(adj["c"]).requires_grad_(True)
    b = to_dev(adj["b"]).requires_grad_(True)
    x = tp.solve(c, b, rtol=1e-10, maxit=100, precision=precision, **hkw(w))
    J = 0.5 * torch.sum((x - to_dev(adj["xt"])) ** 2)
    J.backward()
    gc = host(c.grad)
    gb = host(b.grad)
    e_c = rel_err(gc, adj["g"])
    e_b = rel_err(gb, adj["lam"])
    print(f"[gpu] autograd {precision}: dJ/dc rel err {e_c:.2e}, dJ/db rel err {e_b:.2e}", flush=True)
    assert e_c <= 1e-6 and e_b <= 1e-6


def test_central_finite_differences(adj):
    w = adj["w"]
    H = tp.Hierarchy(to_dev(adj["c"]), **hkw(w))
    bt = to_dev(adj["b"])
    xt = adj["xt"]
    x, _ = H.solve(bt, rtol=1e-13, maxit=200)
    lam, _ = H.solve(x - to_dev(xt), rtol=1e-13, maxit=200)
    g = host(H.face_gradient(lam, x))
    H.close()
    gmax = np.abs(g).max()
    h = w.extra["fd_h"]
    faces = w.fd_faces(w.extra["fd_faces"])
    worst = 0.0
    x_h, xt_h = host(x), xt
    for f, k, j, i in faces:
        # x_pm = x + d_pm with H_pm d_pm = b - H_pm x solved to 1e-12 relative to
        # its own (h-sized) right-hand side: the FD then carries no solver floor.
        ds = []
        for sgn in (1.0, -1.0):
            cc = adj["c"].copy()
            cc[f, k, j, i] += sgn * h
            Hp = tp.Hierarchy(to_dev(cc), **hkw(w))
            r = bt - Hp.apply(x)
            d, info = Hp.solve(r, rtol=1e-12, maxit=100)
            ds.append(host(d))
            Hp.close()
        fd = 0.5 * np.sum((ds[0] - ds[1]) * (2 * (x_h - xt_h) + ds[0] + ds[1])) / (2 * h)
        ga = g[f, k, j, i]
        tol = 1e-6 * gmax + 1e-4 * abs(ga)
        worst = max(worst, abs(fd - ga) / tol)
        assert abs(fd - ga) <= tol, (f, k, j, i, fd, ga)
    print(f"[gpu] FD check on {len(faces)} faces: worst error / tolerance = {worst:.3f}", flush=True)
