"""The full-size GPU tests check sampled columns against the oracle run on a
small periodic patch around each column.  This pins that sampling method:
on a grid the oracle handles whole, the patch results equal the full results
exactly, at interior and wrap-around columns."""
import numpy as np

import oracle
import synthetic as syn
from refs import patch


def test_patches_reproduce_full_oracle():
    w = syn.scaled(syn.CONFIGS["large_1024x1024x128"], 16, 24, 2, "patch16x24")
    c = w.coefficients()
    rng = np.random.default_rng(11)
    P = oracle.Problem(c, a_h=w.a_h, a_z=w.a_z, dz=w.dz(), levels=2, omega=w.omega)
    u, b = rng.standard_normal(c.shape[1:]), rng.standard_normal(c.shape[1:])
    full_apply, full_smooth = P.apply(u), P.smooth(u, b)
    full_restrict = P.restrict(b - P.apply(u))

    def small(cp):
        return oracle.Problem(np.ascontiguousarray(cp), a_h=w.a_h, a_z=w.a_z, dz=w.dz(), levels=1,
                              omega=w.omega)

    for (i, j) in [(0, 0), (15, 15), (0, 15), (15, 0), (3, 7), (8, 1)]:
        Q = small(patch(c, i, j))
        assert np.array_equal(Q.apply(patch(u, i, j))[:, 1, 1], full_apply[:, j, i])
        assert np.array_equal(Q.smooth(patch(u, i, j), patch(b, i, j))[:, 1, 1], full_smooth[:, j, i])
        I, J = i // 2, j // 2
        Q = small(patch(c, 2 * I, 2 * J, size=4))
        r = patch(b, 2 * I, 2 * J, size=4) - Q.apply(patch(u, 2 * I, 2 * J, size=4))
        assert np.array_equal(r[:, 1:3, 1:3].sum(axis=(1, 2)), full_restrict[:, J, I])
