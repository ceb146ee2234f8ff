"""Event timers of the library (tpmg_profile_*): kernel classes and the
per-level breakdown of a V-cycle count the launches the cycle makes on each
level, and the level times add up to (at most) the whole cycle."""
import numpy as np
import pytest

import paper_1605_00492_amd as tp
from paper_1605_00492_amd import binding as B
from gpu_util import device, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("coarse", ["smooth", "direct"])
def test_level_timers_count_every_launch(coarse):
    device()
    n, nz, levels = (64, 32, 4) if coarse == "smooth" else (32, 8, 3)
    print(f"[gpu] level timers: {coarse} {n}x{n}x{nz}, {levels} levels", flush=True)
    rng = np.random.default_rng(3)
    c = 1.0 + 0.5 * rng.random((3, nz, n, n))
    H = tp.Hierarchy(to_dev(c), a_h=1.0, a_z=1e3, levels=levels, coarse=coarse, n_coarse=2, precision="mixed")
    b = to_dev(rng.standard_normal((nz, n, n))).float()
    H.vcycle(b)
    H.profile_enable(True, levels=True)
    reps = 3
    for _ in range(reps):
        H.vcycle(b)
    vc_ms, vc_n = H.profile_read(B.K_VCYCLE)
    assert vc_n == reps
    total = 0.0
    for level in range(levels):
        ms, cnt = H.profile_read_level(level)
        # nu = 2/2: sweep from zero, general sweep, residual + restriction,
        # prolongation sweep, general sweep; the coarsest: its solve
        want = (2 if coarse == "smooth" else 1) if level == levels - 1 else 5
        assert cnt == reps * want, (level, cnt)
        assert ms > 0
        total += ms
    assert total <= vc_ms * 1.02 + 1e-3, (total, vc_ms)
    assert total >= 0.3 * vc_ms, (total, vc_ms)
    with pytest.raises(tp.TpmgError):
        H.profile_read_level(levels)
    H.profile_enable(False)
    H.close()


def test_dg1_timers():
    device()
    print("[gpu] DG1 timers", flush=True)
    rng = np.random.default_rng(4)
    n, nz = 32, 16
    c = 1.0 + 0.5 * rng.random((3, nz, n, n))
    H = tp.Hierarchy(to_dev(c), a_h=1.0, a_z=100.0, levels=3, coarse="direct")
    D = tp.DG1Level(H)
    b = to_dev(rng.standard_normal((6, nz, n, n)))
    H.profile_enable(True)
    D.vcycle(b)
    ms, cnt = H.profile_read(B.K_DG1_VCYCLE)
    assert cnt == 1 and ms > 0
    ms, cnt = H.profile_read(B.K_DG1_SWEEP)
    assert cnt == 3   # one more pre-sweep after the one from zero, two post-sweeps
    ms, cnt = H.profile_read(B.K_VCYCLE)
    assert cnt == 1   # the lowest-order V-cycle inside
    H.profile_enable(False)
    D.close()
    H.close()
