"""The C interface without a GPU: the library loads, exports every function
include/tpmg.h declares, and rejects bad arguments on the host before any
device call."""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpmg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def tp():
    import paper_1605_00492_amd as tp
    if not os.path.exists(tp.binding.LIB_PATH):
        pytest.skip("libtpmg.so not built")
    return tp


def test_every_declared_symbol_is_exported(tp):
    names = declared_functions()
    assert len(names) >= 18
    lib = C.CDLL(tp.binding.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(tp.binding.EXPORTS) == names


def desc(tp, **kw):
    args = dict(n=32, nz=16, levels=3, a_h=1.0, a_z=100.0, dz=None, nu=(2, 2), omega=0.8,
                coarse="direct", n_coarse=2, precision="fp64")
    args.update(kw)
    return tp.make_desc(**args)[0]


@pytest.mark.parametrize("kw,status", [
    (dict(n=30), -2),                       # not divisible by 2^(levels-1)
    (dict(nz=0), -2),
    (dict(nz=257), -2),                     # beyond TPMG_MAX_NZ
    (dict(levels=0), -2),
    (dict(levels=13, n=4096), -2),
    (dict(omega=0.0), -1),
    (dict(omega=1.5), -1),
    (dict(nu=(0, 2)), -1),
    (dict(a_z=-1.0), -1),
    (dict(coarse="smooth", n_coarse=0), -1),
    (dict(n=64, levels=2), -2),             # direct coarse level too large (32*32*16)
    (dict(n=4096, nz=32, levels=9, coarse="smooth"), -2),   # 2^29 cells: FP64 arrays of 4 GiB
])
def test_workspace_bytes_validation(tp, kw, status):
    with pytest.raises(tp.TpmgError) as ei:
        tp.workspace_bytes(desc(tp, **kw))
    assert ei.value.status == status


def test_largest_grids_accepted(tp):
    """Just below the 4 GiB-per-array limit the description is valid."""
    n = tp.workspace_bytes(desc(tp, n=2048, nz=96, levels=8, coarse="smooth"))
    assert n > 3 * 2048 * 2048 * 96 * 8


def test_non_positive_spacing_is_not_spd(tp):
    import numpy as np
    dz = np.ones(16)
    dz[3] = 0.0
    d, keep = tp.make_desc(32, 16, 3, 1.0, 100.0, dz, (2, 2), 0.8, "direct", 2, "fp64")
    with pytest.raises(tp.TpmgError) as ei:
        tp.workspace_bytes(d)
    assert ei.value.status == -3


def test_workspace_sizes_grow_with_precision(tp):
    b64 = tp.workspace_bytes(desc(tp))
    b32 = tp.workspace_bytes(desc(tp, precision="mixed"))
    assert 0 < b64 < b32
    assert b64 % 256 == 0


def test_null_arguments_rejected_on_host(tp):
    L = tp.lib()
    out = C.c_void_p()
    d = desc(tp)
    # NULL coefficients / workspace / handle: argument errors, no device work
    assert L.tpmg_setup_hierarchy(C.byref(d), None, 0, None, 0, None, C.byref(out)) == -1
    assert L.tpmg_apply_operator(None, 0, 0, None, None, 0, None) == -1
    assert L.tpmg_vcycle(None, 0, None, None, 0, None) == -1
    assert L.tpmg_solve(None, None, None, 0, None, None, None) == -1
    assert L.tpmg_face_gradient(None, None, None, None, 0, None) == -1
    assert L.tpmg_destroy(None) == 0
    assert L.tpmg_level_n(None, 0) == -1
    assert L.tpmg_bandwidth_probe(None, None, 16, None) == -1
    assert b"NULL" in L.tpmg_last_error(None) or L.tpmg_last_error(None)
    # the static-scratch apply and the DG1 entry points: NULL handles
    assert L.tpmg_apply_operator_static(None, 0, 0, None, None, 0, None) == -1
    nb = C.c_size_t(0)
    assert L.tpmg_dg1_workspace_bytes(None, C.byref(nb)) == -1
    g = C.c_void_p()
    assert L.tpmg_dg1_setup(None, None, 0, None, C.byref(g)) == -1
    for name in ("tpmg_dg1_apply", "tpmg_dg1_line_solve", "tpmg_dg1_vcycle", "tpmg_dg1_prolong_add"):
        assert getattr(L, name)(None, None, None, None) == -1, name
    assert L.tpmg_dg1_smooth(None, None, None, None, None) == -1
    assert L.tpmg_dg1_residual_restrict(None, None, None, None, None) == -1
    assert L.tpmg_dg1_solve(None, None, None, None, None, None) == -1
    assert L.tpmg_dg1_factors(None, None, None) == -1
    assert L.tpmg_dg1_destroy(None) == 0
    assert L.tpmg_profile_enable(None, 1) == -1
    ms, cnt = C.c_double(0), C.c_int64(0)
    assert L.tpmg_profile_read_level(None, 0, C.byref(ms), C.byref(cnt)) == -1


def test_status_strings(tp):
    L = tp.lib()
    for s in (0, 1, -1, -2, -3, -4, -5, -6):
        assert L.tpmg_status_string(s)
    assert L.tpmg_status_string(0) == b"ok"


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
