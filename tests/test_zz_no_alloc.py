"""tpmg_apply_operator_static (the entry point that allocates nothing and
stages through the library's static device array) against
tpmg_apply_operator, called through the C interface: bit-identical results
on two calls in a row, the second with a smaller input, in both precisions
and both layouts; levels beyond the array's capacity are rejected on the
host before any launch."""
import ctypes as C

import numpy as np
import pytest

import paper_1605_00492_amd as tp
from paper_1605_00492_amd import binding
from gpu_util import device, host, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _coeffs(n, nz, seed, layout):
    rng = np.random.default_rng(seed)
    c = 1.0 + 0.5 * rng.random((3, nz, n, n))
    c[2, nz - 1] = 0.0
    if layout == "column":
        c = np.ascontiguousarray(c.transpose(2, 3, 1, 0))
    return c


def _both(H, x, level):
    """(existing entry point's y, static entry point's y) for the same x."""
    L = binding.lib()
    fp32 = 1 if x.dtype == torch.float32 else 0
    stream = C.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    y_ref = torch.full_like(x, float("nan"))
    y_st = torch.full_like(x, float("nan"))
    st = L.tpmg_apply_operator(H.handle, level, fp32, C.c_void_p(x.data_ptr()), C.c_void_p(y_ref.data_ptr()),
                               H.layout, stream)
    assert st == 0, L.tpmg_last_error(H.handle)
    st = L.tpmg_apply_operator_static(H.handle, level, fp32, C.c_void_p(x.data_ptr()), C.c_void_p(y_st.data_ptr()),
                                      H.layout, stream)
    assert st == 0, L.tpmg_last_error(H.handle)
    return host(y_ref), host(y_st)


@pytest.mark.parametrize("layout", ["level", "column"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_apply_matches_apply_operator(precision, layout):
    device()
    print(f"[gpu] static apply: {precision} {layout}", flush=True)
    dz = 1.05 ** np.arange(24)
    # the second hierarchy is smaller than the first, and each is called on
    # its finest level and then on a coarser (smaller) one
    for n, levels, seed in [(64, 3, 11), (32, 2, 12)]:
        ct = to_dev(_coeffs(n, 24, seed, layout))
        H = tp.Hierarchy(ct, dz=dz, a_h=1.0, a_z=1e3, levels=levels, coarse="smooth", precision=precision,
                         layout=layout)
        for level in (0, levels - 1):
            shape = H.cell_shape(level)
            rng = np.random.default_rng(100 + n + level)
            for dtype in ([torch.float64, torch.float32] if precision == "mixed" else [torch.float64]):
                x = to_dev(rng.standard_normal(shape)).to(dtype).contiguous()
                y_ref, y_st = _both(H, x, level)
                assert np.isfinite(y_ref).all()
                assert np.array_equal(y_ref, y_st), (n, level, dtype)
        H.close()


def test_static_apply_rejects_levels_beyond_capacity():
    device()
    print("[gpu] static apply: capacity", flush=True)
    # 256 x 256 x 80 = 5,242,880 cells: over the FP64 capacity (4,194,304),
    # within the FP32 one (8,388,608); level 1 (1,310,720 cells) fits both
    n, nz = 256, 80
    ct = to_dev(_coeffs(n, nz, 5, "level"))
    H = tp.Hierarchy(ct, a_h=1.0, a_z=1e3, levels=2, coarse="smooth", precision="mixed")
    L = binding.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    x = torch.zeros(H.cell_shape(0), dtype=torch.float64, device=ct.device)
    y = torch.zeros_like(x)
    st = L.tpmg_apply_operator_static(H.handle, 0, 0, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                      H.layout, stream)
    assert st == -4 and b"static scratch" in L.tpmg_last_error(H.handle)
    rng = np.random.default_rng(6)
    x32 = to_dev(rng.standard_normal(H.cell_shape(0))).float().contiguous()
    y_ref, y_st = _both(H, x32, 0)
    assert np.array_equal(y_ref, y_st)
    x1 = to_dev(rng.standard_normal(H.cell_shape(1)))
    y_ref, y_st = _both(H, x1, 1)
    assert np.array_equal(y_ref, y_st)
    H.close()
