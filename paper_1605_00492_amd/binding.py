"""ctypes binding of libtpmg (include/tpmg.h).

Argument marshalling only: every step of the solver runs in the HIP kernels
of libtpmg.so.  PyTorch provides device memory and the stream.  There is no
fallback: if the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpmg.so")

OK, NOT_CONVERGED = 0, 1
LEVEL_MAJOR, COLUMN_MAJOR = 0, 1
FP64, MIXED = 0, 1
COARSE_DIRECT, COARSE_SMOOTH = 0, 1
(K_SWEEP, K_SWEEP0, K_PROLSWEEP, K_RESTRICT, K_PCG_APPLY, K_PCG_UPDATE, K_VCYCLE, K_DG1_SWEEP, K_DG1_PCG_APPLY,
 K_DG1_VCYCLE) = range(10)

EXPORTS = [
    "tpmg_workspace_bytes", "tpmg_setup_hierarchy", "tpmg_level_n", "tpmg_apply_operator",
    "tpmg_apply_operator_static",
    "tpmg_vcycle", "tpmg_solve", "tpmg_face_gradient", "tpmg_smooth", "tpmg_residual_restrict",
    "tpmg_prolong_smooth", "tpmg_coarse_solve", "tpmg_mixed_workspace_bytes", "tpmg_mixed_apply",
    "tpmg_mixed_precondition", "tpmg_mixed_solve", "tpmg_level_coefficients", "tpmg_profile_enable",
    "tpmg_profile_read", "tpmg_profile_read_level", "tpmg_bandwidth_probe", "tpmg_destroy", "tpmg_status_string",
    "tpmg_last_error", "tpmg_dg1_workspace_bytes", "tpmg_dg1_setup", "tpmg_dg1_apply", "tpmg_dg1_line_solve",
    "tpmg_dg1_smooth", "tpmg_dg1_residual_restrict", "tpmg_dg1_prolong_add", "tpmg_dg1_vcycle", "tpmg_dg1_solve",
    "tpmg_dg1_factors", "tpmg_dg1_destroy",
]


class TpmgError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class MixedOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("maxit", C.c_int32), ("history", C.c_void_p)]


class Desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("nz", C.c_int32), ("nlevels", C.c_int32),
                ("a_h", C.c_double), ("a_z", C.c_double), ("dz", C.c_void_p),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("omega", C.c_double),
                ("coarse", C.c_int32), ("n_coarse", C.c_int32), ("precision", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("x0_nonzero", C.c_int32),
                ("flexible", C.c_int32), ("history", C.c_void_p), ("omega_alt", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("rel_residual", C.c_double), ("true_rel_residual", C.c_double)]


_lib = None


def lib():
    """Load libtpmg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1605_00492_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, st = C.c_void_p, C.c_int32, C.c_int
        L.tpmg_workspace_bytes.argtypes = [C.POINTER(Desc), C.POINTER(C.c_size_t)]
        L.tpmg_setup_hierarchy.argtypes = [C.POINTER(Desc), vp, i32, vp, C.c_size_t, vp,
                                           C.POINTER(vp)]
        L.tpmg_level_n.argtypes = [vp, i32]
        L.tpmg_level_n.restype = i32
        L.tpmg_apply_operator.argtypes = [vp, i32, i32, vp, vp, i32, vp]
        L.tpmg_apply_operator_static.argtypes = [vp, i32, i32, vp, vp, i32, vp]
        L.tpmg_vcycle.argtypes = [vp, i32, vp, vp, i32, vp]
        L.tpmg_solve.argtypes = [vp, vp, vp, i32, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.tpmg_face_gradient.argtypes = [vp, vp, vp, vp, i32, vp]
        L.tpmg_smooth.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        L.tpmg_residual_restrict.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        L.tpmg_prolong_smooth.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
        L.tpmg_coarse_solve.argtypes = [vp, i32, vp, vp, vp]
        L.tpmg_mixed_workspace_bytes.argtypes = [vp, i32, C.POINTER(C.c_size_t)]
        L.tpmg_mixed_apply.argtypes = [vp, vp, vp, vp]
        L.tpmg_mixed_precondition.argtypes = [vp, i32, vp, vp, vp]
        L.tpmg_mixed_solve.argtypes = [vp, vp, vp, vp, C.c_size_t, C.POINTER(MixedOpts), C.POINTER(SolveInfo), vp]
        L.tpmg_level_coefficients.argtypes = [vp, i32, i32, vp, vp]
        L.tpmg_profile_enable.argtypes = [vp, i32]
        L.tpmg_profile_read.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.tpmg_profile_read_level.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.tpmg_bandwidth_probe.argtypes = [vp, vp, C.c_size_t, vp]
        L.tpmg_destroy.argtypes = [vp]
        L.tpmg_dg1_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.tpmg_dg1_setup.argtypes = [vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        for name in ("tpmg_dg1_apply", "tpmg_dg1_line_solve", "tpmg_dg1_vcycle", "tpmg_dg1_prolong_add"):
            getattr(L, name).argtypes = [vp, vp, vp, vp]
        L.tpmg_dg1_smooth.argtypes = [vp, vp, vp, vp, vp]
        L.tpmg_dg1_residual_restrict.argtypes = [vp, vp, vp, vp, vp]
        L.tpmg_dg1_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.tpmg_dg1_factors.argtypes = [vp, vp, vp]
        L.tpmg_dg1_destroy.argtypes = [vp]
        L.tpmg_status_string.argtypes = [st]
        L.tpmg_status_string.restype = C.c_char_p
        L.tpmg_last_error.argtypes = [vp]
        L.tpmg_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("tpmg_level_n", "tpmg_status_string", "tpmg_last_error"):
                getattr(L, name).restype = st
        _lib = L
    return _lib


def _check(status: int, where: str, handle=None, ok=(OK,)):
    if status in ok:
        return status
    L = lib()
    detail = L.tpmg_last_error(handle).decode() or L.tpmg_status_string(status).decode()
    raise TpmgError(status, where, detail)


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def make_desc(n, nz, levels, a_h, a_z, dz, nu, omega, coarse, n_coarse, precision):
    d = Desc()
    d.n, d.nz, d.nlevels = int(n), int(nz), int(levels)
    d.a_h, d.a_z = float(a_h), float(a_z)
    d.nu_pre, d.nu_post = int(nu[0]), int(nu[1])
    d.omega = float(omega)
    d.coarse = COARSE_DIRECT if coarse == "direct" else COARSE_SMOOTH
    d.n_coarse = int(n_coarse)
    d.precision = MIXED if precision == "mixed" else FP64
    keep = None
    if dz is not None:
        import numpy as np
        keep = np.ascontiguousarray(dz, dtype=np.float64)
        assert keep.shape == (nz,)
        d.dz = keep.ctypes.data_as(C.c_void_p)
    return d, keep


def workspace_bytes(desc: Desc) -> int:
    out = C.c_size_t(0)
    _check(lib().tpmg_workspace_bytes(C.byref(desc), C.byref(out)), "tpmg_workspace_bytes")
    return out.value


class Hierarchy:
    """Multigrid hierarchy on the GPU for one set of face coefficients.

    c: float64 CUDA tensor of face coefficients, shape (3, nz, n, n) for
    layout='level' (c[f][k][j][i]) or (n, n, nz, 3) for layout='column'
    (c[j][i][k][f]).  Cell vectors are (nz, n, n) / (n, n, nz) respectively.
    """

    def __init__(self, c: torch.Tensor, dz=None, a_h=1.0, a_z=1.0, levels=1, nu=(2, 2), omega=0.8,
                 coarse="smooth", n_coarse=2, precision="fp64", layout="level"):
        if not (c.is_cuda and c.dtype == torch.float64 and c.is_contiguous()):
            raise ValueError("c must be a contiguous float64 CUDA tensor")
        self.layout = LEVEL_MAJOR if layout == "level" else COLUMN_MAJOR
        if self.layout == LEVEL_MAJOR:
            assert c.dim() == 4 and c.shape[0] == 3 and c.shape[2] == c.shape[3], c.shape
            nz, n = c.shape[1], c.shape[2]
        else:
            assert c.dim() == 4 and c.shape[3] == 3 and c.shape[0] == c.shape[1], c.shape
            n, nz = c.shape[0], c.shape[2]
        self.n, self.nz, self.levels = n, nz, levels
        self.device = c.device
        self.precision = precision
        self.mixed = precision == "mixed"
        self.params = dict(dz=dz, a_h=a_h, a_z=a_z, levels=levels, nu=tuple(nu), omega=omega,
                           coarse=coarse, n_coarse=n_coarse, precision=precision, layout=layout)
        self._desc, self._dz_keep = make_desc(n, nz, levels, a_h, a_z, dz, nu, omega, coarse,
                                              n_coarse, precision)
        self.ws_bytes = workspace_bytes(self._desc)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=c.device)
        h = C.c_void_p()
        _check(lib().tpmg_setup_hierarchy(C.byref(self._desc), _ptr(c), self.layout,
                                          _ptr(self.workspace), self.ws_bytes,
                                          _stream(self.device), C.byref(h)),
               "tpmg_setup_hierarchy")
        self._h = h

    # -- lifetime -------------------------------------------------------------
    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().tpmg_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("hierarchy is closed")
        return self._h

    # -- shapes ----------------------------------------------------------------
    def level_n(self, level: int) -> int:
        return int(lib().tpmg_level_n(self.handle, level))

    def cell_shape(self, level: int = 0):
        nl = self.level_n(level)
        return (self.nz, nl, nl) if self.layout == LEVEL_MAJOR else (nl, nl, self.nz)

    def _cells(self, t: torch.Tensor, level: int, dtype=None, name="x"):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous CUDA tensor")
        if dtype is not None and t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}")
        if tuple(t.shape) != self.cell_shape(level):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {self.cell_shape(level)}")
        return t

    @staticmethod
    def _fp32(t: torch.Tensor) -> int:
        if t.dtype == torch.float32:
            return 1
        if t.dtype == torch.float64:
            return 0
        raise ValueError("buffers must be float32 or float64")

    # -- operations --------------------------------------------------------------
    def apply(self, x: torch.Tensor, level: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
        self._cells(x, level)
        y = torch.empty_like(x) if out is None else out
        _check(lib().tpmg_apply_operator(self.handle, level, self._fp32(x), _ptr(x), _ptr(y),
                                         self.layout, _stream(self.device)),
               "tpmg_apply_operator", self.handle)
        return y

    def apply_static(self, x: torch.Tensor, level: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
        """y = H_level x staged through the library's static device array
        (no allocation inside the call; see tpmg_apply_operator_static)."""
        self._cells(x, level)
        y = torch.empty_like(x) if out is None else out
        _check(lib().tpmg_apply_operator_static(self.handle, level, self._fp32(x), _ptr(x), _ptr(y),
                                                self.layout, _stream(self.device)),
               "tpmg_apply_operator_static", self.handle)
        return y

    def vcycle(self, b: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._cells(b, 0, name="b")
        z = torch.empty_like(b) if out is None else out
        _check(lib().tpmg_vcycle(self.handle, self._fp32(b), _ptr(b), _ptr(z), self.layout,
                                 _stream(self.device)), "tpmg_vcycle", self.handle)
        return z

    def solve(self, b: torch.Tensor, rtol: float = 1e-8, maxit: int = 100,
              x0: torch.Tensor | None = None, flexible: bool | None = None,
              out: torch.Tensor | None = None, history: bool = False, omega_alt: float = 0.0):
        """Returns (x, info dict).  Raises on breakdown or argument errors.
        omega_alt > 0: V-cycles with an odd index use that damping (a
        deliberately variable preconditioner)."""
        import numpy as np
        self._cells(b, 0, torch.float64, "b")
        if x0 is not None:
            self._cells(x0, 0, torch.float64, "x0")
            x = x0.clone() if out is None else out.copy_(x0)
        else:
            x = torch.empty_like(b) if out is None else out
        opts = SolveOpts()
        opts.rtol, opts.maxit = float(rtol), int(maxit)
        opts.x0_nonzero = 1 if x0 is not None else 0
        opts.flexible = int(self.mixed if flexible is None else bool(flexible))
        opts.omega_alt = float(omega_alt)
        hist = np.zeros(maxit + 1) if history else None
        opts.history = hist.ctypes.data_as(C.c_void_p) if hist is not None else None
        info = SolveInfo()
        st = lib().tpmg_solve(self.handle, _ptr(b), _ptr(x), self.layout, C.byref(opts),
                              C.byref(info), _stream(self.device))
        _check(st, "tpmg_solve", self.handle, ok=(OK, NOT_CONVERGED))
        res = dict(iterations=info.iterations, converged=bool(info.converged),
                   rel_residual=info.rel_residual, true_rel_residual=info.true_rel_residual,
                   status=st)
        if hist is not None:
            res["history"] = hist[: info.iterations + 1].copy()
        return x, res

    def face_gradient(self, lam: torch.Tensor, x: torch.Tensor,
                      out: torch.Tensor | None = None) -> torch.Tensor:
        self._cells(lam, 0, torch.float64, "lambda")
        self._cells(x, 0, torch.float64, "x")
        shape = (3, self.nz, self.n, self.n) if self.layout == LEVEL_MAJOR else (self.n, self.n, self.nz, 3)
        g = torch.empty(shape, dtype=torch.float64, device=self.device) if out is None else out
        _check(lib().tpmg_face_gradient(self.handle, _ptr(lam), _ptr(x), _ptr(g), self.layout,
                                        _stream(self.device)), "tpmg_face_gradient", self.handle)
        return g

    # -- V-cycle components (level-major buffers) ----------------------------------
    def smooth(self, b: torch.Tensor, u: torch.Tensor | None = None, level: int = 0) -> torch.Tensor:
        out = torch.empty_like(b)
        _check(lib().tpmg_smooth(self.handle, level, self._fp32(b), _ptr(u) if u is not None else None,
                                 _ptr(b), _ptr(out), _stream(self.device)), "tpmg_smooth", self.handle)
        return out

    def residual_restrict(self, u: torch.Tensor, b: torch.Tensor, level: int = 0) -> torch.Tensor:
        nc = self.level_n(level + 1)
        out = torch.empty((self.nz, nc, nc), dtype=b.dtype, device=self.device)
        _check(lib().tpmg_residual_restrict(self.handle, level, self._fp32(b), _ptr(u), _ptr(b), _ptr(out),
                                            _stream(self.device)), "tpmg_residual_restrict", self.handle)
        return out

    def prolong_smooth(self, u: torch.Tensor, e: torch.Tensor, b: torch.Tensor, level: int = 0) -> torch.Tensor:
        out = torch.empty_like(u)
        _check(lib().tpmg_prolong_smooth(self.handle, level, self._fp32(b), _ptr(u), _ptr(e), _ptr(b),
                                         _ptr(out), _stream(self.device)), "tpmg_prolong_smooth", self.handle)
        return out

    def coarse_solve(self, b: torch.Tensor) -> torch.Tensor:
        out = torch.empty_like(b)
        _check(lib().tpmg_coarse_solve(self.handle, self._fp32(b), _ptr(b), _ptr(out), _stream(self.device)),
               "tpmg_coarse_solve", self.handle)
        return out

    def level_coefficients(self, level: int, fp32: bool = False) -> torch.Tensor:
        nl = self.level_n(level)
        out = torch.empty((3, self.nz, nl, nl), dtype=torch.float32 if fp32 else torch.float64,
                          device=self.device)
        _check(lib().tpmg_level_coefficients(self.handle, level, int(fp32), _ptr(out), _stream(self.device)),
               "tpmg_level_coefficients", self.handle)
        return out

    # -- velocity-pressure system (finest level, FP64, level-major) -------------------
    def _mixed_vec(self, t: torch.Tensor, name: str):
        shape = (4, self.nz, self.n, self.n)
        if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64 and tuple(t.shape) == shape):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {shape}")
        if self.layout != LEVEL_MAJOR:
            raise ValueError("the velocity-pressure system is level-major only")
        return t

    def mixed_apply(self, x: torch.Tensor) -> torch.Tensor:
        """y = A x for x = [u_E, u_N, u_U, p] stacked as (4, nz, n, n)."""
        self._mixed_vec(x, "x")
        y = torch.empty_like(x)
        _check(lib().tpmg_mixed_apply(self.handle, _ptr(x), _ptr(y), _stream(self.device)), "tpmg_mixed_apply",
               self.handle)
        return y

    def mixed_precondition(self, r: torch.Tensor, fp32: bool | None = None) -> torch.Tensor:
        """z = P^{-1} r (Schur-complement factorisation, one V-cycle)."""
        self._mixed_vec(r, "r")
        z = torch.empty_like(r)
        f32 = self.mixed if fp32 is None else bool(fp32)
        _check(lib().tpmg_mixed_precondition(self.handle, int(f32), _ptr(r), _ptr(z), _stream(self.device)),
               "tpmg_mixed_precondition", self.handle)
        return z

    def mixed_workspace_bytes(self, restart: int = 30) -> int:
        nb = C.c_size_t(0)
        _check(lib().tpmg_mixed_workspace_bytes(self.handle, int(restart), C.byref(nb)),
               "tpmg_mixed_workspace_bytes", self.handle)
        return nb.value

    def mixed_solve(self, b: torch.Tensor, rtol: float = 1e-5, restart: int = 30, maxit: int = 300,
                    history: bool = False, workspace: torch.Tensor | None = None):
        """Restarted flexible GMRES on A x = b with the Schur-complement
        preconditioner.  Returns (x, info dict)."""
        import numpy as np
        self._mixed_vec(b, "b")
        x = torch.empty_like(b)
        need = self.mixed_workspace_bytes(restart)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        opts = MixedOpts()
        opts.rtol, opts.restart, opts.maxit = float(rtol), int(restart), int(maxit)
        hist = np.zeros(maxit + 1) if history else None
        opts.history = hist.ctypes.data_as(C.c_void_p) if hist is not None else None
        info = SolveInfo()
        st = lib().tpmg_mixed_solve(self.handle, _ptr(b), _ptr(x), _ptr(workspace), need, C.byref(opts),
                                    C.byref(info), _stream(self.device))
        _check(st, "tpmg_mixed_solve", self.handle, ok=(OK, NOT_CONVERGED))
        res = dict(iterations=info.iterations, converged=bool(info.converged), rel_residual=info.rel_residual,
                   true_rel_residual=info.true_rel_residual, status=st)
        if hist is not None:
            res["history"] = hist[: info.iterations + 1].copy()
        return x, res

    # -- profiling ------------------------------------------------------------------
    def profile_enable(self, on: bool = True, levels: bool = False):
        """Event timers: kernel classes, and with levels=True every launch per
        V-cycle level too."""
        mode = (2 if levels else 1) if on else 0
        _check(lib().tpmg_profile_enable(self.handle, mode), "tpmg_profile_enable", self.handle)

    def profile_read(self, kernel_class: int):
        ms, n = C.c_double(0), C.c_int64(0)
        _check(lib().tpmg_profile_read(self.handle, kernel_class, C.byref(ms), C.byref(n)),
               "tpmg_profile_read", self.handle)
        return ms.value, n.value

    def profile_read_level(self, level: int):
        """(total ms, launches) of the kernels on one V-cycle level."""
        ms, n = C.c_double(0), C.c_int64(0)
        _check(lib().tpmg_profile_read_level(self.handle, level, C.byref(ms), C.byref(n)),
               "tpmg_profile_read_level", self.handle)
        return ms.value, n.value


class DG1Level:
    """The next-to-lowest-order (DG1) pressure level on the finest grid of a
    level-major hierarchy (tpmg_dg1_*): the band LU of every column block is
    formed at construction; the operator, line solve, sweeps, p-transfers,
    NLO V-cycle and CG then run on it.  DG1 arrays are contiguous float64 CUDA
    tensors of shape (6, nz, n, n), unknown a = 3 v + h of cell (i, j, k);
    lowest-order arrays are (nz, n, n).  Calls must not overlap other calls
    on the same hierarchy."""

    def __init__(self, H: Hierarchy):
        if H.layout != LEVEL_MAJOR:
            raise ValueError("the DG1 level needs a level-major hierarchy")
        self.H, self.n, self.nz, self.device = H, H.n, H.nz, H.device
        nb = C.c_size_t(0)
        _check(lib().tpmg_dg1_workspace_bytes(H.handle, C.byref(nb)), "tpmg_dg1_workspace_bytes", H.handle)
        self.ws_bytes = nb.value
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=H.device)
        g = C.c_void_p()
        _check(lib().tpmg_dg1_setup(H.handle, _ptr(self.workspace), self.ws_bytes, _stream(H.device),
                                    C.byref(g)), "tpmg_dg1_setup", H.handle)
        self._g = g

    def close(self):
        g = getattr(self, "_g", None)
        if g is not None and g.value:
            lib().tpmg_dg1_destroy(g)
        self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._g is None:
            raise RuntimeError("DG1 level is closed")
        return self._g

    @property
    def shape(self):
        return (6, self.nz, self.n, self.n)

    def _vec(self, t: torch.Tensor, name: str, shape=None):
        shape = self.shape if shape is None else shape
        if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64 and tuple(t.shape) == shape):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {shape}")
        return t

    def _unary(self, fn: str, x: torch.Tensor) -> torch.Tensor:
        self._vec(x, "x")
        y = torch.empty_like(x)
        _check(getattr(lib(), fn)(self.handle, _ptr(x), _ptr(y), _stream(self.device)), fn, self.H.handle)
        return y

    def apply(self, x: torch.Tensor) -> torch.Tensor:
        """y = H1 x."""
        return self._unary("tpmg_dg1_apply", x)

    def line_solve(self, r: torch.Tensor) -> torch.Tensor:
        """x = H1_z^{-1} r in every column (forward / back substitution)."""
        return self._unary("tpmg_dg1_line_solve", r)

    def vcycle(self, b: torch.Tensor) -> torch.Tensor:
        """z = V1 b, the NLO V-cycle from a zero guess."""
        return self._unary("tpmg_dg1_vcycle", b)

    def smooth(self, b: torch.Tensor, u: torch.Tensor | None = None) -> torch.Tensor:
        self._vec(b, "b")
        if u is not None:
            self._vec(u, "u")
        out = torch.empty_like(b)
        _check(lib().tpmg_dg1_smooth(self.handle, _ptr(u) if u is not None else None, _ptr(b), _ptr(out),
                                     _stream(self.device)), "tpmg_dg1_smooth", self.H.handle)
        return out

    def residual_restrict(self, u: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        """b0 = R1 (b - H1 u) on the lowest-order level 0."""
        self._vec(u, "u")
        self._vec(b, "b")
        out = torch.empty((self.nz, self.n, self.n), dtype=torch.float64, device=self.device)
        _check(lib().tpmg_dg1_residual_restrict(self.handle, _ptr(u), _ptr(b), _ptr(out), _stream(self.device)),
               "tpmg_dg1_residual_restrict", self.H.handle)
        return out

    def prolong_add(self, e0: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
        """u + P1 e0 (u is not modified; a new tensor is returned)."""
        self._vec(e0, "e0", (self.nz, self.n, self.n))
        out = self._vec(u, "u").clone()
        _check(lib().tpmg_dg1_prolong_add(self.handle, _ptr(e0), _ptr(out), _stream(self.device)),
               "tpmg_dg1_prolong_add", self.H.handle)
        return out

    def factors(self) -> torch.Tensor:
        """Band factors, shape (n, n, 6 nz, 11): [j, i, row r = 6 k + a, entry]
        with L(r, r-5..r-1), U(r, r), U(r, r+1..r+5)."""
        out = torch.empty((self.n, self.n, 6 * self.nz, 11), dtype=torch.float64, device=self.device)
        _check(lib().tpmg_dg1_factors(self.handle, _ptr(out), _stream(self.device)), "tpmg_dg1_factors",
               self.H.handle)
        return out

    def solve(self, b: torch.Tensor, rtol: float = 1e-8, maxit: int = 100, flexible: bool | None = None,
              history: bool = False):
        """CG on H1 x = b from x = 0, one NLO V-cycle per iteration.
        Returns (x, info dict)."""
        import numpy as np
        self._vec(b, "b")
        x = torch.empty_like(b)
        opts = SolveOpts()
        opts.rtol, opts.maxit = float(rtol), int(maxit)
        opts.x0_nonzero = 0
        opts.flexible = int(self.H.mixed if flexible is None else bool(flexible))
        opts.omega_alt = 0.0
        hist = np.zeros(maxit + 1) if history else None
        opts.history = hist.ctypes.data_as(C.c_void_p) if hist is not None else None
        info = SolveInfo()
        st = lib().tpmg_dg1_solve(self.handle, _ptr(b), _ptr(x), C.byref(opts), C.byref(info),
                                  _stream(self.device))
        _check(st, "tpmg_dg1_solve", self.H.handle, ok=(OK, NOT_CONVERGED))
        res = dict(iterations=info.iterations, converged=bool(info.converged), rel_residual=info.rel_residual,
                   true_rel_residual=info.true_rel_residual, status=st)
        if hist is not None:
            res["history"] = hist[: info.iterations + 1].copy()
        return x, res


def bandwidth_probe(dst: torch.Tensor, src: torch.Tensor):
    nbytes = src.numel() * src.element_size()
    _check(lib().tpmg_bandwidth_probe(_ptr(dst), _ptr(src), nbytes, _stream(src.device)),
           "tpmg_bandwidth_probe")


class _Solve(torch.autograd.Function):
    """x = H(c)^{-1} b with a hand-written adjoint.

    backward: lambda = H^{-1} dJ/dx (H symmetric: the same hierarchy and
    solver), dJ/dc from the fused face-gradient kernel, dJ/db = lambda."""

    @staticmethod
    def forward(ctx, c, b, hier_kw, solve_kw):
        H = Hierarchy(c.detach().contiguous(), **hier_kw)
        x, info = H.solve(b.detach().contiguous(), **solve_kw)
        if not info["converged"]:
            raise TpmgError(NOT_CONVERGED, "solve (forward)", f"not converged: {info}")
        ctx.H, ctx.solve_kw = H, solve_kw
        ctx.info = info
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        H = ctx.H
        lam, info = H.solve(gx.contiguous(), **ctx.solve_kw)
        if not info["converged"]:
            raise TpmgError(NOT_CONVERGED, "solve (adjoint)", f"not converged: {info}")
        gc = H.face_gradient(lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gc, gb, None, None


def solve(c: torch.Tensor, b: torch.Tensor, rtol: float = 1e-8, maxit: int = 100, **hier_kw) -> torch.Tensor:
    """Differentiable solve of H(c) x = b (see Hierarchy for the keyword arguments)."""
    return _Solve.apply(c, b, hier_kw, dict(rtol=rtol, maxit=maxit))
