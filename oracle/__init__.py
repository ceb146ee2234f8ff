"""Python access to the plain CPU oracle (``liboracle.so``, built from C).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use this package; the GPU library and its binding never import it.

Arrays cross this interface in the logical layout: cells as (nz, n, n) and
faces as (3, nz, n, n) with f in {E, N, U}, i fastest.  The oracle itself
stores columns contiguously (cell (i,j,k) at (j*n+i)*nz+k); the conversion
below is plain reshaping.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "tpmg_oracle.c"), os.path.join(_HERE, "oracle_level.inc"),
        os.path.join(_HERE, "oracle_mixed.inc"), os.path.join(_HERE, "oracle_dg1.inc")]


# Portable optimised build: the library is built on one host and may be loaded
# on another, so it targets x86-64-v3 (AVX2, FMA) rather than the build host.
# Floating-point contraction stays off, so every operation rounds as written.
CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-std=c11", "-fPIC", "-shared"]
# Build tuned for the host that runs it (for timing the oracle on that host).
NATIVE_CFLAGS = ["-O3", "-march=native", "-ffp-contract=off", "-fopenmp", "-std=c11", "-fPIC", "-shared"]


def build(force: bool = True, path: str = LIB_PATH, native: bool = False) -> str:
    """Compile the oracle library with gcc (plain C, no GPU code)."""
    if not force and os.path.exists(path):
        return path
    tmp = path + ".tmp"
    flags = NATIVE_CFLAGS if native else CFLAGS
    subprocess.check_call(["gcc", *flags, "-o", tmp, _SRC[0], "-lm"])
    os.replace(tmp, path)
    return path


def use_library(path: str) -> None:
    """Load the oracle from another build of the same sources (e.g. native)."""
    global _lib, LIB_PATH
    LIB_PATH = path
    _lib = None


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.oracle_create.restype = vp
        L.oracle_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, vp,
                                    _dp, _dp, _dp, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int]
        L.oracle_destroy.argtypes = [vp]
        L.oracle_threads.argtypes = [C.c_int]
        L.oracle_threads.restype = C.c_int
        L.oracle_level_n.argtypes = [vp, C.c_int]
        L.oracle_level_n.restype = C.c_int
        L.oracle_get_coeffs.argtypes = [vp, C.c_int, _dp, _dp, _dp]
        for name, p in [("", _dp), ("_f", _fp)]:
            for fn in ("apply", "line_solve", "restrict", "prolong_add"):
                getattr(L, f"oracle_{fn}{name}").argtypes = [vp, C.c_int, p, p]
            getattr(L, f"oracle_smooth{name}").argtypes = [vp, C.c_int, p, p, p]
            getattr(L, f"oracle_vcycle{name}").argtypes = [vp, p, p]
            getattr(L, f"oracle_coarse_solve{name}").argtypes = [vp, p, p]
        L.oracle_dense.argtypes = [vp, C.c_int, _dp]
        L.oracle_pcg.argtypes = [vp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int,
                                 C.c_double, vp, _dp, vp, vp]
        L.oracle_pcg.restype = C.c_int
        L.oracle_face_gradient.argtypes = [vp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_mixed_apply.argtypes = [vp, _dp, _dp]
        L.oracle_mixed_precondition.argtypes = [vp, C.c_int, _dp, _dp]
        L.oracle_mixed_fgmres.argtypes = [vp, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int, vp, _dp]
        L.oracle_mixed_fgmres.restype = C.c_int
        L.oracle_dg1_create.restype = vp
        L.oracle_dg1_create.argtypes = [vp]
        L.oracle_dg1_destroy.argtypes = [vp]
        for fn in ("apply", "line_solve"):
            getattr(L, f"oracle_dg1_{fn}").argtypes = [vp, _dp, _dp]
        L.oracle_dg1_smooth.argtypes = [vp, vp, _dp, _dp]
        L.oracle_dg1_restrict.argtypes = [vp, _dp, _dp]
        L.oracle_dg1_prolong_add.argtypes = [vp, _dp, _dp]
        L.oracle_dg1_vcycle.argtypes = [vp, _dp, _dp]
        L.oracle_dg1_column_block.argtypes = [vp, C.c_int, C.c_int, _dp]
        L.oracle_dg1_factors.argtypes = [vp, _dp]
        L.oracle_dg1_dense.argtypes = [vp, _dp]
        L.oracle_dg1_pcg.argtypes = [vp, _dp, _dp, C.c_double, C.c_int, vp, _dp]
        L.oracle_dg1_pcg.restype = C.c_int
        _lib = L
    return _lib


def threads(n: int = 0) -> int:
    """Set the oracle's OpenMP thread count (n > 0) and return the count in use."""
    return int(lib().oracle_threads(int(n)))


def to_columns(a: np.ndarray) -> np.ndarray:
    """(nz, n, n) -> column-contiguous flat array [(j*n+i)*nz + k]."""
    return np.ascontiguousarray(np.transpose(a, (1, 2, 0))).reshape(-1)


def from_columns(a: np.ndarray, n: int, nz: int) -> np.ndarray:
    return np.ascontiguousarray(a.reshape(n, n, nz).transpose(2, 0, 1))


class Problem:
    """The oracle's multigrid hierarchy for one set of face coefficients."""

    def __init__(self, c, a_h=1.0, a_z=1.0, dz=None, levels=1, nu=(2, 2), omega=0.8,
                 coarse="smooth", n_coarse=2):
        c = np.asarray(c, dtype=np.float64)
        assert c.ndim == 4 and c.shape[0] == 3 and c.shape[2] == c.shape[3]
        self.nz, self.n = c.shape[1], c.shape[2]
        self.levels = levels
        cols = [to_columns(c[f]) for f in range(3)]
        self._dz = None if dz is None else np.ascontiguousarray(dz, dtype=np.float64)
        dzp = None if self._dz is None else self._dz.ctypes.data_as(C.c_void_p)
        self._h = lib().oracle_create(self.n, self.nz, levels, float(a_h), float(a_z), dzp,
                                      cols[0], cols[1], cols[2], int(nu[0]), int(nu[1]),
                                      float(omega), 1 if coarse == "direct" else 0, int(n_coarse))
        if not self._h:
            raise ValueError("oracle_create rejected the problem")
        self.a_h, self.a_z, self.omega = a_h, a_z, omega

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_destroy(h)
            self._h = None

    def n_at(self, level: int) -> int:
        return lib().oracle_level_n(self._h, level)

    def _col(self, x, level, dtype):
        n = self.n_at(level)
        x = np.asarray(x, dtype=dtype)
        assert x.shape == (self.nz, n, n), (x.shape, (self.nz, n, n))
        return to_columns(x), n

    def coeffs(self, level: int) -> np.ndarray:
        n = self.n_at(level)
        m = n * n * self.nz
        out = [np.empty(m) for _ in range(3)]
        lib().oracle_get_coeffs(self._h, level, *out)
        return np.stack([from_columns(o, n, self.nz) for o in out])

    def _unary(self, fn, x, level, fp32=False):
        dt = np.float32 if fp32 else np.float64
        xc, n = self._col(x, level, dt)
        y = np.empty_like(xc)
        getattr(lib(), fn + ("_f" if fp32 else ""))(self._h, level, xc, y)
        return from_columns(y, n, self.nz)

    def apply(self, x, level=0, fp32=False):
        return self._unary("oracle_apply", x, level, fp32)

    def line_solve(self, r, level=0, fp32=False):
        return self._unary("oracle_line_solve", r, level, fp32)

    def smooth(self, u, b, level=0, fp32=False):
        dt = np.float32 if fp32 else np.float64
        uc, n = self._col(u, level, dt)
        bc, _ = self._col(b, level, dt)
        out = np.empty_like(uc)
        getattr(lib(), "oracle_smooth" + ("_f" if fp32 else ""))(self._h, level, uc, bc, out)
        return from_columns(out, n, self.nz)

    def restrict(self, r, level=0, fp32=False):
        """Sum of the four children: fine level -> level+1."""
        dt = np.float32 if fp32 else np.float64
        rc, _ = self._col(r, level, dt)
        nc = self.n_at(level + 1)
        out = np.empty(nc * nc * self.nz, dtype=dt)
        getattr(lib(), "oracle_restrict" + ("_f" if fp32 else ""))(self._h, level, rc, out)
        return from_columns(out, nc, self.nz)

    def prolong_add(self, e, u, level=0, fp32=False):
        """u + P e, with e on level+1 and u on level."""
        dt = np.float32 if fp32 else np.float64
        ec, _ = self._col(e, level + 1, dt)
        uc, n = self._col(u, level, dt)
        uc = uc.copy()
        getattr(lib(), "oracle_prolong_add" + ("_f" if fp32 else ""))(self._h, level, ec, uc)
        return from_columns(uc, n, self.nz)

    def coarse_solve(self, b, fp32=False):
        dt = np.float32 if fp32 else np.float64
        bc, n = self._col(b, self.levels - 1, dt)
        out = np.empty_like(bc)
        getattr(lib(), "oracle_coarse_solve" + ("_f" if fp32 else ""))(self._h, bc, out)
        return from_columns(out, n, self.nz)

    def vcycle(self, b, fp32=False):
        dt = np.float32 if fp32 else np.float64
        bc, n = self._col(b, 0, dt)
        out = np.empty_like(bc)
        getattr(lib(), "oracle_vcycle" + ("_f" if fp32 else ""))(self._h, bc, out)
        return from_columns(out, n, self.nz)

    def dense(self, level=0) -> np.ndarray:
        """Dense H at a level, rows/columns in the logical cell order (k, j, i)."""
        n = self.n_at(level)
        m = n * n * self.nz
        A = np.empty(m * m)
        lib().oracle_dense(self._h, level, A)
        A = A.reshape(m, m)
        # column-contiguous index -> logical index permutation
        perm = to_columns(np.arange(m).reshape(self.nz, n, n))
        out = np.empty_like(A)
        out[np.ix_(perm, perm)] = A
        return out

    def pcg(self, b, rtol=1e-8, maxit=100, x0=None, mixed=False, flexible=False, omega_alt=0.0,
            trace=False):
        """Returns (x, info) with info = dict(status, iterations, rel_residual,
        true_rel_residual, history).  omega_alt > 0: V-cycles with an odd
        index use that damping (a deliberately variable preconditioner).
        trace: info also holds the direction p of every iteration and the
        residual after its update (logical layout, shape (iterations, nz, n, n))."""
        bc, n = self._col(b, 0, np.float64)
        x = to_columns(np.asarray(x0, dtype=np.float64)) if x0 is not None else np.zeros_like(bc)
        x = np.ascontiguousarray(x)
        hist = np.zeros(maxit + 1)
        info = np.zeros(3)
        m = bc.size
        tp = np.zeros(max(maxit, 1) * m) if trace else None
        tr = np.zeros(max(maxit, 1) * m) if trace else None
        vpt = (lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None)
        st = lib().oracle_pcg(self._h, bc, x, float(rtol), int(maxit), 1 if x0 is not None else 0,
                              1 if mixed else 0, 1 if flexible else 0, float(omega_alt),
                              hist.ctypes.data_as(C.c_void_p), info, vpt(tp), vpt(tr))
        it = int(info[2])
        res = dict(status=st, iterations=it, converged=st >= 0, rel_residual=info[0],
                   true_rel_residual=info[1], history=hist[: it + 1].copy())
        if trace:
            res["directions"] = np.stack([from_columns(tp[i * m:(i + 1) * m], n, self.nz) for i in range(it)])
            res["residuals"] = np.stack([from_columns(tr[i * m:(i + 1) * m], n, self.nz) for i in range(it)])
        return from_columns(x, n, self.nz), res

    def face_gradient(self, lam, x) -> np.ndarray:
        lc, n = self._col(lam, 0, np.float64)
        xc, _ = self._col(x, 0, np.float64)
        g = [np.empty_like(lc) for _ in range(3)]
        lib().oracle_face_gradient(self._h, lc, xc, *g)
        return np.stack([from_columns(o, n, self.nz) for o in g])

    # -- velocity-pressure system (faces E, N, U then pressure, stacked (4, nz, n, n)) --
    def _mixed_cols(self, x):
        x = np.asarray(x, dtype=np.float64)
        assert x.shape == (4, self.nz, self.n, self.n), x.shape
        return np.ascontiguousarray(np.concatenate([to_columns(x[f]) for f in range(4)]))

    def _mixed_logical(self, v):
        m = self.n * self.n * self.nz
        return np.stack([from_columns(v[f * m:(f + 1) * m], self.n, self.nz) for f in range(4)])

    def mixed_apply(self, x):
        xc = self._mixed_cols(x)
        y = np.empty_like(xc)
        lib().oracle_mixed_apply(self._h, xc, y)
        return self._mixed_logical(y)

    def mixed_precondition(self, r, fp32=False):
        rc = self._mixed_cols(r)
        z = np.empty_like(rc)
        lib().oracle_mixed_precondition(self._h, 1 if fp32 else 0, rc, z)
        return self._mixed_logical(z)

    def mixed_fgmres(self, b, rtol=1e-5, restart=30, maxit=300, fp32=False):
        """Returns (x, info) with info = dict(status, iterations, converged,
        rel_residual (Arnoldi estimate), true_rel_residual, history)."""
        bc = self._mixed_cols(b)
        x = np.empty_like(bc)
        hist = np.zeros(maxit + 1)
        info = np.zeros(3)
        st = lib().oracle_mixed_fgmres(self._h, bc, x, float(rtol), int(restart), int(maxit), 1 if fp32 else 0,
                                       hist.ctypes.data_as(C.c_void_p), info)
        it = int(info[2])
        return self._mixed_logical(x), dict(status=st, iterations=it, converged=st >= 0, rel_residual=info[0],
                                            true_rel_residual=info[1], history=hist[: it + 1].copy())


# -- next-to-lowest order: DG1 pressure (6 unknowns per cell) ------------------
DG1_NB, DG1_KL, DG1_KU = 6, 5, 5
DG1_NF = DG1_KL + DG1_KU + 1


def dg1_to_columns(a: np.ndarray) -> np.ndarray:
    """(6, nz, n, n) -> the oracle's order [((j*n+i)*nz + k)*6 + a]."""
    return np.ascontiguousarray(np.transpose(a, (2, 3, 1, 0))).reshape(-1)


def dg1_from_columns(a: np.ndarray, n: int, nz: int) -> np.ndarray:
    return np.ascontiguousarray(a.reshape(n, n, nz, DG1_NB).transpose(3, 2, 0, 1))


class DG1:
    """The DG1 pressure level on the finest grid of a Problem (whose DG0
    hierarchy is the coarse part of the NLO V-cycle).  Arrays in the logical
    layout (6, nz, n, n): unknown a = 3 v + h of cell (i, j, k), v = bottom /
    top value in the vertical, h = 1, xi, eta in the horizontal."""

    def __init__(self, P: Problem):
        self.P, self.n, self.nz = P, P.n, P.nz
        self._h = lib().oracle_dg1_create(P._h)
        if not self._h:
            raise ValueError("oracle_dg1_create rejected the problem")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_dg1_destroy(h)
            self._h = None

    def _in(self, x):
        x = np.asarray(x, dtype=np.float64)
        assert x.shape == (DG1_NB, self.nz, self.n, self.n), x.shape
        return dg1_to_columns(x)

    def _out(self, v):
        return dg1_from_columns(v, self.n, self.nz)

    def _unary(self, fn, x):
        xc = self._in(x)
        y = np.empty_like(xc)
        getattr(lib(), fn)(self._h, xc, y)
        return self._out(y)

    def apply(self, x):
        return self._unary("oracle_dg1_apply", x)

    def line_solve(self, r):
        return self._unary("oracle_dg1_line_solve", r)

    def vcycle(self, b):
        return self._unary("oracle_dg1_vcycle", b)

    def smooth(self, u, b):
        bc = self._in(b)
        out = np.empty_like(bc)
        uc = self._in(u) if u is not None else None
        lib().oracle_dg1_smooth(self._h, uc.ctypes.data_as(C.c_void_p) if uc is not None else None, bc, out)
        return self._out(out)

    def restrict(self, r):
        out = np.empty(self.n * self.n * self.nz)
        lib().oracle_dg1_restrict(self._h, self._in(r), out)
        return from_columns(out, self.n, self.nz)

    def prolong_add(self, e0, u):
        uc = self._in(u).copy()
        lib().oracle_dg1_prolong_add(self._h, to_columns(np.asarray(e0, dtype=np.float64)), uc)
        return self._out(uc)

    def column_block(self, i, j):
        m = DG1_NB * self.nz
        A = np.empty(m * m)
        lib().oracle_dg1_column_block(self._h, int(i), int(j), A)
        return A.reshape(m, m)

    def factors(self):
        """Band LU factors: (n, n, 6 nz, 11) indexed [j, i, row, entry], row
        r = 6 k + a, entries L(r, r-5..r-1), U(r, r), U(r, r+1..r+5)."""
        F = np.empty(self.n * self.n * DG1_NB * self.nz * DG1_NF)
        lib().oracle_dg1_factors(self._h, F)
        return F.reshape(self.n, self.n, DG1_NB * self.nz, DG1_NF)

    def dense(self):
        """Dense H1 in the logical order (a, k, j, i)."""
        M = DG1_NB * self.n * self.n * self.nz
        A = np.empty(M * M)
        lib().oracle_dg1_dense(self._h, A)
        A = A.reshape(M, M)
        perm = dg1_to_columns(np.arange(M).reshape(DG1_NB, self.nz, self.n, self.n))
        out = np.empty_like(A)
        out[np.ix_(perm, perm)] = A
        return out

    def pcg(self, b, rtol=1e-8, maxit=100):
        bc = self._in(b)
        x = np.zeros_like(bc)
        hist = np.zeros(maxit + 1)
        info = np.zeros(3)
        st = lib().oracle_dg1_pcg(self._h, bc, x, float(rtol), int(maxit), hist.ctypes.data_as(C.c_void_p), info)
        it = int(info[2])
        return self._out(x), dict(status=st, iterations=it, converged=st >= 0, rel_residual=info[0],
                                  true_rel_residual=info[1], history=hist[: it + 1].copy())


def problem_for(w, c=None, **overrides) -> Problem:
    """Oracle problem for a synthetic workload description."""
    if c is None:
        c = w.coefficients()
    kw = dict(a_h=w.a_h, a_z=w.a_z, dz=w.dz(), levels=w.levels, nu=w.nu, omega=w.omega,
              coarse=w.coarse, n_coarse=w.n_coarse)
    kw.update(overrides)
    return Problem(c, **kw)
