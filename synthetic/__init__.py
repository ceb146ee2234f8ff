"""Seeded synthetic inputs for the anisotropic pressure problem.

This module is shared by the oracle tests, the GPU parity tests and the
benchmark.  It holds no arithmetic of the solver: it only draws random
numbers and describes workloads (grid sizes, coupling scales, vertical
spacings).  Values depend only on (seed, stream, logical index), never on the
storage layout, so any layout can be produced from the same draws.

Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  The generator with state
``key`` returns, as its idx-th output (0-based), ``mix64(key + (idx+1)*G)``
with ``G = 0x9E3779B97F4A7C15`` and the published finaliser ``mix64``.
A stream is keyed by ``seed XOR (stream * G)``.

Logical indices:
  cell  (i, j, k)    -> (k * N + j) * N + i
  face  (f, i, j, k) -> ((f * nz + k) * N + j) * N + i,   f in {E=0, N=1, U=2}
so the natural array shapes are (nz, N, N) for cells and (3, nz, N, N) for
faces, with i fastest.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

SEED = 160500492
STREAM_COEFF = 1      # face coefficients c_f
STREAM_RHS = 2        # right-hand side b
STREAM_TARGET = 3     # target field x_t of the adjoint loss
STREAM_FD_FACES = 4   # faces picked for finite-difference checks
STREAM_TEST = 5       # test vectors
STREAM_MIXED_RHS = 6  # right-hand side of the velocity-pressure system
STREAM_DG1_RHS = 7    # right-hand side on the next-to-lowest-order (DG1) level

_CHUNK = 1 << 22


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    return np.uint64((seed ^ ((stream * 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF))
                     & 0xFFFFFFFFFFFFFFFF)


def splitmix64(key: int, idx: np.ndarray) -> np.ndarray:
    """idx-th output (0-based) of SplitMix64 started from state ``key``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(key) + (idx + np.uint64(1)) * GOLDEN)


def _parallel_fill(out: np.ndarray, fn) -> np.ndarray:
    n = out.size
    flat = out.reshape(-1)
    starts = list(range(0, n, _CHUNK))
    if len(starts) <= 1:
        fn(flat, 0, n)
        return out
    workers = min(len(starts), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda s: fn(flat, s, min(n, s + _CHUNK)), starts))
    return out


def uniform(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """U[0,1) draws for logical indices offset .. offset+n-1 (float64)."""
    key = _key(seed, stream)
    out = np.empty(n, dtype=np.float64)

    def fill(flat, a, b):
        idx = np.arange(offset + a, offset + b, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = _mix64(key + (idx + np.uint64(1)) * GOLDEN)
        flat[a:b] = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    return _parallel_fill(out, fill)


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    """N(0,1) draws by Box-Muller on the uniform pair (2*idx, 2*idx+1)."""
    key = _key(seed, stream)
    out = np.empty(n, dtype=np.float64)

    def fill(flat, a, b):
        idx = np.arange(a, b, dtype=np.uint64) * np.uint64(2)
        with np.errstate(over="ignore"):
            z1 = _mix64(key + (idx + np.uint64(1)) * GOLDEN)
            z2 = _mix64(key + (idx + np.uint64(2)) * GOLDEN)
        u1 = (z1 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        u2 = (z2 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        flat[a:b] = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)

    return _parallel_fill(out, fill)


@dataclass(frozen=True)
class Workload:
    """One problem instance: grid, couplings, vertical spacing, MG settings."""
    name: str
    n: int                 # periodic n x n columns
    nz: int                # cells per column
    levels: int            # multigrid levels (horizontal semi-coarsening)
    a_h: float
    a_z: float
    graded: bool           # dz_k proportional to 1.05**k (k = 0 at the bottom)
    coeff: str             # "uniform" (1 + 0.5 U) or "lognormal" (exp(0.3 g))
    coarse: str = "smooth"  # "smooth" (n_coarse sweeps) or "direct"
    n_coarse: int = 2
    nu: tuple = (2, 2)
    omega: float = 0.8
    rtol: float = 1e-8
    extra: dict = field(default_factory=dict)

    @property
    def dof(self) -> int:
        return self.n * self.n * self.nz

    def dz(self) -> np.ndarray | None:
        if not self.graded:
            return None
        return 1.05 ** np.arange(self.nz, dtype=np.float64)

    def coefficients(self, seed: int = SEED) -> np.ndarray:
        """Face coefficients c[f, k, j, i] (float64); dummy top U faces included."""
        m = 3 * self.dof
        if self.coeff == "uniform":
            c = uniform(seed, STREAM_COEFF, m)
            c *= 0.5
            c += 1.0
        elif self.coeff == "lognormal":
            c = normal(seed, STREAM_COEFF, m)
            c *= 0.3
            np.exp(c, out=c)
        else:
            raise ValueError(self.coeff)
        return c.reshape(3, self.nz, self.n, self.n)

    def rhs(self, seed: int = SEED) -> np.ndarray:
        return normal(seed, STREAM_RHS, self.dof).reshape(self.nz, self.n, self.n)

    def mixed_rhs(self, seed: int = SEED) -> np.ndarray:
        """Right-hand side of the velocity-pressure system, (4, nz, n, n): the
        E, N, U face components then the pressure; logical index
        (f * nz + k) * n^2 + j * n + i.  The U slot of the top cell holds no
        face and is 0."""
        b = normal(seed, STREAM_MIXED_RHS, 4 * self.dof).reshape(4, self.nz, self.n, self.n)
        b[2, self.nz - 1] = 0.0
        return b

    def dg1_rhs(self, seed: int = SEED) -> np.ndarray:
        """Right-hand side on the DG1 level, (6, nz, n, n): unknown a of cell
        (i, j, k) at logical index (a * nz + k) * n^2 + j * n + i."""
        return normal(seed, STREAM_DG1_RHS, 6 * self.dof).reshape(6, self.nz, self.n, self.n)

    def target(self, seed: int = SEED) -> np.ndarray:
        return normal(seed, STREAM_TARGET, self.dof).reshape(self.nz, self.n, self.n)

    def fd_faces(self, count: int, seed: int = SEED) -> np.ndarray:
        """Distinct real faces (f, k, j, i) for finite-difference checks.

        Real faces exclude the dummy U face above the top cell."""
        real = 3 * self.dof - self.n * self.n
        u = uniform(seed, STREAM_FD_FACES, 4 * count)
        picks = []
        for v in u:
            r = int(v * real)
            if r not in picks:
                picks.append(r)
            if len(picks) == count:
                break
        out = []
        nn = self.n * self.n
        for r in picks:
            if r < 2 * self.dof:
                f, rem = divmod(r, self.dof)
            else:
                f, rem = 2, r - 2 * self.dof   # U faces with k < nz-1
            k, rem = divmod(rem, nn)
            j, i = divmod(rem, self.n)
            out.append((f, k, j, i))
        return np.array(out, dtype=np.int64)


# The five workloads.  Sizes and parameters follow the problem statements;
# where they leave a choice open the choice is stated (levels of config 4).
CONFIGS = {
    "fp64_ref_32x32x16": Workload("fp64_ref_32x32x16", 32, 16, 3, 1.0, 100.0, False,
                                  "uniform", coarse="direct"),
    "fp64_512x512x64": Workload("fp64_512x512x64", 512, 64, 6, 1.0, 1e4, True, "uniform"),
    "mixed_512x512x64": Workload("mixed_512x512x64", 512, 64, 6, 1.0, 1e4, True, "uniform",
                                 extra={"precision": "mixed"}),
    "adjoint_256x256x32": Workload("adjoint_256x256x32", 256, 32, 5, 1.0, 1e3, False,
                                   "lognormal", extra={"fd_faces": 32, "fd_h": 1e-6}),
    "large_1024x1024x128": Workload("large_1024x1024x128", 1024, 128, 7, 1.0, 1e4, True,
                                    "uniform", extra={"precision": "mixed"}),
}

CONFIG_ORDER = list(CONFIGS)

# The next-to-lowest-order (DG1, six unknowns per cell) workload.  The paper's
# NLO grid has 5,120 columns of 64 layers (m = 384 unknowns per column); this
# periodic grid keeps the column (64 graded layers, m = 384) and the physics of
# the 512 x 512 x 64 workload, with 65,536 columns (25.2 M DG1 unknowns, band
# factors of 2.2 GB) so that one GPU is filled and the data is far larger than
# the last-level cache.  The lowest-order hierarchy below it has 5 levels
# (coarsest 16 x 16).
NLO_WORKLOADS = {
    "nlo_dg1_256x256x64": Workload("nlo_dg1_256x256x64", 256, 64, 5, 1.0, 1e4, True, "uniform"),
    # four times the columns (100.7 M DG1 unknowns, band factors of 8.9 GB)
    "nlo_dg1_512x512x64": Workload("nlo_dg1_512x512x64", 512, 64, 6, 1.0, 1e4, True, "uniform"),
}


def scaled(w: Workload, n: int, nz: int | None = None, levels: int | None = None,
           name: str | None = None, **kw) -> Workload:
    """Same physics on a different grid (used for bounded samples and small tests)."""
    d = dict(w.__dict__)
    d.update(n=n, nz=w.nz if nz is None else nz,
             levels=w.levels if levels is None else levels,
             name=name or f"{w.name}@{n}x{n}x{w.nz if nz is None else nz}")
    d.update(kw)
    return Workload(**d)
