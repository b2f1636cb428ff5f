"""Plain FP64 CPU oracle for the multigrid elasticity solve (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  It shares no code with the GPU
library (``paper_2001_04789_amd``) and never imports it; the GPU library never
imports this package.  Its inputs come from ``synth`` (problem data only).

What it computes, in the paper's order (arXiv 2001.04789):
  * the discrete operator D_H, its right-hand side -(D(0) + b) with the
    boundary operators of Sec. 2.1 (Dirichlet u0, traction t0, Neumann
    normal derivative du0), the stress
    sigma = C(grad u - eps0), the Jacobi relaxation of Sec. 3.1 and the
    transfers of Sec. 3.2 -- in ``emg_oracle.c``, one plain loop each;
  * the multigrid hierarchy (levels -1, -2, ... of Fig. "hierarchy", Sec. 3.1)
    and the correction-scheme V- and F-cycles, written here step by step;
  * the exact solution of the discrete system on tiny grids, by a dense
    solve of the matrix assembled column by column from unit vectors.

The stopping rule and residual norm are the readings listed in the design
notes: relative 2-norm of the residual over non-Dirichlet rows, relative to
the residual of the Dirichlet lift.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "emg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DIRICHLET, TRACTION, PERIODIC, NEUMANN = 0, 1, 2, 3
ISO, ANISO = 0, 1
ROW_INTERIOR, ROW_TRACTION, ROW_DIRICHLET, ROW_NEUMANN = 0, 1, 2, 3
_BC = {"dirichlet": DIRICHLET, "traction": TRACTION, "periodic": PERIODIC, "neumann": NEUMANN}


# -O3 for the host's instruction set.  The oracle is built where the sources
# are and may run on another host, so -march=native of the build host could
# fault there: two builds are made, x86-64-v4 (AVX-512) and x86-64-v3 (AVX2,
# FMA), and the one the running CPU supports is loaded.
_LIB_V4 = os.path.join(_HERE, "liboracle_v4.so")
_BASE_FLAGS = ["-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99"]
_V4_CPU_FLAGS = ("avx512f", "avx512dq", "avx512cd", "avx512bw", "avx512vl")


def _cpu_has_v4() -> bool:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("flags"):
                    have = set(line.split(":", 1)[1].split())
                    return all(f in have for f in _V4_CPU_FLAGS)
    except OSError:
        pass
    return False


def _variants():
    return [(_LIB, "x86-64-v3"), (_LIB_V4, "x86-64-v4")]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP only splits node loops), in both
    instruction-set variants; returns the one this CPU loads."""
    for path, march in _variants():
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            tmp = path + f".tmp{os.getpid()}"
            subprocess.check_call(["gcc"] + _BASE_FLAGS + ["-march=" + march, "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB_V4 if _cpu_has_v4() else _LIB


def build_flags() -> List[str]:
    """gcc flags of the variant this CPU loads."""
    return _BASE_FLAGS + ["-march=" + ("x86-64-v4" if _cpu_has_v4() else "x86-64-v3")]


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's node loops (omp_set_num_threads)."""
    fn = lib().omp_set_num_threads
    fn.argtypes = [ctypes.c_int]
    fn.restype = None
    fn(int(n))


def max_threads() -> int:
    fn = lib().omp_get_max_threads
    fn.restype = ctypes.c_int
    return int(fn())


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("m", ctypes.c_int * 3), ("h", ctypes.c_double * 3),
                ("bc", ctypes.c_int * 6), ("kind", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        g = P(_Grid)
        sig = {
            "ora_apply": [g, dp, dp, dp],
            "ora_diag": [g, dp, dp],
            "ora_row_class": [g, P(ctypes.c_int)],
            "ora_rhs": [g, dp, dp, dp, P(dp), dp],
            "ora_stress": [g, dp, dp, dp, dp],
            "ora_residual": [g, dp, dp, dp, dp],
            "ora_jacobi": [g, dp, dp, dp, ctypes.c_double, dp],
            "ora_restrict": [g, g, dp, dp],
            "ora_prolong_add": [g, g, dp, dp],
            "ora_coarsen_moduli": [g, g, dp, dp],
            "ora_norm2": [g, dp],
        }
        for name, args in sig.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_double if name == "ora_norm2" else None
    return _lib


class Grid:
    """One level of the node grid: stored node counts m, spacing h, face BCs."""

    def __init__(self, dim, m, h, bc, kind):
        self.dim, self.m, self.h, self.bc, self.kind = dim, tuple(m), tuple(h), tuple(bc), kind
        self._c = _Grid(dim, (ctypes.c_int * 3)(*self.m), (ctypes.c_double * 3)(*self.h),
                        (ctypes.c_int * 6)(*self.bc), kind)

    @classmethod
    def of(cls, prob) -> "Grid":
        bc = [_BC[b] for b in prob.bc]
        for f in range(2 * prob.dim, 6):
            bc[f] = PERIODIC
        return cls(prob.dim, prob.m, prob.h, bc, ISO if prob.kind == "iso" else ANISO)

    @property
    def N(self) -> int:
        return self.m[0] * self.m[1] * self.m[2]

    @property
    def ncomp_moduli(self) -> int:
        return 2 if self.kind == ISO else (21 if self.dim == 3 else 6)

    def periodic(self, a) -> bool:
        return self.bc[2 * a] == PERIODIC

    def can_coarsen(self) -> bool:
        """All axes halve together while every non-periodic axis has an even
        cell count >= 8 (the coarse axis keeps >= 5 nodes, so it still has
        interior nodes between its boundary rows) and every periodic axis an
        even node count >= 8."""
        for a in range(self.dim):
            if self.periodic(a):
                if self.m[a] % 2 or self.m[a] < 8:
                    return False
            else:
                cells = self.m[a] - 1
                if cells % 2 or cells < 8:
                    return False
        return True

    def coarse(self) -> "Grid":
        m = [1, 1, 1]
        for a in range(self.dim):
            m[a] = self.m[a] // 2 if self.periodic(a) else (self.m[a] - 1) // 2 + 1
        h = [2 * self.h[a] if a < self.dim else self.h[a] for a in range(3)]
        return Grid(self.dim, m, h, self.bc, self.kind)

    def shape(self, comps):
        return (comps, self.m[2], self.m[1], self.m[0])

    def ptr(self):
        return ctypes.byref(self._c)


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ---- one-call wrappers of the C primitives ----

def apply(g: Grid, C, u):
    C, u = _c(C), _c(u)
    out = np.empty(g.shape(g.dim))
    lib().ora_apply(g.ptr(), _dp(C), _dp(u), _dp(out))
    return out


def diag(g: Grid, C):
    C = _c(C)
    out = np.empty(g.shape(g.dim))
    lib().ora_diag(g.ptr(), _dp(C), _dp(out))
    return out


def row_class(g: Grid):
    out = np.empty(g.N, dtype=np.int32)
    lib().ora_row_class(g.ptr(), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return out.reshape(g.m[2], g.m[1], g.m[0])


def rhs(g: Grid, C, eps0=None, b=None, face=None):
    C, eps0, b = _c(C), _c(eps0), _c(b)
    faces = [(_c(face.get(f)) if face else None) for f in range(6)]
    arr = (ctypes.POINTER(ctypes.c_double) * 6)(*[_dp(x) for x in faces])
    out = np.empty(g.shape(g.dim))
    lib().ora_rhs(g.ptr(), _dp(C), _dp(eps0), _dp(b), arr, _dp(out))
    return out


def stress(g: Grid, C, eps0, u):
    C, eps0, u = _c(C), _c(eps0), _c(u)
    out = np.empty(g.shape(6 if g.dim == 3 else 3))
    lib().ora_stress(g.ptr(), _dp(C), _dp(eps0), _dp(u), _dp(out))
    return out


def von_mises(sigma):
    """Von Mises stress sqrt(3/2 S_ij S_ij), S the deviator of the stress
    (Sec. 4.3, von Mises definition), per node from the 3D Voigt-ordered
    stress [11, 22, 33, 23, 31, 12] (shape (6, ...)): the full symmetric
    tensor is rebuilt and its trace removed, written out as the definition."""
    s = np.asarray(sigma, dtype=np.float64)
    assert s.shape[0] == 6, "3D Voigt stress expected"
    T = np.empty((3, 3) + s.shape[1:])
    T[0, 0], T[1, 1], T[2, 2] = s[0], s[1], s[2]
    T[1, 2] = T[2, 1] = s[3]
    T[2, 0] = T[0, 2] = s[4]
    T[0, 1] = T[1, 0] = s[5]
    tr = T[0, 0] + T[1, 1] + T[2, 2]
    S = T.copy()
    for i in range(3):
        S[i, i] = S[i, i] - tr / 3.0
    return np.sqrt(1.5 * np.sum(S * S, axis=(0, 1)))


def residual(g: Grid, C, u, f):
    C, u, f = _c(C), _c(u), _c(f)
    out = np.empty(g.shape(g.dim))
    lib().ora_residual(g.ptr(), _dp(C), _dp(u), _dp(f), _dp(out))
    return out


def jacobi(g: Grid, C, u, f, omega):
    C, u, f = _c(C), _c(u), _c(f)
    out = np.empty(g.shape(g.dim))
    lib().ora_jacobi(g.ptr(), _dp(C), _dp(u), _dp(f), float(omega), _dp(out))
    return out


def restrict(gf: Grid, gc: Grid, r):
    r = _c(r)
    out = np.empty(gc.shape(gf.dim))
    lib().ora_restrict(gf.ptr(), gc.ptr(), _dp(r), _dp(out))
    return out


def prolong_add(gc: Grid, gf: Grid, e, u):
    """Returns u + P e (u is not modified)."""
    e = _c(e)
    out = np.array(u, dtype=np.float64, order="C", copy=True)
    lib().ora_prolong_add(gc.ptr(), gf.ptr(), _dp(e), _dp(out))
    return out


def coarsen_moduli(gf: Grid, gc: Grid, C):
    C = _c(C)
    out = np.empty(gc.shape(gf.ncomp_moduli))
    lib().ora_coarsen_moduli(gf.ptr(), gc.ptr(), _dp(C), _dp(out))
    return out


def norm(g: Grid, r) -> float:
    return float(np.sqrt(lib().ora_norm2(g.ptr(), _dp(_c(r)))))


# ---- hierarchy, dense matrices and the V-cycle ----

def hierarchy(g: Grid) -> List[Grid]:
    levels = [g]
    while levels[-1].can_coarsen():
        levels.append(levels[-1].coarse())
    return levels


def dense_matrix(g: Grid, C) -> np.ndarray:
    """Matrix of D_H assembled column by column (unit vectors); tiny grids only."""
    n = g.dim * g.N
    A = np.empty((n, n))
    e = np.zeros(n)
    for q in range(n):
        e[q] = 1.0
        A[:, q] = apply(g, C, e.reshape(g.shape(g.dim))).ravel()
        e[q] = 0.0
    return A


def dirichlet_mask(g: Grid) -> np.ndarray:
    return np.broadcast_to(row_class(g) == ROW_DIRICHLET, g.shape(g.dim))


class Hierarchy:
    """Levels 0 (finest), -1, -2, ...: grids, coarsened moduli and the dense
    factorisation of the coarsest operator."""

    def __init__(self, g: Grid, C):
        import scipy.linalg
        self.grids = hierarchy(g)
        self.C = [_c(C)]
        for ell in range(1, len(self.grids)):
            self.C.append(coarsen_moduli(self.grids[ell - 1], self.grids[ell], self.C[-1]))
        gb = self.grids[-1]
        self.bottom = scipy.linalg.lu_factor(dense_matrix(gb, self.C[-1]))

    def bottom_solve(self, f):
        import scipy.linalg
        gb = self.grids[-1]
        return scipy.linalg.lu_solve(self.bottom, f.ravel()).reshape(gb.shape(gb.dim))


def vcycle(H: Hierarchy, ell: int, x, f, nu1=2, nu2=2, omega=2.0 / 3.0, counts=None):
    """One correction-scheme V-cycle on level ell (Sec. 3.1): nu1 damped
    Jacobi sweeps, residual, full-weighting restriction, recursive solve of
    the coarse correction from zero, interpolation, nu2 sweeps.  The coarsest
    level is solved exactly.  Returns the new x.  `counts[l]`, if given,
    gathers the Jacobi sweeps run on each level."""
    g, C = H.grids[ell], H.C[ell]
    if ell == len(H.grids) - 1:
        return H.bottom_solve(f)
    for _ in range(nu1):
        x = jacobi(g, C, x, f, omega)
    r = residual(g, C, x, f)
    gc = H.grids[ell + 1]
    fc = restrict(g, gc, r)
    ec = vcycle(H, ell + 1, np.zeros(gc.shape(g.dim)), fc, nu1, nu2, omega, counts)
    x = prolong_add(gc, g, ec, x)
    for _ in range(nu2):
        x = jacobi(g, C, x, f, omega)
    if counts is not None:
        counts[ell] += nu1 + nu2
    return x


def fcycle(H: Hierarchy, ell: int, x, f, nu1=2, nu2=2, omega=2.0 / 3.0, counts=None):
    """One F-cycle on level ell (Sec. 3.1 names F-cycles as the solver's
    cycle; the recursive form of the multigrid literature it cites): nu1
    sweeps, residual, restriction, then on the coarse level an F-cycle from
    zero followed by a V-cycle from that result, interpolation, nu2 sweeps.
    The coarsest level is solved exactly.  `counts[l]`, if given, gathers
    the Jacobi sweeps run on each level."""
    g, C = H.grids[ell], H.C[ell]
    if ell == len(H.grids) - 1:
        return H.bottom_solve(f)
    for _ in range(nu1):
        x = jacobi(g, C, x, f, omega)
    r = residual(g, C, x, f)
    gc = H.grids[ell + 1]
    fc = restrict(g, gc, r)
    ec = fcycle(H, ell + 1, np.zeros(gc.shape(g.dim)), fc, nu1, nu2, omega, counts)
    ec = vcycle(H, ell + 1, ec, fc, nu1, nu2, omega, counts)
    x = prolong_add(gc, g, ec, x)
    for _ in range(nu2):
        x = jacobi(g, C, x, f, omega)
    if counts is not None:
        counts[ell] += nu1 + nu2
    return x


class SolveResult:
    def __init__(self, u, cycles, history, seconds, rhs_, converged):
        self.u, self.cycles, self.history, self.seconds, self.rhs, self.converged = \
            u, cycles, history, seconds, rhs_, converged

    @property
    def rel_res(self):
        return self.history[-1]


def solve(prob, tol: float = 1e-13, max_cycles: int = 200, nu1: int = 2, nu2: int = 2,
          omega: float = 2.0 / 3.0, H: Optional[Hierarchy] = None, stagnation: float = 0.95,
          cycle: str = "V") -> SolveResult:
    """V-cycles (or F-cycles, cycle="F") from the Dirichlet lift until the
    relative residual (2-norm over non-Dirichlet rows, relative to the lift's
    residual) is <= tol, or until it stops decreasing (ratio > stagnation
    over 3 cycles once below 1e-11, i.e. at rounding level)."""
    step = {"V": vcycle, "F": fcycle}[cycle]
    g = Grid.of(prob)
    t0 = time.perf_counter()
    if H is None:
        H = Hierarchy(g, prob.C)
    f = rhs(g, H.C[0], prob.eps0, prob.b, prob.face)
    dmask = dirichlet_mask(g)
    u = np.where(dmask, f, 0.0)
    r0 = norm(g, residual(g, H.C[0], u, f))
    hist = [1.0]
    if r0 == 0.0:
        return SolveResult(u, 0, hist, time.perf_counter() - t0, f, True)
    cycles = 0
    converged = False
    while cycles < max_cycles:
        u = step(H, 0, u, f, nu1, nu2, omega)
        cycles += 1
        rel = norm(g, residual(g, H.C[0], u, f)) / r0
        hist.append(rel)
        if rel <= tol:
            converged = True
            break
        if rel < 1e-11 and len(hist) > 3 and hist[-1] > stagnation * hist[-4]:
            break
    return SolveResult(u, cycles, hist, time.perf_counter() - t0, f, converged)


def dense_solve(prob) -> np.ndarray:
    """Exact discrete solution by a dense solve (tiny grids only)."""
    g = Grid.of(prob)
    C = _c(prob.C)
    A = dense_matrix(g, C)
    f = rhs(g, C, prob.eps0, prob.b, prob.face)
    return np.linalg.solve(A, f.ravel()).reshape(g.shape(g.dim))
