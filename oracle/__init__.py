"""CPU oracle for restarted GMRES(m) with level-1 MGS, one-reduce lagged MGS,
two-reduce lagged CGS2, re-orthogonalized CGS (three reductions per step) and
two-synchronization CGS (arXiv:1809.05805, Sections II-III).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. The arithmetic lives in
``oracle_gmres.c`` (plain sequential FP64 C, built with gcc, no HIP); this
module is its ctypes wrapper plus NumPy diagnostics that read the basis and the
Hessenberg matrix the oracle dumps. It shares no code with the GPU library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_gmres.c")
_LIB = os.path.join(_HERE, "liboracle_gmres.so")
# Builds of the same source: "double" is the oracle; "long double" the
# test-only reference whose long sums (SpMV rows and length-n dot products)
# accumulate in long double (ORACLE_ACC); "openmp" a timing-only build whose
# length-n loops run on all host cores (ORACLE_OMP), never used for parity.
_BUILDS = {
    "double": (_LIB, []),
    "long double": (os.path.join(_HERE, "liboracle_gmres_ld.so"), ["-DORACLE_ACC=long double"]),
    "openmp": (os.path.join(_HERE, "liboracle_gmres_omp.so"), ["-fopenmp", "-DORACLE_OMP"]),
}
# A checking build of the oracle itself (not one of its arithmetic variants):
# AddressSanitizer and UndefinedBehaviorSanitizer, any report fatal. With
# ORACLE_SANITIZE=1 in the environment it replaces the "double" build; the
# process must then preload the sanitizer runtimes (tests/test_oracle_sanitize.py).
_SANITIZED = (os.path.join(_HERE, "liboracle_gmres_san.so"),
              ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all"])

SCHEMES = {"mgs": 0, "mgs1r": 1, "cgs2": 2, "cgs2_3r": 3, "two_synch": 4}
STATUS = {0: "ok", -1: "invalid argument", -3: "non-finite value"}


def _compile(out: str, extra: list[str]) -> None:
    tmp = out + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                    "-ffp-contract=off", *extra, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2: no FMA contraction, no vector ISA
    flags), its long-double-sum reference build and its OpenMP timing build."""
    for path, extra in _BUILDS.values():
        if force or not os.path.exists(path):
            _compile(path, extra)
    return _LIB


def build_sanitized() -> str:
    """Compile the checking build (AddressSanitizer + UBSan) of the oracle."""
    _compile(*_SANITIZED)
    return _SANITIZED[0]


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("cycles", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("breakdown", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("rel_res_true", ctypes.c_double),
                ("rel_res_est", ctypes.c_double), ("reductions", ctypes.c_int64)]


_libs: dict[str, ctypes.CDLL] = {}


def _load(acc: str = "double"):
    """The oracle library: acc "double" (the oracle), "long double" (the
    test-only reference build whose long sums carry 11 more bits) or "openmp"
    (the timing build)."""
    if acc not in _BUILDS:
        raise ValueError(acc)
    if acc not in _libs:
        path = _BUILDS[acc][0]
        if acc == "double" and os.environ.get("ORACLE_SANITIZE") == "1":
            path = _SANITIZED[0]
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_gmres_solve.restype = ctypes.c_int
        lib.oracle_gmres_solve.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, ctypes.c_int32,
                                           ctypes.c_int32, P, P, ctypes.c_double, ctypes.c_int64,
                                           ctypes.POINTER(_Info), P, P, P, P, P, P, P]
        lib.oracle_gmres_solve_depth.restype = ctypes.c_int
        lib.oracle_gmres_solve_depth.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P,
                                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 P, P, ctypes.c_double, ctypes.c_int64,
                                                 ctypes.POINTER(_Info), P, P, P, P, P, P, P]
        lib.oracle_spmv.restype = None
        lib.oracle_spmv.argtypes = [ctypes.c_int64, P, P, P, P, P]
        lib.oracle_cgs_two_passes.restype = None
        lib.oracle_cgs_two_passes.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P]
        lib.oracle_cgs2_update.restype = None
        lib.oracle_cgs2_update.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P,
                                           ctypes.c_double, P, P, P, P, P]
        _libs[acc] = lib
    return _libs[acc]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class OracleResult:
    status: int
    x: np.ndarray
    iters: int
    cycles: int
    converged: bool
    breakdown: bool
    rel_res_true: float
    rel_res_est: float
    reductions: int
    hist: np.ndarray          # |g_k|/||b|| per completed column
    j: int = 0                # columns of the last cycle that completed any
    V: np.ndarray | None = None   # n x (m+2), basis of that cycle
    H: np.ndarray | None = None   # (m+1) x m, unrotated Hessenberg matrix
    T: np.ndarray | None = None   # (m+2) x (m+2), Malard-Paige T (one-reduce), L (cgs2, two_synch)
    g: np.ndarray | None = None   # rotated right-hand side
    S2: np.ndarray | None = None  # (m+1) x m, CGS2 second-pass coefficients


def solve(row_ptr, col_idx, vals, b, x0, m: int, scheme: str = "mgs1r", rtol: float = 1e-8,
          max_iters: int | None = None, dump: bool = False, depth: int = 1,
          acc: str = "double") -> OracleResult:
    """Restarted GMRES(m) on host arrays; see ``oracle_gmres.h`` for the contract.
    depth: the pipeline depth of the lagged schemes (rotations and the stopping
    test applied depth columns at a time). acc: "long double" runs the
    test-only reference build (long sums in extended precision), "openmp" the
    timing build (threads from OMP_NUM_THREADS)."""
    lib = _load(acc)
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = row_ptr.shape[0] - 1
    x = np.array(x0, dtype=np.float64, copy=True)
    if max_iters is None:
        max_iters = min(10 * n, 10**6)
    hist = np.full(max(int(max_iters), 1), np.nan)
    V = H = T = g = S2 = None
    if dump:
        V = np.zeros((m + 2, n))            # row-major (m+2, n) == column-major n x (m+2)
        H = np.zeros((m, m + 1))
        T = np.zeros((m + 2, m + 2))
        g = np.zeros(m + 2)
        S2 = np.zeros((m, m + 1))
    j = ctypes.c_int32(0)
    info = _Info()
    st = lib.oracle_gmres_solve_depth(n, col_idx.shape[0], _ptr(row_ptr), _ptr(col_idx),
                                      _ptr(vals), m, SCHEMES[scheme], int(depth), _ptr(b), _ptr(x),
                                      float(rtol), int(max_iters), ctypes.byref(info), _ptr(hist),
                                      _ptr(V), _ptr(H), _ptr(T), _ptr(g), _ptr(S2),
                                      ctypes.byref(j))
    res = OracleResult(st, x, info.iters, info.cycles, bool(info.converged), bool(info.breakdown),
                       info.rel_res_true, info.rel_res_est, info.reductions,
                       hist[: info.iters].copy(), j.value)
    if dump:
        res.V = V.T          # n x (m+2) view
        res.H = H.T          # (m+1) x m
        res.T = T.T
        res.g = g
        res.S2 = S2.T
    return res


def cgs_two_passes(V, w):
    """Alg 1's two CGS passes of w against the columns of V (n x (i+1)), as
    the CGS-with-re-orthogonalization cycle runs them: (w after both passes,
    the Hessenberg column = both passes' coefficients summed)."""
    V = np.asfortranarray(V, dtype=np.float64)
    n, c = V.shape
    w = np.array(w, dtype=np.float64, copy=True)
    hcol = np.zeros(c)
    _load().oracle_cgs_two_passes(n, c - 1, _ptr(V), _ptr(w), _ptr(hcol))
    return w, hcol


def cgs2_update(V, L, r, rho, w):
    """The lagged CGS2 update of one step (Alg 5), as its cycle runs it, for a
    basis V (n x (k+1)) whose Gram matrix has strictly lower part L: (the new
    column, h = (I - L) r, the second pass's s, the Hessenberg column h + s)."""
    V = np.asfortranarray(V, dtype=np.float64)
    n, c = V.shape
    L = np.asfortranarray(np.tril(L, -1), dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    vnext, h, s, hcol = np.zeros(n), np.zeros(c), np.zeros(c), np.zeros(c)
    _load().oracle_cgs2_update(n, c - 1, _ptr(V), _ptr(L), _ptr(r), float(rho), _ptr(w),
                               _ptr(vnext), _ptr(h), _ptr(s), _ptr(hcol))
    return vnext, h, s, hcol


def omp_threads(n: int = 0) -> int:
    """Threads the OpenMP timing build uses from now on (n >= 1), or the count
    in effect (n = 0)."""
    lib = _load("openmp")
    f = lib.oracle_omp_threads
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int]
    return int(f(int(n)))


def spmv(row_ptr, col_idx, vals, x, acc: str = "double") -> np.ndarray:
    lib = _load(acc)
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(row_ptr.shape[0] - 1)
    lib.oracle_spmv(y.shape[0], _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(x), _ptr(y))
    return y
