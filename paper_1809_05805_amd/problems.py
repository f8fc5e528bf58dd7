"""Seeded synthetic linear systems ``A x = b`` in CSR form.

This module only builds inputs: matrices, right-hand sides and initial guesses.
It holds none of the solver's arithmetic, and it is the one module that both the
GPU path's callers (tests, benchmark) and the CPU oracle's callers draw inputs
from.

The paper's matrices (thermal1, Parabolic FEM, the Nalu wind-turbine systems of
Section V) are not available, so the workloads are synthetic stand-ins with the
same row structure (7 and 27 nonzeros per row) and the same physics family
(advection-diffusion, Section V's incompressible-flow momentum systems):

* ``convdiff``: -eps*Laplace(u) + a.grad(u) on the unit square/cube, N interior
  points per side, h = 1/(N+1), zero Dirichlet boundary with the boundary
  couplings dropped, lexicographic ordering with x fastest, first-order upwind
  convection, global Peclet number Pe = |a|_2 / eps.
* ``stencil27_illcond``: 27-point stencil with unit diagonal, off-diagonals
  N(0,1)/27, rows scaled by 10**(8*U(0,1)) for a condition number near 1e8.
* ``simonici``: the diagonal test matrix of Section V-A,
  diag(1e-8, 2, 3, ..., 100) with a normalized random right-hand side.

* ``make_batch``: many independent 2D convection-diffusion systems of uneven
  sizes, the diagonal blocks of one block-diagonal CSR matrix.

Random numbers come from ``numpy.random.PCG64`` seeded by
``SeedSequence([config_id, stream, seed])``; stream 0 draws x_true, stream 1
off-diagonal values, stream 2 row scales, stream 3 right-hand sides (of the
batch: the per-system grid sides, Peclet numbers and wind angles).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Problem",
    "CONFIGS",
    "rng",
    "csr_from_scipy",
    "convdiff",
    "stencil27_illcond",
    "simonici",
    "cyclic_shift",
    "random_dense",
    "make_config",
    "BatchProblem",
    "make_batch",
]


@dataclass
class Problem:
    """A CSR system with everything a solve needs.

    ``row_ptr`` int32[n+1], ``col_idx`` int32[nnz] (sorted within each row),
    ``vals`` float64[nnz]; ``b``, ``x0`` and ``x_true`` float64[n] (``x_true``
    may be None when b is not built from a known solution).
    """

    name: str
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray
    b: np.ndarray
    x0: np.ndarray
    x_true: np.ndarray | None
    m: int
    rtol: float
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def rng(config_id: int, stream: int, seed: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([config_id, stream, seed])))


def csr_from_scipy(A) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """int32/float64 CSR arrays with sorted column indices and no duplicates."""
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    if A.nnz >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return (np.ascontiguousarray(A.indptr, dtype=np.int32),
            np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


def _upwind_1d(N: int, h: float, eps: float, a: float) -> sp.csr_matrix:
    """1-D operator for -eps u'' + a u' on N interior points, first-order upwind."""
    main = np.full(N, 2.0 * eps / h**2 + abs(a) / h)
    off = np.full(N - 1, -eps / h**2)
    lower = off.copy()
    upper = off.copy()
    if a > 0:      # information flows from the left: the upwind neighbour is i-1
        lower = lower - a / h
    elif a < 0:    # upwind neighbour is i+1
        upper = upper - abs(a) / h
    return sp.diags([lower, main, upper], [-1, 0, 1], shape=(N, N), format="csr")


def convdiff(N: int, dim: int, wind, peclet: float) -> sp.csr_matrix:
    """Upwind convection-diffusion matrix on an N^dim grid (x index fastest)."""
    wind = np.asarray(wind, dtype=np.float64)
    if wind.shape != (dim,):
        raise ValueError("wind must have one component per dimension")
    eps = float(np.linalg.norm(wind)) / peclet
    h = 1.0 / (N + 1)
    A = None
    for d in range(dim):
        K = _upwind_1d(N, h, eps, float(wind[d]))
        term = sp.kron(sp.kron(sp.identity(N ** (dim - 1 - d), format="csr"), K, format="csr"),
                       sp.identity(N ** d, format="csr"), format="csr")
        A = term if A is None else (A + term)
    return sp.csr_matrix(A)


def stencil27_illcond(N: int, config_id: int = 3, seed: int = 0, log10_scale: float = 8.0):
    """27-point stencil, M_ii = 1, M_ij ~ N(0,1)/27 over in-grid neighbours, A = D M.

    D_ii = 10**(log10_scale * U_i), U_i ~ U(0,1). Returns (row_ptr, col_idx, vals).
    """
    n = N ** 3
    g_off = rng(config_id, 1, seed)
    g_row = rng(config_id, 2, seed)
    idx = np.arange(n, dtype=np.int64)
    ix = idx % N
    iy = (idx // N) % N
    iz = idx // (N * N)
    rows, cols, vals = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == 0 and dy == 0 and dz == 0:
                    rows.append(idx)
                    cols.append(idx)
                    vals.append(np.ones(n))
                    continue
                # one full draw per offset, in a fixed order, masked afterwards
                v = g_off.standard_normal(n) / 27.0
                ok = ((ix + dx >= 0) & (ix + dx < N) & (iy + dy >= 0) & (iy + dy < N)
                      & (iz + dz >= 0) & (iz + dz < N))
                rows.append(idx[ok])
                cols.append(idx[ok] + dx + N * dy + N * N * dz)
                vals.append(v[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    scale = 10.0 ** (log10_scale * g_row.random(n))
    vals = vals * scale[rows]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return csr_from_scipy(A)


def simonici(seed: int = 0) -> Problem:
    """Section V-A test: A = diag(1e-8, 2, ..., 100), b = randn normalized, no preconditioner."""
    d = np.concatenate([[1e-8], np.arange(2.0, 101.0)])
    A = sp.diags(d, 0, format="csr")
    b = rng(100, 3, seed).standard_normal(100)
    b /= np.linalg.norm(b)
    rp, ci, va = csr_from_scipy(A)
    return Problem("simonici", rp, ci, va, b, np.zeros(100), None, m=100, rtol=0.0,
                   meta={"kappa": 1e10})


def cyclic_shift(n: int) -> Problem:
    """A e_i = e_{i+1 mod n}, b = e_0: GMRES stagnates at |r| = 1 until step n."""
    rows = np.arange(n)
    cols = (rows - 1) % n
    A = sp.csr_matrix((np.ones(n), (rows, cols)), shape=(n, n))
    rp, ci, va = csr_from_scipy(A)
    b = np.zeros(n)
    b[0] = 1.0
    x_true = np.zeros(n)
    x_true[n - 1] = 1.0
    return Problem(f"cyclic{n}", rp, ci, va, b, np.zeros(n), x_true, m=n, rtol=0.0)


def random_dense(n: int, seed: int = 0, shift: float = 4.0) -> Problem:
    """Dense nonsymmetric, well-conditioned matrix shift*I + randn/sqrt(n), stored as CSR."""
    g = rng(200 + n, 1, seed)
    M = g.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)
    x_true = rng(200 + n, 0, seed).uniform(-1.0, 1.0, n)
    b = M @ x_true
    rp, ci, va = csr_from_scipy(sp.csr_matrix(M))
    return Problem(f"dense{n}", rp, ci, va, b, np.zeros(n), x_true, m=n, rtol=0.0)


# name -> (config id, description)
CONFIGS = {
    "convdiff2d": (1, "2D 5-point upwind convection-diffusion, 64^2, wind (1,1), Pe 10, m=30, rtol 1e-8"),
    "convdiff3d": (2, "3D 7-point upwind convection-diffusion, 128^3, wind (1,0.5,0.25), Pe 50, m=50, rtol 1e-10"),
    "stencil27": (3, "3D 27-point random stencil, 100^3, rows scaled log-uniform in [1,1e8], m=100, rtol 1e-10"),
}


def make_config(name: str, seed: int = 0, N: int | None = None) -> Problem:
    """Build one of the named workloads. ``N`` overrides the grid side (smaller test copies)."""
    if name not in CONFIGS:
        raise KeyError(f"unknown config {name!r}; known: {sorted(CONFIGS)}")
    cid = CONFIGS[name][0]
    if name == "convdiff2d":
        N = 64 if N is None else N
        A = convdiff(N, 2, (1.0, 1.0), 10.0)
        rp, ci, va = csr_from_scipy(A)
        m, rtol = 30, 1e-8
    elif name == "convdiff3d":
        N = 128 if N is None else N
        A = convdiff(N, 3, (1.0, 0.5, 0.25), 50.0)
        rp, ci, va = csr_from_scipy(A)
        m, rtol = 50, 1e-10
    else:
        N = 100 if N is None else N
        rp, ci, va = stencil27_illcond(N, cid, seed)
        m, rtol = 100, 1e-10
    n = rp.shape[0] - 1
    x_true = rng(cid, 0, seed).uniform(-1.0, 1.0, n)
    b = sp.csr_matrix((va, ci, rp), shape=(n, n)) @ x_true
    return Problem(name, rp, ci, va, np.ascontiguousarray(b), np.zeros(n), x_true, m, rtol,
                   meta={"N": N, "config_id": cid})



@dataclass
class BatchProblem:
    """Independent systems as the diagonal blocks of one CSR matrix.

    System i owns rows and columns [row_off[i], row_off[i+1]); ``sides``,
    ``peclet`` and ``angle`` are its grid side, Peclet number and wind angle.
    """

    name: str
    row_off: np.ndarray
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray
    b: np.ndarray
    x0: np.ndarray
    x_true: np.ndarray
    m: int
    rtol: float
    sides: np.ndarray
    peclet: np.ndarray
    angle: np.ndarray

    @property
    def nsys(self) -> int:
        return int(self.row_off.shape[0] - 1)

    @property
    def n(self) -> int:
        return int(self.row_off[-1])

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def system(self, i: int) -> Problem:
        """System i as a stand-alone Problem (local row and column indices)."""
        r0, r1 = int(self.row_off[i]), int(self.row_off[i + 1])
        e0, e1 = int(self.row_ptr[r0]), int(self.row_ptr[r1])
        rp = (self.row_ptr[r0: r1 + 1] - e0).astype(np.int32)
        ci = (self.col_idx[e0:e1] - r0).astype(np.int32)
        return Problem(f"{self.name}[{i}]", rp, ci, self.vals[e0:e1].copy(), self.b[r0:r1].copy(),
                       self.x0[r0:r1].copy(), self.x_true[r0:r1].copy(), self.m, self.rtol,
                       meta={"N": int(self.sides[i]), "peclet": float(self.peclet[i]),
                             "angle": float(self.angle[i])})


def _batch_of(name: str, cid: int, seed: int, dim: int, sides, peclet, angle, m: int,
              rtol: float) -> BatchProblem:
    """The block-diagonal batch of upwind convection-diffusion systems with the
    given grid sides, Peclet numbers and wind angles (in 3D the wind is
    (cos t, sin t, 1/2)); x_true ~ U(-1, 1) over the batch from stream 0."""
    sizes = sides.astype(np.int64) ** dim
    row_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(row_off[-1])
    rps, cis, vas = [], [], []
    nnz = 0
    for i in range(len(sides)):
        wind = (np.cos(angle[i]), np.sin(angle[i])) + ((0.5,) if dim == 3 else ())
        A = convdiff(int(sides[i]), dim, wind, float(peclet[i]))
        rp, ci, va = csr_from_scipy(A)
        rps.append(rp[:-1].astype(np.int64) + nnz)
        cis.append(ci.astype(np.int64) + row_off[i])
        vas.append(va)
        nnz += int(rp[-1])
    if nnz >= 2**31 or n >= 2**31:
        raise ValueError("batch too large for int32 CSR indices")
    row_ptr = np.concatenate(rps + [np.array([nnz])]).astype(np.int32)
    col_idx = np.concatenate(cis).astype(np.int32)
    vals = np.concatenate(vas)
    x_true = rng(cid, 0, seed).uniform(-1.0, 1.0, n)
    b = sp.csr_matrix((vals, col_idx, row_ptr), shape=(n, n)) @ x_true
    return BatchProblem(name, row_off, row_ptr, col_idx, vals, np.ascontiguousarray(b),
                        np.zeros(n), x_true, m, rtol, sides, peclet, angle)


def make_batch(nsys: int = 512, seed: int = 0, side_lo: int = 32, side_hi: int = 256,
               m: int = 30, rtol: float = 1e-10) -> BatchProblem:
    """Batch of 2D 5-point upwind convection-diffusion systems (config id 5).

    Per system: grid side N ~ U{side_lo..side_hi} (n = N^2), Peclet ~ U(1, 100)
    and wind (cos t, sin t) with t ~ U(0, 2 pi), all from stream 3;
    x_true ~ U(-1, 1) over the whole batch from stream 0; b = A x_true, x0 = 0.
    """
    if nsys < 1 or side_lo < 1 or side_hi < side_lo:
        raise ValueError("need nsys >= 1 and 1 <= side_lo <= side_hi")
    cid = 5
    g = rng(cid, 3, seed)
    sides = g.integers(side_lo, side_hi + 1, size=nsys)
    peclet = g.uniform(1.0, 100.0, size=nsys)
    angle = g.uniform(0.0, 2.0 * np.pi, size=nsys)
    return _batch_of(f"batch{nsys}", cid, seed, 2, sides, peclet, angle, m, rtol)


def make_batch3d(nsys: int = 64, seed: int = 0, side_lo: int = 32, side_hi: int = 64,
                 m: int = 50, rtol: float = 1e-10) -> BatchProblem:
    """Batch of 3D 7-point upwind convection-diffusion systems (id 6), sized so
    that the bases in use at once far exceed the GPU's 256 MB last-level cache
    (64 systems of 32^3..64^3 rows at m = 50: about 3 GB of basis).

    Per system: grid side N ~ U{side_lo..side_hi} (n = N^3), Peclet ~ U(1, 50)
    and wind (cos t, sin t, 1/2) with t ~ U(0, 2 pi), all from stream 3;
    x_true ~ U(-1, 1) over the whole batch from stream 0; b = A x_true, x0 = 0.
    """
    if nsys < 1 or side_lo < 1 or side_hi < side_lo:
        raise ValueError("need nsys >= 1 and 1 <= side_lo <= side_hi")
    cid = 6
    g = rng(cid, 3, seed)
    sides = g.integers(side_lo, side_hi + 1, size=nsys)
    peclet = g.uniform(1.0, 50.0, size=nsys)
    angle = g.uniform(0.0, 2.0 * np.pi, size=nsys)
    return _batch_of(f"batch3d_{nsys}", cid, seed, 3, sides, peclet, angle, m, rtol)
