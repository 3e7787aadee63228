"""Seeded test matrices and right-hand sides (inputs only).

Grids are ordered lexicographically with x fastest: the unknown at grid point
(i, j, k), 0 <= i, j, k < N, has index ``i + N*j + N*N*k``.  Boundary
(Dirichlet) nodes are eliminated, so an N^3 grid has N^3 unknowns.  Matrices
are returned as :class:`CSR` with int64 row pointers, int32 column indices in
ascending order within each row (the diagonal always stored) and float64
values.

* ``poisson3d`` is the finite-difference Poisson model problem of the
  paper's benchmark section (eq. 2: -Laplace(u) = 1 on the unit cube, zero
  Dirichlet data, uniform mesh), scaled by h^2: diagonal 6, neighbours -1.
  At N = 150 it has 3,375,000 unknowns and 23,490,000 nonzeros, the sizes
  quoted in the shared-memory benchmark (section 4.1).
* ``diffusion3d`` is the variable-coefficient extension used for the
  heterogeneous and served workloads: node coefficients k = exp(g) with g a
  stationary Gaussian field, harmonic-mean face coefficients, a Dirichlet face
  contributing k_i to the diagonal, and optional first-order upwind
  convection.  With g == 0 and no convection it is bit-identical to
  ``poisson3d``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import ndimage


@dataclass
class CSR:
    """Square sparse matrix in compressed sparse row form."""

    n: int
    row_ptr: np.ndarray  # int64[n + 1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def poisson3d_nnz(N: int) -> int:
    """Nonzeros of the 7-point operator on N^3 interior nodes: 7N^3 - 6N^2."""
    return 7 * N**3 - 6 * N**2


def _structure7(N: int):
    """Row pointers, columns and the (n, 7) existence mask of the 7-point pattern."""
    n = N**3
    idx = np.arange(n, dtype=np.int64)
    i = idx % N
    j = (idx // N) % N
    k = idx // (N * N)
    strides = (1, N, N * N)
    coords = (i, j, k)
    cols, mask = [], []
    for d in (2, 1, 0):
        cols.append(idx - strides[d])
        mask.append(coords[d] > 0)
    cols.append(idx)
    mask.append(np.ones(n, dtype=bool))
    for d in (0, 1, 2):
        cols.append(idx + strides[d])
        mask.append(coords[d] < N - 1)
    M = np.stack(mask, axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(M.sum(axis=1), out=row_ptr[1:])
    col = np.stack(cols, axis=1)[M].astype(np.int32)
    for a in (row_ptr, col, M):
        a.flags.writeable = False
    return row_ptr, col, M


_STRUCT_CACHE: dict = {}


def _assemble7(N: int, diag: np.ndarray, lo: list, hi: list) -> CSR:
    """Assemble a 7-point operator.

    ``lo[d]`` holds, for every node, the matrix entry coupling it to its
    neighbour at -e_d (d = 0: x, 1: y, 2: z); ``hi[d]`` the entry to +e_d.
    Entries whose neighbour lies outside the grid are dropped.  Columns come
    out sorted: -z, -y, -x, diag, +x, +y, +z.  The (read-only) row pointers and
    columns of grids up to 128^3 are shared between calls.
    """
    if N <= 128:
        if N not in _STRUCT_CACHE:
            if len(_STRUCT_CACHE) >= 16:
                _STRUCT_CACHE.pop(next(iter(_STRUCT_CACHE)))
            _STRUCT_CACHE[N] = _structure7(N)
        row_ptr, col, M = _STRUCT_CACHE[N]
    else:
        row_ptr, col, M = _structure7(N)
    V = np.stack([lo[2], lo[1], lo[0], diag, hi[0], hi[1], hi[2]], axis=1)
    return CSR(N**3, row_ptr, col, V[M].astype(np.float64, copy=False))


def poisson3d(N: int) -> CSR:
    """h^2-scaled 7-point Poisson matrix on N^3 interior nodes."""
    n = N**3
    six = np.full(n, 6.0)
    m1 = np.full(n, -1.0)
    return _assemble7(N, six, [m1, m1, m1], [m1, m1, m1])


def gaussian_field(N: int, sigma: float, ell: float, seed: int) -> np.ndarray:
    """Stationary Gaussian field on N^3 nodes, flattened x-fastest.

    Covariance sigma^2 exp(-d^2 / (2 ell^2)) with d in grid cells.  White noise
    from ``numpy.random.default_rng(seed).standard_normal`` on an (N+2r)^3 grid
    is convolved ("valid" part only) with the separable Gaussian kernel of
    standard deviation ell/sqrt(2), truncated at r = ceil(3 ell / sqrt(2)) and
    scaled to unit L2 norm, so every node has variance sigma^2 (up to the
    truncation) and the correlation length is ell.
    """
    s = ell / math.sqrt(2.0)
    r = int(math.ceil(3.0 * s))
    t = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-(t * t) / (2.0 * s * s))
    w /= math.sqrt(float(np.sum(w * w)))
    M = N + 2 * r
    a = np.random.default_rng(seed).standard_normal((M, M, M))
    for axis in range(3):
        # centred correlation, then keep the "valid" part along this axis
        a = ndimage.correlate1d(a, w, axis=axis, mode="constant")
        sl = [slice(None)] * 3
        sl[axis] = slice(r, r + N)
        a = a[tuple(sl)]
    return (sigma * a).reshape(-1)


def diffusion3d(N: int, g: np.ndarray | None = None, velocity=None) -> CSR:
    """Variable-coefficient diffusion (+ optional upwind convection), h^2-scaled.

    ``g`` is the log-coefficient per node (k = exp(g)); None means k == 1.
    ``velocity`` = (vx, vy, vz) in physical units; each positive component
    adds v_d*h to the diagonal and -v_d*h to the upwind (-e_d) neighbour, with
    h = 1/(N+1).  The result is an M-matrix whose interior rows sum to zero.
    """
    n = N**3
    kcoef = np.ones(n) if g is None else np.exp(np.asarray(g, dtype=np.float64))
    idx = np.arange(n, dtype=np.int64)
    coords = (idx % N, (idx // N) % N, idx // (N * N))
    strides = (1, N, N * N)
    diag = np.zeros(n)
    lo, hi = [None] * 3, [None] * 3
    for d in range(3):
        nb_hi = np.minimum(idx + strides[d], n - 1)
        k_hi = kcoef[nb_hi]
        c_hi = 2.0 * kcoef * k_hi / (kcoef + k_hi)
        c_hi = np.where(coords[d] < N - 1, c_hi, kcoef)  # Dirichlet face: k_i
        nb_lo = np.maximum(idx - strides[d], 0)
        k_lo = kcoef[nb_lo]
        c_lo = 2.0 * kcoef * k_lo / (kcoef + k_lo)
        c_lo = np.where(coords[d] > 0, c_lo, kcoef)
        diag = diag + c_lo
        diag = diag + c_hi
        lo[d] = -c_lo
        hi[d] = -c_hi
    if velocity is not None:
        h = 1.0 / (N + 1)
        for d in range(3):
            v = float(velocity[d])
            if v > 0.0:
                diag = diag + v * h
                lo[d] = lo[d] - v * h
            elif v < 0.0:
                diag = diag - v * h
                hi[d] = hi[d] + v * h
    return _assemble7(N, diag, lo, hi)


def tridiag1d(n: int) -> CSR:
    """1-D Laplacian tridiag(-1, 2, -1) of order n."""
    rows, cols, vals = [], [], []
    row_ptr = [0]
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                cols.append(j)
                vals.append(v)
        row_ptr.append(len(cols))
    return CSR(n, np.array(row_ptr, dtype=np.int64), np.array(cols, dtype=np.int32),
               np.array(vals, dtype=np.float64))


def rhs_ones(n: int) -> np.ndarray:
    """The paper's unit source term (eq. 2) as a right-hand side."""
    return np.ones(n, dtype=np.float64)


def rhs_uniform(n: int, seed: int = 0) -> np.ndarray:
    """Right-hand side with entries uniform in [0, 1), from ``default_rng(seed)``."""
    return np.random.default_rng(seed).random(n)
