"""Seeded test matrices beyond the 7-point grids (inputs only).

These widen the structures the solve path is checked on; every matrix is
symmetric positive definite, with sorted columns and the diagonal stored:

* ``poisson3d_27``: the 27-point Laplacian on N^3 interior nodes (diagonal
  26, every neighbour in the 3x3x3 box -1): rows of up to 27 entries.
* ``anisotropic3d``: the 7-point operator with z-couplings scaled by eps
  (diagonal 4 + 2 eps): for small eps the z-couplings are weak, so the
  strength graph drops them.
* ``decoupled_boundary``: an (N+2)^3 grid whose boundary nodes are identity
  rows without couplings and whose interior is the 7-point Poisson matrix:
  every boundary node is isolated.
* ``random_laplacian``: a weighted random graph on n nodes (a chain for
  connectivity, local random edges, and a few hub nodes joined to many
  others) turned into L + shift I: irregular row lengths, some rows longer
  than a stream block.
* ``banded_spd``: the Laplacian of the band graph (i ~ j for 0 < |i - j| <= b)
  plus shift * I: every row is long (up to 2b + 1 entries), so the mean row
  length exceeds what the LDS-staged SpMV schedule is chosen for.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .grids import CSR


def _to_csr(A) -> CSR:
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    return CSR(A.shape[0], A.indptr.astype(np.int64), A.indices.astype(np.int32),
               A.data.astype(np.float64))


def _grid_coords(N: int):
    idx = np.arange(N**3, dtype=np.int64)
    return idx % N, (idx // N) % N, idx // (N * N)


def poisson3d_27(N: int) -> CSR:
    """27-point Laplacian on N^3 interior nodes, zero Dirichlet data."""
    n = N**3
    i, j, k = _grid_coords(N)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, 26.0)]
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == dz == 0:
                    continue
                ok = ((i + dx >= 0) & (i + dx < N) & (j + dy >= 0) & (j + dy < N)
                      & (k + dz >= 0) & (k + dz < N))
                r = np.nonzero(ok)[0]
                rows.append(r)
                cols.append(r + dx + N * dy + N * N * dz)
                vals.append(np.full(r.size, -1.0))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return _to_csr(A)


def anisotropic3d(N: int, eps: float) -> CSR:
    """7-point operator -u_xx - u_yy - eps u_zz on N^3 interior nodes."""
    n = N**3
    i, j, k = _grid_coords(N)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, 4.0 + 2.0 * eps)]
    for d, (c, stride, w) in enumerate(((i, 1, 1.0), (j, N, 1.0), (k, N * N, eps))):
        for s in (-1, 1):
            ok = (c + s >= 0) & (c + s < N)
            r = np.nonzero(ok)[0]
            rows.append(r)
            cols.append(r + s * stride)
            vals.append(np.full(r.size, -w))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return _to_csr(A)


def decoupled_boundary(N: int) -> CSR:
    """(N+2)^3 grid: boundary nodes are identity rows, interior nodes the
    7-point Poisson stencil restricted to interior neighbours."""
    M = N + 2
    n = M**3
    i, j, k = _grid_coords(M)
    interior = (i > 0) & (i < M - 1) & (j > 0) & (j < M - 1) & (k > 0) & (k < M - 1)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.where(interior, 6.0, 1.0)]
    for c, stride in ((i, 1), (j, M), (k, M * M)):
        for s in (-1, 1):
            nb = c + s
            ok = interior & (nb > 0) & (nb < M - 1)
            r = np.nonzero(ok)[0]
            rows.append(r)
            cols.append(r + s * stride)
            vals.append(np.full(r.size, -1.0))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return _to_csr(A)


def random_laplacian(n: int, local_edges: int = 4, window: int = 64, hubs: int = 3, hub_degree: int = 1500,
                     shift: float = 0.05, seed: int = 0) -> CSR:
    """Weighted graph Laplacian plus shift * I on a seeded random graph.

    Edges: the chain (i, i+1); for every node, ``local_edges`` partners drawn
    from the next ``window`` nodes; ``hubs`` nodes joined to ``hub_degree``
    distinct random nodes each.  Edge weights are uniform in [0.5, 1.5)
    (repeated edges add up).  A_ii = sum of the row's weights + shift.
    """
    rng = np.random.default_rng(seed)
    src = [np.arange(n - 1)]
    dst = [np.arange(1, n)]
    for _ in range(local_edges):
        a = np.arange(n)
        b = a + rng.integers(1, window + 1, size=n)
        keep = b < n
        src.append(a[keep])
        dst.append(b[keep])
    for h in rng.choice(n, size=hubs, replace=False):
        others = rng.choice(n - 1, size=min(hub_degree, n - 1), replace=False)
        others = others + (others >= h)
        src.append(np.full(others.size, h))
        dst.append(others)
    s = np.concatenate(src)
    d = np.concatenate(dst)
    w = rng.uniform(0.5, 1.5, size=s.size)
    # sum repeated edges once, on the upper triangle, so that W is exactly symmetric
    U = sp.csr_matrix(sp.coo_matrix((w, (np.minimum(s, d), np.maximum(s, d))), shape=(n, n)))
    U.sum_duplicates()
    W = (U + U.T).tocsr()
    deg = np.asarray(W.sum(axis=1)).ravel()
    A = sp.diags(deg + shift) - W
    return _to_csr(A)


def banded_spd(n: int, bandwidth: int, shift: float = 0.05) -> CSR:
    """Band-graph Laplacian plus shift * I: a_ij = -1 for 0 < |i - j| <= b,
    a_ii = (number of off-diagonal entries of row i) + shift."""
    offs = np.arange(-bandwidth, bandwidth + 1)
    offs = offs[offs != 0]
    rows, cols = [], []
    for o in offs:
        r = np.arange(max(0, -o), min(n, n - o))
        rows.append(r)
        cols.append(r + o)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    W = sp.csr_matrix((np.ones(r.size), (r, c)), shape=(n, n))
    deg = np.asarray(W.sum(axis=1)).ravel()
    return _to_csr(sp.diags(deg + shift) - W)
