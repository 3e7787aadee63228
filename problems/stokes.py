"""Generalised Stokes systems: the two-field saddle-point structure of the
paper's Navier-Stokes runs (section 4, eq. 3: [[K, G], [D, S]] for velocity
and pressure), which are assembled from matrices not available here.

This is a seeded, structured stand-in with the same block structure: the
unsteady Stokes operator on an N^3 grid with velocity and pressure at the
same nodes (equal order, as the paper's stabilised tetrahedral elements) and
a pressure-Laplacian stabilisation, h^2-scaled:

* K = alpha I + L for each velocity component (L the 7-point Laplacian with
  Dirichlet boundaries: diagonal 6, neighbours -1), alpha = h^2 / dt; the
  default alpha = 2 is an implicit step of dt = h^2 / 2 (unit viscosity), the
  mass-dominated velocity block of a time-stepping flow solver;
* G: centred gradient, (G_d p)_i = (h/2) (p_{i+e_d} - p_{i-e_d}) along axis d,
  neighbours outside the grid dropped (p = 0 there);
* D = -G^T (the divergence, with the continuity equation's sign);
* S = beta L (pressure stabilisation), beta = h^2 / 12.

Unknowns: u_x, u_y, u_z (N^3 each, lexicographic), then p (N^3); the first
3 N^3 unknowns are the velocity field.  Every diagonal entry is positive.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .grids import CSR, poisson3d


def stokes3d(N: int, alpha: float | None = None, beta: float | None = None):
    """(CSR of the 4 N^3 x 4 N^3 system, number of velocity unknowns 3 N^3)."""
    n = N**3
    h = 1.0 / (N + 1)
    if alpha is None:
        alpha = 2.0
    if beta is None:
        beta = h * h / 12.0
    L = poisson3d(N).to_scipy()
    K1 = (L + alpha * sp.identity(n, format="csr")).tocsr()
    idx = np.arange(n, dtype=np.int64)
    coords = (idx % N, (idx // N) % N, idx // (N * N))
    strides = (1, N, N * N)
    grads = []
    for d in range(3):
        up = coords[d] < N - 1
        dn = coords[d] > 0
        rows = np.concatenate([idx[up], idx[dn]])
        cols = np.concatenate([idx[up] + strides[d], idx[dn] - strides[d]])
        vals = np.concatenate([np.full(int(up.sum()), 0.5 * h), np.full(int(dn.sum()), -0.5 * h)])
        grads.append(sp.csr_matrix((vals, (rows, cols)), shape=(n, n)))
    G = sp.vstack(grads).tocsr()
    K = sp.block_diag([K1, K1, K1], format="csr")
    A = sp.bmat([[K, G], [-G.T, beta * L]], format="csr")
    A.sum_duplicates()
    A.sort_indices()
    A.eliminate_zeros()
    return (CSR(4 * n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)),
            3 * n)


def stokes_rhs(N: int) -> np.ndarray:
    """Body force 1 on every velocity unknown, 0 on the continuity rows."""
    n = N**3
    return np.concatenate([np.ones(3 * n), np.zeros(n)])
