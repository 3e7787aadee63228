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


# ---------------------------------------------------------------------------
# Equal-order tetrahedral elements (the paper's Navier-Stokes discretisation)

def _kuhn_tets():
    """The six tetrahedra of the Kuhn (Freudenthal) subdivision of the unit
    cube: vertex offsets (4 x 3 integer array) per tetrahedron, all sharing
    the main diagonal (0,0,0)-(1,1,1)."""
    import itertools

    tets = []
    for perm in itertools.permutations(range(3)):
        v = [np.zeros(3, dtype=np.int64)]
        for a in perm:
            nxt = v[-1].copy()
            nxt[a] = 1
            v.append(nxt)
        tets.append(np.array(v))
    return tets


def oseen_p1(N: int, nu: float = 0.01, dt: float | None = None, wind_speed: float = 1.0):
    """Linearised (Oseen) step of incompressible Navier-Stokes on the unit
    cube with equal-order P1 tetrahedra and an ASGS-type stabilisation:
    the structure of section 4's Navier-Stokes systems (4 unknowns per mesh
    node; each node coupled to its 14 mesh neighbours).

    Mesh: the Kuhn subdivision of an (N+1)^3 cube grid, h = 1/(N+1); the N^3
    interior vertices carry u_x, u_y, u_z and p (velocity Dirichlet and the
    pressure pinned at the boundary vertices).  Per tetrahedron (volume V,
    basis gradients g_i, wind w at the centroid, tau = 1/(4 nu/h^2 + 2|w|/h
    + 1/dt)):
      K_ij = V/20 (1 + d_ij)/dt + nu V g_i.g_j + V/4 w.g_j + tau V (w.g_i)(w.g_j)
      G_d,ij = V/4 g_j,d  (pressure gradient),  D = -G^T (divergence rows),
      S_ij = tau V g_i.g_j (pressure stabilisation).
    The wind is the rotating field w = s (0.5 - y, x - 0.5, 0.25); dt = 2h
    by default (a time step at Courant number about 1).  Returns (CSR,
    number of velocity unknowns 3 N^3); unknowns: u_x, u_y, u_z (N^3 each,
    lexicographic), then p.
    """
    h = 1.0 / (N + 1)
    if dt is None:
        dt = 2.0 * h
    n = N**3
    M1 = N + 1  # cubes per axis
    ci = np.arange(M1**3, dtype=np.int64)
    cx, cy, cz = ci % M1, (ci // M1) % M1, ci // (M1 * M1)
    names = ("K", "G0", "G1", "G2", "S")
    rows, cols = [], []  # one pattern for all five element matrices
    vals = {k: [] for k in names}
    for off in _kuhn_tets():
        X = off.astype(np.float64) * h
        T = np.hstack([np.ones((4, 1)), X])
        coef = np.linalg.inv(T)  # column j: coefficients of basis j
        grads = coef[1:, :].T  # (4, 3)
        V = abs(np.linalg.det(X[1:] - X[0])) / 6.0
        # vertex indices of this tetrahedron in every cube (-1: boundary)
        gidx = []
        for a in range(4):
            vx, vy, vz = cx + off[a, 0], cy + off[a, 1], cz + off[a, 2]
            inside = (vx >= 1) & (vx <= N) & (vy >= 1) & (vy <= N) & (vz >= 1) & (vz <= N)
            gidx.append(np.where(inside, (vx - 1) + N * (vy - 1) + N * N * (vz - 1), -1))
        cent = (np.stack([cx, cy, cz], axis=1) + off.mean(axis=0)) * h
        w = wind_speed * np.stack([0.5 - cent[:, 1], cent[:, 0] - 0.5, np.full(len(ci), 0.25)], axis=1)
        wn = np.linalg.norm(w, axis=1)
        tau = 1.0 / (4.0 * nu / h**2 + 2.0 * wn / h + 1.0 / dt)
        wg = w @ grads.T  # (cubes, 4): w . g_j
        for a in range(4):
            for b in range(4):
                ok = (gidx[a] >= 0) & (gidx[b] >= 0)
                if not ok.any():
                    continue
                rows.append(gidx[a][ok])
                cols.append(gidx[b][ok])
                lap = V * float(grads[a] @ grads[b])
                mass = V / 20.0 * (2.0 if a == b else 1.0)
                vals["K"].append(mass / dt + nu * lap + V / 4.0 * wg[ok, b] + tau[ok] * V * wg[ok, a] * wg[ok, b])
                for d in range(3):
                    vals[f"G{d}"].append(np.full(int(ok.sum()), V / 4.0 * grads[b, d]))
                vals["S"].append(tau[ok] * lap)
    keys = np.concatenate(rows) * n + np.concatenate(cols)
    uniq, inv = np.unique(keys, return_inverse=True)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(uniq // n, minlength=n), out=indptr[1:])
    indices = (uniq % n).astype(np.int32)
    mats = {}
    for k in names:
        data = np.bincount(inv, weights=np.concatenate(vals[k]), minlength=uniq.size)
        if k.startswith("G"):
            # the diagonal of G_d integrates a derivative over a vertex patch:
            # zero in exact arithmetic, dropped
            data[np.abs(data) <= 1e-12 * np.abs(data).max()] = 0.0
        M = sp.csr_matrix((data, indices.copy(), indptr.copy()), shape=(n, n))  # own arrays: pruned below
        M.eliminate_zeros()
        mats[k] = M
    K, S = mats["K"], mats["S"]
    G = [mats[f"G{d}"] for d in range(3)]
    Z = None
    A = sp.bmat([[K, Z, Z, G[0]], [Z, K, Z, G[1]], [Z, Z, K, G[2]],
                 [-G[0].T, -G[1].T, -G[2].T, S]], format="csr")
    A.sum_duplicates()
    A.sort_indices()
    A.eliminate_zeros()
    return (CSR(4 * n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)),
            3 * n)


def oseen_rhs(N: int) -> np.ndarray:
    """Body force (1, 0.5, 0.25) per velocity unknown scaled by the lumped
    nodal volume h^3; zero continuity right-hand side."""
    n = N**3
    h = 1.0 / (N + 1)
    return np.concatenate([np.full(n, h**3), np.full(n, 0.5 * h**3), np.full(n, 0.25 * h**3), np.zeros(n)])
