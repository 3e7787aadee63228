"""Seeded block systems: several unknowns per grid node (inputs only).

The paper's Navier-Stokes runs (section 4) solve systems whose matrix entries
are 4 x 4 blocks, one per pair of coupled grid nodes.  Those matrices are
external downloads; the stand-in here is a coupled 4-field diffusion system
on the same 7-point grids as the scalar problems:

    A_ij = a_ij C            (j != i, a_ij the scalar 7-point entry)
    A_ii = a_ii C + rho R_i

with C a fixed 4 x 4 symmetric positive definite coupling of the fields and
R_i = B_i B_i^T + I a seeded symmetric positive definite reaction block per
node (B_i with standard normal entries).  For a symmetric scalar operator L
this is L (x) C plus a positive block diagonal, hence symmetric positive
definite; with upwind convection in L it is nonsymmetric.  With C diagonal
and rho = 0 the four fields decouple into scaled copies of L.

Unknowns are interlaced: unknown 4 i + f is field f at node i.  Blocks are
stored row-major; block columns ascend within a block row and the diagonal
block is always stored.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .grids import diffusion3d

# A fixed symmetric positive definite coupling of four fields.
COUPLING = np.array([[2.0, 0.5, 0.2, 0.1],
                     [0.5, 1.5, 0.3, 0.2],
                     [0.2, 0.3, 1.0, 0.25],
                     [0.1, 0.2, 0.25, 0.8]])

# Four decoupled fields: scaled copies of the scalar operator.
DECOUPLED = np.diag([1.0, 2.0, 0.5, 4.0])


@dataclass
class BSR:
    """Square block sparse matrix: nb block rows of b x b blocks."""

    nb: int
    b: int
    row_ptr: np.ndarray  # int64[nb + 1]
    col: np.ndarray  # int32[nnzb], ascending per block row
    val: np.ndarray  # float64[nnzb * b * b], block k at val[k b^2 : (k+1) b^2], row-major

    @property
    def n(self) -> int:
        return self.nb * self.b

    @property
    def nnzb(self) -> int:
        return int(self.row_ptr[-1])

    def blocks(self) -> np.ndarray:
        return self.val.reshape(-1, self.b, self.b)

    def to_scipy(self):
        """Scalar CSR form (every stored block entry kept)."""
        import scipy.sparse as sp

        M = sp.bsr_matrix((self.blocks(), self.col, self.row_ptr), shape=(self.n, self.n)).tocsr()
        M.sort_indices()
        return M


def coupled_diffusion3d(N: int, g=None, velocity=None, coupling=None, rho: float = 0.05,
                        seed: int = 0) -> BSR:
    """4-field system on the N^3 grid built from ``diffusion3d(N, g, velocity)``."""
    C = COUPLING if coupling is None else np.asarray(coupling, dtype=np.float64)
    b = C.shape[0]
    L = diffusion3d(N, g, velocity)
    n = L.n
    rows = np.repeat(np.arange(n), np.diff(L.row_ptr))
    blocks = L.val[:, None, None] * C[None, :, :]
    if rho != 0.0:
        Bn = np.random.default_rng(seed).standard_normal((n, b, b))
        R = np.einsum("nij,nkj->nik", Bn, Bn) + np.eye(b)[None, :, :]
        diag = rows == L.col
        blocks[diag] = blocks[diag] + rho * R[rows[diag]]
    return BSR(n, b, np.asarray(L.row_ptr, dtype=np.int64).copy(), np.asarray(L.col, dtype=np.int32).copy(),
               np.ascontiguousarray(blocks).reshape(-1))


def decoupled_diffusion3d(N: int, g=None) -> BSR:
    """Four decoupled fields: A_ij = a_ij diag(1, 2, 0.5, 4), no reaction."""
    return coupled_diffusion3d(N, g, coupling=DECOUPLED, rho=0.0)


def random_block_rhs(nb: int, b: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).random(nb * b)
