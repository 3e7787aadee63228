"""Oracle for smoothed-aggregation AMG whose matrix entries are small dense blocks.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 NumPy,
written to be checked against the method by eye.

Where it comes from
-------------------
Section 3, "Value types": the value type of a matrix may be a small static
matrix (the paper's Navier-Stokes runs of section 4 use 4 x 4 blocks, one
per grid node, coupling the node's unknowns).  The method is then the one of
section 2 ("AMG setup", "AMG solve") taken blockwise: the unknowns of one
node move together through the hierarchy.  Readings (the paper gives no
formulas; each is the scalar reading of the scalar oracle with |.| replaced
by a block norm, a division by a block inverse, the unit by the identity):

* strength: node j != i is strong for i when s_ij^2 > eps^4 s_ii s_jj, with
  s_ij = ||A_ij||_F^2 (the scalar test a_ij^2 > eps^2 |a_ii a_jj| squared);
  symmetrised by union; the same three-phase aggregation over nodes;
* tentative prolongator: P_hat_ic = I_b for node i in aggregate c (each of
  the b unknowns of a node is constant on an aggregate, field by field);
* filtered matrix: weak blocks are summed into the diagonal block; a
  non-isolated node whose lumped diagonal block has a symmetric part that is
  not positive definite keeps A_ii;
* damping: omega = (4/3) / rho, rho the Gershgorin bound of D_F^-1 A_F
  (D_F the block diagonal of A_F): the largest row sum of |D_F^-1 A_F| over
  the unknowns of non-isolated nodes;
* P = P_hat - omega D_F^-1 A_F P_hat; R = P^T (blocks transposed);
  A_{l+1} = R (A P);
* smoother: block SPAI-0, M_i = A_ii^T (sum_j A_ij A_ij^T)^-1 (the
  block-diagonal M minimising ||I - M A||_F, row block by row block; b = 1
  gives a_ii / sum_j a_ij^2), or block Jacobi, M_i = omega A_ii^-1; a
  pre-sweep is z <- z + M (f - A z) and a post-sweep z <- z + M^T (f - A z),
  the adjoint of the pre-sweep (the same sweep for the scalar, diagonal
  smoothers), so that the V-cycle of a symmetric A is symmetric although the
  block SPAI-0 M is not;
* coarsest level: dense LU of the scalar form of A_L.

Arithmetic order (so that a second implementation can reproduce it): a
block product T = X Y is T[r, s] = ((X[r,0] Y[0,s] + X[r,1] Y[1,s]) + ...)
in c = 0..b-1; a sparse block product C = X Y accumulates C_ij += X_ik Y_kj
over k in X's row order, starting from zero; a block inverse is Gauss-Jordan
elimination with partial pivoting (largest |entry| of the column, lowest row
on ties) on [B | I]; a squared Frobenius norm adds the b^2 squares in
row-major order.

Block matrices are held as (indptr, indices, data) with data[k] the b x b
block k (row-major), block columns ascending within a block row.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import sa_amg


@dataclass
class Bsr:
    """Square block sparse matrix: nb block rows of b x b blocks."""

    indptr: np.ndarray  # int64[nb + 1]
    indices: np.ndarray  # int64[nnzb], ascending per block row
    data: np.ndarray  # float64[nnzb, b, b]
    nb: int
    ncb: int = -1  # block columns (default nb)

    def __post_init__(self):
        if self.ncb < 0:
            self.ncb = self.nb

    @property
    def b(self) -> int:
        return int(self.data.shape[1])

    def to_scipy(self) -> sp.csr_matrix:
        """Scalar CSR form (b nb x b ncb), every stored block entry kept."""
        b = self.b
        M = sp.bsr_matrix((self.data, self.indices, self.indptr), shape=(b * self.nb, b * self.ncb))
        M = M.tocsr()
        M.sort_indices()
        return M


def _rows(A: Bsr) -> np.ndarray:
    return np.repeat(np.arange(A.nb), np.diff(A.indptr))


def block_product(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """T = X Y for stacks of b x b blocks, summed in c = 0..b-1."""
    b = X.shape[-1]
    T = X[..., :, 0:1] * Y[..., 0:1, :]
    for c in range(1, b):
        T = T + X[..., :, c:c + 1] * Y[..., c:c + 1, :]
    return T


def block_inverse(B: np.ndarray) -> np.ndarray:
    """Inverse of each b x b block: Gauss-Jordan with partial pivoting."""
    B = np.array(B, dtype=np.float64)
    m, b, _ = B.shape
    W = np.concatenate([B, np.broadcast_to(np.eye(b), (m, b, b))], axis=2)  # [B | I]
    idx = np.arange(m)
    for c in range(b):
        # pivot: largest |entry| of column c in rows c..b-1, lowest row on ties
        p = c + np.argmax(np.abs(W[:, c:, c]), axis=1)
        row_c = W[idx, c, :].copy()
        W[idx, c, :] = W[idx, p, :]
        W[idx, p, :] = row_c
        piv = W[:, c, c].copy()
        W[:, c, :] = W[:, c, :] / piv[:, None]
        for r in range(b):
            if r == c:
                continue
            W[:, r, :] = W[:, r, :] - W[:, r, c:c + 1] * W[:, c, :]
    return W[:, :, b:]


def frobenius_sq(B: np.ndarray) -> np.ndarray:
    """||B||_F^2 of each block, squares added in row-major order."""
    b = B.shape[-1]
    s = np.zeros(B.shape[0])
    for r in range(b):
        for c in range(b):
            s = s + B[:, r, c] * B[:, r, c]
    return s


def diagonal_blocks(A: Bsr) -> np.ndarray:
    """A_ii for every block row (zero block where none is stored)."""
    D = np.zeros((A.nb, A.b, A.b))
    rows = _rows(A)
    on = A.indices == rows
    D[rows[on]] = A.data[on]
    return D


def spgemm(X: Bsr, Y: Bsr) -> Bsr:
    """C = X Y: C_ij = sum over k in X's row order of X_ik Y_kj, from zero.

    Every structurally generated block is kept (no dropping by value).
    """
    xr = _rows(X)
    ylen = np.diff(Y.indptr)
    reps = ylen[X.indices]  # products generated by each block of X
    i = np.repeat(xr, reps)
    xk = np.repeat(np.arange(X.indices.size), reps)
    # position of each product inside Y's row k
    starts = Y.indptr[X.indices]
    offs = np.arange(reps.sum()) - np.repeat(np.cumsum(reps) - reps, reps)
    yk = np.repeat(starts, reps) + offs
    j = Y.indices[yk]
    prods = block_product(X.data[xk], Y.data[yk])
    # output blocks sorted by (i, j); contributions added in generation order
    key = i * Y.ncb + j
    ukey, slot = np.unique(key, return_inverse=True)
    C = np.zeros((ukey.size, X.b, X.b))
    np.add.at(C, slot, prods)
    ci = ukey // Y.ncb
    cj = ukey % Y.ncb
    indptr = np.zeros(X.nb + 1, dtype=np.int64)
    np.add.at(indptr, ci + 1, 1)
    indptr = np.cumsum(indptr)
    return Bsr(indptr, cj.astype(np.int64), C, X.nb, Y.ncb)


def transpose(P: Bsr) -> Bsr:
    """R = P^T: block (j, i) = P_ij^T, block columns ascending."""
    rows = _rows(P)
    order = np.lexsort((rows, P.indices))  # by new row (old column), then old row
    nr = P.indices[order]
    indptr = np.zeros(P.ncb + 1, dtype=np.int64)
    np.add.at(indptr, nr + 1, 1)
    indptr = np.cumsum(indptr)
    data = np.transpose(P.data[order], (0, 2, 1)).copy()
    return Bsr(indptr, rows[order].astype(np.int64), data, P.ncb, P.nb)


# --------------------------------------------------------------------------
# Setup
# --------------------------------------------------------------------------


def strength_graph(A: Bsr, eps: float) -> sp.csr_matrix:
    """Symmetrised strong-connection graph over the nodes (block rows)."""
    s = frobenius_sq(A.data)
    sd = frobenius_sq(diagonal_blocks(A))
    rows = _rows(A)
    cols = A.indices
    e4 = (eps * eps) * (eps * eps)
    strong = (cols != rows) & (s * s > e4 * (sd[rows] * sd[cols]))
    n = A.nb
    S = sp.csr_matrix((np.ones(int(strong.sum()), dtype=np.int8), (rows[strong], cols[strong])), shape=(n, n))
    S = ((S + S.T) > 0).astype(np.int8).tocsr()
    S.sort_indices()
    return S


def _pos_def_sym_part(B: np.ndarray) -> np.ndarray:
    """Whether the symmetric part of each block is positive definite."""
    Hs = 0.5 * (B + np.transpose(B, (0, 2, 1)))
    return np.all(np.linalg.eigvalsh(Hs) > 0.0, axis=1)


def filtered_matrix(A: Bsr, S: sp.csr_matrix):
    """A_F (strong off-diagonal blocks, weak ones summed into the diagonal
    block in column order) and its diagonal blocks D_F."""
    rows = _rows(A)
    cols = A.indices
    in_graph = np.asarray(S[rows, cols]).ravel() != 0 if A.indices.size else np.zeros(0, dtype=bool)
    offdiag = cols != rows
    weak = offdiag & ~in_graph
    D = diagonal_blocks(A)
    lumped = np.zeros_like(D)
    np.add.at(lumped, rows[weak], A.data[weak])  # in storage (column) order per row
    D_F = D + lumped
    isolated = np.diff(S.indptr) == 0
    bad = (~isolated) & ~_pos_def_sym_part(D_F)
    D_F[bad] = D[bad]
    keep = (offdiag & in_graph) | ~offdiag
    data = A.data[keep].copy()
    krows = rows[keep]
    kcols = cols[keep]
    diag_pos = krows == kcols
    data[diag_pos] = D_F[krows[diag_pos]]
    indptr = np.zeros(A.nb + 1, dtype=np.int64)
    np.add.at(indptr, krows + 1, 1)
    indptr = np.cumsum(indptr)
    return Bsr(indptr, kcols.astype(np.int64), data, A.nb), D_F, isolated


def prolongator_damping(A_F: Bsr, D_F: np.ndarray, isolated: np.ndarray) -> float:
    """omega = (4/3) / rho, rho the Gershgorin bound of D_F^-1 A_F."""
    Dinv = block_inverse(D_F)
    rows = _rows(A_F)
    scaled = block_product(Dinv[rows], A_F.data)  # blocks of D_F^-1 A_F
    absrow = np.zeros((A_F.nb, A_F.b))
    np.add.at(absrow, rows, np.sum(np.abs(scaled), axis=2))  # per unknown of the node
    live = ~isolated
    rho = float(absrow[live].max()) if live.any() else 1.0
    return (4.0 / 3.0) / rho


def tentative_prolongator(agg: np.ndarray, b: int) -> Bsr:
    n = agg.shape[0]
    nc = int(agg.max()) + 1 if n else 0
    live = agg >= 0
    indptr = np.concatenate([[0], np.cumsum(live.astype(np.int64))])
    data = np.broadcast_to(np.eye(b), (int(live.sum()), b, b)).copy()
    return Bsr(indptr, agg[live].astype(np.int64), data, n, nc)


def smoothed_prolongator(A_F: Bsr, D_F: np.ndarray, P_hat: Bsr, omega: float) -> Bsr:
    """P = P_hat - omega D_F^-1 (A_F P_hat)."""
    Y = spgemm(A_F, P_hat)
    Dinv = block_inverse(D_F)
    rows = _rows(Y)
    X = block_product(Dinv[rows], Y.data)
    # P_hat's blocks sit inside Y's pattern (the diagonal block of A_F is stored)
    hat = np.zeros_like(X)
    ph_rows = _rows(P_hat)
    key_y = rows * Y.ncb + Y.indices
    key_h = ph_rows * P_hat.ncb + P_hat.indices
    pos = np.searchsorted(key_y, key_h)
    hat[pos] = P_hat.data
    return Bsr(Y.indptr.copy(), Y.indices.copy(), hat - omega * X, Y.nb, Y.ncb)


def spai0_blocks(A: Bsr) -> np.ndarray:
    """M_i = A_ii^T (sum_j A_ij A_ij^T)^-1, sums in column order."""
    rows = _rows(A)
    G = block_product(A.data, np.transpose(A.data, (0, 2, 1)))
    acc = np.zeros((A.nb, A.b, A.b))
    np.add.at(acc, rows, G)
    D = diagonal_blocks(A)
    return block_product(np.transpose(D, (0, 2, 1)), block_inverse(acc))


def jacobi_blocks(A: Bsr, omega: float) -> np.ndarray:
    """M_i = omega A_ii^-1."""
    return omega * block_inverse(diagonal_blocks(A))


@dataclass
class BlockLevel:
    A: Bsr
    agg: np.ndarray | None = None
    P: Bsr | None = None
    R: Bsr | None = None
    M: np.ndarray | None = None  # smoother blocks, one per node
    omega: float | None = None
    # scalar forms used by the solve
    As: sp.csr_matrix | None = None
    Ps: sp.csr_matrix | None = None
    Rs: sp.csr_matrix | None = None
    Ms: sp.csr_matrix | None = None
    Mts: sp.csr_matrix | None = None  # transposed smoother blocks (post-sweeps)


@dataclass
class BlockHierarchy:
    levels: list
    lu: tuple
    params: sa_amg.Params
    b: int
    stats: dict = field(default_factory=dict)

    @property
    def nlevels(self) -> int:
        return len(self.levels)


def _block_diag(M: np.ndarray) -> sp.csr_matrix:
    n, b, _ = M.shape
    return Bsr(np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int64), M, n).to_scipy()


def setup(A: Bsr, params: sa_amg.Params | None = None) -> BlockHierarchy:
    """The block hierarchy (section 2, "AMG setup", blockwise).  The level
    size compared with coarse_enough is the number of unknowns (b nb)."""
    prm = params or sa_amg.Params()
    if prm.relax not in ("spai0", "jacobi"):
        raise ValueError("block values support the spai0 and jacobi smoothers")
    b = A.b
    levels = []
    stats = {"omega": [], "eps": []}
    while True:
        n = A.nb
        lvl_no = len(levels) + 1
        if b * n <= prm.coarse_enough or lvl_no == prm.max_levels:
            break
        eps = prm.eps_strong * 0.5 ** (lvl_no - 1)
        S = strength_graph(A, eps)
        agg = sa_amg.aggregate(S)
        nc = int(agg.max()) + 1 if n else 0
        if nc == 0 or nc >= n:
            break
        A_F, D_F, isolated = filtered_matrix(A, S)
        omega = prolongator_damping(A_F, D_F, isolated)
        P = smoothed_prolongator(A_F, D_F, tentative_prolongator(agg, b), omega)
        R = transpose(P)
        M = spai0_blocks(A) if prm.relax == "spai0" else jacobi_blocks(A, prm.jacobi_omega)
        levels.append(BlockLevel(A=A, agg=agg, P=P, R=R, M=M, omega=omega,
                                 As=A.to_scipy(), Ps=P.to_scipy(), Rs=R.to_scipy(), Ms=_block_diag(M),
                                 Mts=_block_diag(np.transpose(M, (0, 2, 1)))))
        stats["omega"].append(omega)
        stats["eps"].append(eps)
        A = spgemm(R, spgemm(A, P))
    if b * A.nb > prm.max_coarse:
        raise ValueError("coarsest level too large for a dense direct solve")
    levels.append(BlockLevel(A=A, As=A.to_scipy()))
    lu = sla.lu_factor(levels[-1].As.toarray())
    return BlockHierarchy(levels=levels, lu=lu, params=prm, b=b, stats=stats)


# --------------------------------------------------------------------------
# Solve
# --------------------------------------------------------------------------


def vcycle(h: BlockHierarchy, f: np.ndarray, level: int = 0) -> np.ndarray:
    """One V-cycle on ``level`` (0-based) with zero initial guess."""
    lv = h.levels[level]
    if level == h.nlevels - 1:
        return sla.lu_solve(h.lu, f)
    prm = h.params
    z = np.zeros_like(f)
    for _ in range(prm.npre):
        z = z + lv.Ms @ (f - lv.As @ z)
    r = f - lv.As @ z
    z_c = vcycle(h, lv.Rs @ r, level + 1)
    z = z + lv.Ps @ z_c
    for _ in range(prm.npost):
        z = z + lv.Mts @ (f - lv.As @ z)
    return z


def vcycle_fp32(h: BlockHierarchy, f: np.ndarray) -> np.ndarray:
    """The V-cycle on FP32 copies (round to nearest) of A_l, P_l, R_l and M_l
    with FP32 arithmetic; the coarsest solve stays FP64."""
    def cycle(level, f32):
        if level == h.nlevels - 1:
            return sla.lu_solve(h.lu, f32.astype(np.float64)).astype(np.float32)
        lv = h.levels[level]
        A, P, R, M, Mt = (m.astype(np.float32) for m in (lv.As, lv.Ps, lv.Rs, lv.Ms, lv.Mts))
        z = np.zeros_like(f32)
        for _ in range(h.params.npre):
            z = z + M @ (f32 - A @ z)
        r = f32 - A @ z
        z = z + P @ cycle(level + 1, R @ r)
        for _ in range(h.params.npost):
            z = z + Mt @ (f32 - A @ z)
        return z

    return cycle(0, np.asarray(f).astype(np.float32)).astype(np.float64)


def solve(A: Bsr, f: np.ndarray, params: sa_amg.Params | None = None, mixed: bool = False,
          h: BlockHierarchy | None = None):
    """AMG-preconditioned CG, BiCGStab or flexible GMRES on the scalar form of
    A; the Krylov methods are the scalar oracle's, one block V-cycle per
    preconditioning step."""
    prm = params or sa_amg.Params()
    if h is None:
        h = setup(A, prm)
    As = h.levels[0].As

    def precond(r):
        return vcycle_fp32(h, r) if mixed else vcycle(h, r)

    if prm.solver == "cg":
        x, info = sa_amg.pcg(As, f, precond, prm.tol, prm.max_iter)
    elif prm.solver == "bicgstab":
        x, info = sa_amg.bicgstab(As, f, precond, prm.tol, prm.max_iter)
    elif prm.solver == "gmres":
        x, info = sa_amg.gmres(As, f, precond, m=prm.gmres_m, tol=prm.tol, max_iter=prm.max_iter)
    else:
        raise ValueError("block values support cg, bicgstab and gmres")
    return x, info, h
