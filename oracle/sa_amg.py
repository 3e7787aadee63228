"""Oracle for smoothed-aggregation AMG as a preconditioner for CG and BiCGStab.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 NumPy /
SciPy, written for a reader who checks it against the paper by eye: no
blocking, no fusion, no reordering beyond what each step's definition says.
SciPy's sparse products, CSR transpose and LAPACK LU are used as library
primitives.

Where it comes from
-------------------
* Section 2, algorithm "AMG setup": start from A_1 = A; while A_i is too large
  for a direct solve, build P_i and R_i and form the Galerkin operator
  A_{i+1} = R_i A_i P_i with R = P^T; then build a direct solver for the
  coarsest A_L.                                     -> :func:`setup`
* Section 3, "Coarsening strategies": the transfer operators come from
  smoothed aggregation (Vanek, Mandel and Brezina, 1996, the paper's cited
  source).  Its steps: strength graph, greedy three-phase aggregation,
  piecewise-constant tentative prolongator, damped-Jacobi smoothing of it with
  the weak connections lumped into the diagonal (the "filtered" matrix).
                                                    -> :func:`strength_graph`,
  :func:`aggregate`, :func:`tentative_prolongator`, :func:`filtered_matrix`,
  :func:`prolongator_damping`, :func:`smoothed_prolongator`
* Section 3, "Relaxation methods": damped Jacobi and the sparse approximate
  inverse SPAI-0 (Broeker and Grote, 2002: the diagonal M minimising
  ||I - M A||_F row by row); Chebyshev relaxation as the diagonally scaled
  Chebyshev iteration of Saad 2003 (cited by the paper for its relaxation
  methods) on [hi/30, hi], hi the Gershgorin bound of D^-1 A.
                                            -> :func:`spai0_diagonal`,
  :func:`jacobi_diagonal`, :func:`chebyshev_sweep`
* Section 2, algorithm "AMG solve": one V-cycle -- pre-relaxation, residual,
  restriction on the way down; a direct solve on the coarsest level;
  prolongation with correction and post-relaxation on the way up.
                                                    -> :func:`vcycle`
* Section 2, closing remark: used as a preconditioner, a single V-cycle is
  one preconditioning step of a Krylov method (section 3 names CG and
  BiCGStab; the textbook forms of Saad 2003 and Barrett et al. 1994, both
  cited by the paper, are followed).                -> :func:`pcg`,
  :func:`bicgstab`
* Section 3, "Value types" (double or float): the mixed-precision form keeps
  the Krylov loop in FP64 and runs the V-cycle on an FP32 copy of the
  hierarchy with FP32 arithmetic; the coarse direct solve stays FP64.
                                                    -> :func:`vcycle_fp32`

Readings where the paper is silent (each is listed with its reason in the
design notes): strength threshold eps_l = eps * 2^-(l-1) and the squared
test a_ij^2 > eps_l^2 |a_ii a_jj|; the strong graph symmetrised by union; the
three aggregation phases in natural index order, a leftover node joining the
phase-1 aggregate of its lowest-index strong neighbour; unit (unnormalised)
tentative prolongator; weak entries lumped into the diagonal; damping
omega = (4/3) / rho with rho the Gershgorin bound of D_F^-1 A_F; no entry
dropped by value; zero initial guess on every level; recursive residual test
||r|| <= tol ||f|| followed by one restart if the true residual misses tol.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

# Aggregation markers.
UNAGGREGATED = -2
ISOLATED = -1


@dataclass
class Params:
    """Method parameters (the paper's nested ``params``, section 3.1, flattened)."""

    solver: str = "cg"  # "cg" | "bicgstab" | "gmres"
    relax: str = "spai0"  # "spai0" | "jacobi" | "chebyshev"
    eps_strong: float = 0.08  # strength threshold on level 1, halved per level
    jacobi_omega: float = 0.72
    cheb_degree: int = 3  # Chebyshev steps per sweep
    cheb_ratio: float = 30.0  # lower end of the Chebyshev interval = upper / ratio
    npre: int = 1
    npost: int = 1
    coarse_enough: int = 3000
    max_levels: int = 30
    max_coarse: int = 20000  # a coarsest level above this is refused
    max_iter: int = 500
    tol: float = 1e-8
    gmres_m: int = 30  # GMRES restart length


@dataclass
class Level:
    A: sp.csr_matrix
    agg: np.ndarray | None = None  # aggregate id per node, -1 = isolated
    P: sp.csr_matrix | None = None
    R: sp.csr_matrix | None = None
    m: np.ndarray | None = None  # smoother diagonal (Chebyshev: 1 / a_ii)
    omega: float | None = None  # prolongator damping
    cheb_hi: float | None = None  # Chebyshev: upper end of the spectrum bound of D^-1 A


@dataclass
class Hierarchy:
    levels: list  # levels 1..L; the last one is the coarsest
    lu: tuple  # scipy lu_factor of the coarsest matrix
    params: Params
    stats: dict = field(default_factory=dict)

    @property
    def nlevels(self) -> int:
        return len(self.levels)


def _as_csr(A) -> sp.csr_matrix:
    if hasattr(A, "to_scipy"):
        A = A.to_scipy()
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    return A


def _row_of_entry(A: sp.csr_matrix) -> np.ndarray:
    return np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))


# --------------------------------------------------------------------------
# Setup (section 2, "AMG setup"; section 3, smoothed aggregation)
# --------------------------------------------------------------------------


def strength_graph(A: sp.csr_matrix, eps: float) -> sp.csr_matrix:
    """Symmetrised strong-connection graph N_i (boolean CSR, no diagonal).

    j != i is a strong neighbour of i when a_ij^2 > eps^2 |a_ii a_jj|; the
    graph is then made symmetric, N_i <- N_i U {j : i in N_j}, so that
    nonsymmetric matrices get an undirected graph.
    """
    A = _as_csr(A)
    d = A.diagonal()
    rows = _row_of_entry(A)
    cols = A.indices
    vals = A.data
    strong = (cols != rows) & (vals * vals > eps * eps * np.abs(d[rows] * d[cols]))
    n = A.shape[0]
    S = sp.csr_matrix((np.ones(int(strong.sum()), dtype=np.int8), (rows[strong], cols[strong])),
                      shape=(n, n))
    S = ((S + S.T) > 0).astype(np.int8).tocsr()
    S.sort_indices()
    return S


def aggregate(S: sp.csr_matrix) -> np.ndarray:
    """Greedy three-phase aggregation over the strong graph, natural order.

    Phase 1: visit i = 0..n-1; an unaggregated, non-isolated node all of whose
    strong neighbours are unaggregated starts a new aggregate {i} U N_i.
    Phase 2: each node left over (and not isolated) joins the aggregate of its
    lowest-index strong neighbour that phase 1 aggregated (membership frozen
    at the end of phase 1).
    Phase 3: visit the nodes still left in natural order; each starts a new
    aggregate with its still-unaggregated strong neighbours.
    Aggregates are numbered in creation order; isolated nodes get -1.
    """
    n = S.shape[0]
    ptr = S.indptr.tolist()
    nbr = S.indices.tolist()
    agg = [UNAGGREGATED] * n
    count = 0
    for i in range(n):
        if ptr[i] == ptr[i + 1]:
            agg[i] = ISOLATED
    # phase 1
    for i in range(n):
        if agg[i] != UNAGGREGATED:
            continue
        neigh = nbr[ptr[i]:ptr[i + 1]]
        if all(agg[j] == UNAGGREGATED for j in neigh):
            agg[i] = count
            for j in neigh:
                agg[j] = count
            count += 1
    # phase 2
    after_phase1 = list(agg)
    for i in range(n):
        if agg[i] != UNAGGREGATED:
            continue
        for j in nbr[ptr[i]:ptr[i + 1]]:  # ascending: the first hit is the lowest index
            if after_phase1[j] >= 0:
                agg[i] = after_phase1[j]
                break
    # phase 3
    for i in range(n):
        if agg[i] != UNAGGREGATED:
            continue
        agg[i] = count
        for j in nbr[ptr[i]:ptr[i + 1]]:
            if agg[j] == UNAGGREGATED:
                agg[j] = count
        count += 1
    return np.array(agg, dtype=np.int64)


def tentative_prolongator(agg: np.ndarray) -> sp.csr_matrix:
    """P_hat[i, agg(i)] = 1 (piecewise constant, unnormalised); isolated rows empty."""
    n = agg.shape[0]
    nc = int(agg.max()) + 1 if n else 0
    rows = np.nonzero(agg >= 0)[0]
    return sp.csr_matrix((np.ones(rows.size), (rows, agg[rows])), shape=(n, nc))


def filtered_matrix(A: sp.csr_matrix, S: sp.csr_matrix) -> tuple[sp.csr_matrix, np.ndarray]:
    """A_F: strong off-diagonal entries of A kept, weak ones lumped into the diagonal.

    a_F(i,j) = a_ij for j in N_i; a_F(i,i) = a_ii + sum of the weak a_ij
    (so A_F times the constant vector equals A times it).  Returns (A_F, d_F),
    d_F being the diagonal of A_F; a non-isolated row whose lumped diagonal
    would not be positive keeps a_ii instead.
    """
    A = _as_csr(A)
    n = A.shape[0]
    rows = _row_of_entry(A)
    cols = A.indices
    vals = A.data
    in_graph = np.asarray(S[rows, cols]).ravel() != 0 if A.nnz else np.zeros(0, dtype=bool)
    offdiag = cols != rows
    weak = offdiag & ~in_graph
    lumped = np.zeros(n)
    np.add.at(lumped, rows[weak], vals[weak])
    a_diag = A.diagonal()
    d_F = a_diag + lumped
    isolated = np.diff(S.indptr) == 0
    bad = (~isolated) & (d_F <= 0.0)
    d_F = np.where(bad, a_diag, d_F)
    keep = offdiag & in_graph
    A_F = sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)) + sp.diags(d_F)
    A_F = A_F.tocsr()
    A_F.sort_indices()
    return A_F, d_F


def prolongator_damping(A_F: sp.csr_matrix, d_F: np.ndarray, isolated: np.ndarray) -> float:
    """omega = (4/3) / rho, rho = max_i sum_j |a_F(i,j)| / |a_F(i,i)| over non-isolated i.

    rho is the Gershgorin bound on the spectral radius of D_F^-1 A_F.
    """
    absrow = abs(A_F) @ np.ones(A_F.shape[0])  # row sums, entries in column order
    ratio = absrow / np.abs(d_F)
    live = ~isolated
    rho = float(ratio[live].max()) if live.any() else 1.0
    return (4.0 / 3.0) / rho


def smoothed_prolongator(A_F, d_F, P_hat, omega) -> sp.csr_matrix:
    """P = P_hat - omega D_F^-1 A_F P_hat (one damped-Jacobi step on each column)."""
    P = P_hat - omega * (sp.diags(1.0 / d_F) @ (A_F @ P_hat))
    P = sp.csr_matrix(P)
    P.sort_indices()
    return P


def spai0_diagonal(A: sp.csr_matrix) -> np.ndarray:
    """SPAI-0: m_i = a_ii / sum_j a_ij^2, the diagonal M minimising ||I - M A||_F."""
    A = _as_csr(A)
    rowsq = A.multiply(A) @ np.ones(A.shape[0])  # row sums, entries in column order
    return A.diagonal() / rowsq


def jacobi_diagonal(A: sp.csr_matrix, omega: float) -> np.ndarray:
    """Damped Jacobi: m_i = omega / a_ii."""
    return omega / _as_csr(A).diagonal()


def chebyshev_upper_bound(A: sp.csr_matrix) -> float:
    """Gershgorin bound of the spectrum of D^-1 A: max_i sum_j |a_ij| / |a_ii|."""
    A = _as_csr(A)
    absrow = abs(A) @ np.ones(A.shape[0])
    return float(np.max(absrow / np.abs(A.diagonal())))


def chebyshev_sweep(A, dinv, f, x, hi, lo, degree):
    """Diagonally scaled Chebyshev iteration (Saad 2003, Alg. 12.1, with the
    preconditioner D) of `degree` steps for A x = f from the guess x, for a
    spectrum of D^-1 A inside [lo, hi].  Returns (x, r) with r = f - A x.

    theta = (hi + lo) / 2, delta = (hi - lo) / 2, sigma = theta / delta;
    r = f - A x, rho = 1 / sigma, d = D^-1 r / theta; then repeatedly
    x += d, r -= A d, rho' = 1 / (2 sigma - rho),
    d = rho' rho d + (2 rho' / delta) D^-1 r.
    """
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    r = f - A @ x
    rho = 1.0 / sigma
    d = (dinv * r) / theta
    for step in range(degree):
        x = x + d
        r = r - A @ d
        if step == degree - 1:
            break
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        rho = rho_new
    return x, r


def chebyshev_sweep_fp32(A32, dinv32, f32, x32, hi, lo, degree):
    """:func:`chebyshev_sweep` in FP32 arithmetic (coefficients rounded to FP32)."""
    f32_ = np.float32
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    r = f32 - A32 @ x32
    rho = 1.0 / sigma
    d = (dinv32 * r) / f32_(theta)
    x = x32
    for step in range(degree):
        x = x + d
        r = r - A32 @ d
        if step == degree - 1:
            break
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = f32_(rho_new * rho) * d + f32_(2.0 * rho_new / delta) * (dinv32 * r)
        rho = rho_new
    return x, r


def setup(A, params: Params | None = None) -> Hierarchy:
    """Build the hierarchy (section 2, "AMG setup"), FP64."""
    prm = params or Params()
    A = _as_csr(A)
    levels = []
    stats = {"omega": [], "eps": []}
    while True:
        n = A.shape[0]
        lvl_no = len(levels) + 1  # 1-based number of the level being considered
        if n <= prm.coarse_enough or lvl_no == prm.max_levels:
            break
        eps = prm.eps_strong * 0.5 ** (lvl_no - 1)
        S = strength_graph(A, eps)
        agg = aggregate(S)
        nc = int(agg.max()) + 1 if n else 0
        if nc == 0 or nc >= n:
            break
        isolated = np.diff(S.indptr) == 0
        A_F, d_F = filtered_matrix(A, S)
        omega = prolongator_damping(A_F, d_F, isolated)
        P = smoothed_prolongator(A_F, d_F, tentative_prolongator(agg), omega)
        R = P.T.tocsr()
        R.sort_indices()
        cheb_hi = None
        if prm.relax == "spai0":
            m = spai0_diagonal(A)
        elif prm.relax == "jacobi":
            m = jacobi_diagonal(A, prm.jacobi_omega)
        elif prm.relax == "chebyshev":
            m = 1.0 / A.diagonal()
            cheb_hi = chebyshev_upper_bound(A)
        else:
            raise ValueError(prm.relax)
        levels.append(Level(A=A, agg=agg, P=P, R=R, m=m, omega=omega, cheb_hi=cheb_hi))
        stats["omega"].append(omega)
        stats["eps"].append(eps)
        Ac = (R @ (A @ P)).tocsr()
        Ac.sort_indices()
        A = Ac
    if A.shape[0] > prm.max_coarse:
        raise ValueError("coarsest level too large for a dense direct solve")
    levels.append(Level(A=A))
    lu = sla.lu_factor(A.toarray())
    return Hierarchy(levels=levels, lu=lu, params=prm, stats=stats)


# --------------------------------------------------------------------------
# Solve (section 2, "AMG solve"; one V-cycle per preconditioning step)
# --------------------------------------------------------------------------


def vcycle(h: Hierarchy, f: np.ndarray, level: int = 0) -> np.ndarray:
    """One V-cycle applied to f on ``level`` (0-based), zero initial guess."""
    lv = h.levels[level]
    if level == h.nlevels - 1:
        return sla.lu_solve(h.lu, f)
    prm = h.params
    z = np.zeros_like(f)
    if prm.relax == "chebyshev":
        # the residual restricted is the one the Chebyshev iteration carries
        lo = lv.cheb_hi / prm.cheb_ratio
        r = f
        for _ in range(prm.npre):
            z, r = chebyshev_sweep(lv.A, lv.m, f, z, lv.cheb_hi, lo, prm.cheb_degree)
        z = z + lv.P @ vcycle(h, lv.R @ r, level + 1)
        for _ in range(prm.npost):
            z, _r = chebyshev_sweep(lv.A, lv.m, f, z, lv.cheb_hi, lo, prm.cheb_degree)
        return z
    for _ in range(prm.npre):
        z = z + lv.m * (f - lv.A @ z)
    r = f - lv.A @ z
    f_c = lv.R @ r
    z_c = vcycle(h, f_c, level + 1)
    z = z + lv.P @ z_c
    for _ in range(prm.npost):
        z = z + lv.m * (f - lv.A @ z)
    return z


def hierarchy_fp32(h: Hierarchy) -> list:
    """FP32 copies (round to nearest) of A_l, P_l, R_l, m_l for l < L."""
    out = []
    for lv in h.levels[:-1]:
        out.append(dict(A=lv.A.astype(np.float32), P=lv.P.astype(np.float32),
                        R=lv.R.astype(np.float32), m=lv.m.astype(np.float32), cheb_hi=lv.cheb_hi))
    return out


def vcycle_fp32(h: Hierarchy, f: np.ndarray, h32: list | None = None) -> np.ndarray:
    """The V-cycle on the FP32 copy of the hierarchy, FP32 arithmetic throughout.

    f (FP64) is rounded to FP32 on entry and z returned as FP64; the coarsest
    level is solved with the FP64 LU (f_L widened, z_L rounded back).  SciPy's
    CSR product of FP32 operands accumulates in FP32.
    """
    if h32 is None:
        h32 = hierarchy_fp32(h)
    prm = h.params

    def cycle(level, f32):
        if level == h.nlevels - 1:
            return sla.lu_solve(h.lu, f32.astype(np.float64)).astype(np.float32)
        lv = h32[level]
        z = np.zeros_like(f32)
        if prm.relax == "chebyshev":
            hi = lv["cheb_hi"]
            lo = hi / prm.cheb_ratio
            r = f32
            for _ in range(prm.npre):
                z, r = chebyshev_sweep_fp32(lv["A"], lv["m"], f32, z, hi, lo, prm.cheb_degree)
            z = z + lv["P"] @ cycle(level + 1, lv["R"] @ r)
            for _ in range(prm.npost):
                z, _r = chebyshev_sweep_fp32(lv["A"], lv["m"], f32, z, hi, lo, prm.cheb_degree)
            return z
        for _ in range(prm.npre):
            z = z + lv["m"] * (f32 - lv["A"] @ z)
        r = f32 - lv["A"] @ z
        z_c = cycle(level + 1, lv["R"] @ r)
        z = z + lv["P"] @ z_c
        for _ in range(prm.npost):
            z = z + lv["m"] * (f32 - lv["A"] @ z)
        return z

    return cycle(0, np.asarray(f).astype(np.float32)).astype(np.float64)


@dataclass
class SolveInfo:
    iters: int
    rel_resid: float  # recursive residual at exit, relative to ||f||
    true_rel_resid: float
    converged: bool
    restarts: int = 0
    history: list = field(default_factory=list)


def pcg(A, f, precond, tol=1e-8, max_iter=500, x0=None):
    """Preconditioned CG (Saad 2003, Alg. 9.1), recursive residual test.

    The iteration count is the number of products q = A p.  Convergence is
    ||r|| <= tol ||f|| checked after each update of x; if the true residual
    then misses tol, the iteration restarts once from the current x (the count
    continues).
    """
    A = _as_csr(A)
    f = np.asarray(f, dtype=np.float64)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    nf = float(np.linalg.norm(f))
    if nf == 0.0:
        return np.zeros_like(f), SolveInfo(0, 0.0, 0.0, True)
    it = 0
    hist = []
    restarts = 0
    rel = 0.0
    converged = False
    for attempt in range(2):
        r = f - A @ x
        rel = float(np.linalg.norm(r)) / nf
        if rel <= tol:
            converged = True
        else:
            z = precond(r)
            p = z.copy()
            rho = float(r @ z)
            while it < max_iter:
                q = A @ p
                alpha = rho / float(p @ q)
                x = x + alpha * p
                r = r - alpha * q
                it += 1
                rel = float(np.linalg.norm(r)) / nf
                hist.append(rel)
                if rel <= tol:
                    converged = True
                    break
                z = precond(r)
                rho_new = float(r @ z)
                beta = rho_new / rho
                p = z + beta * p
                rho = rho_new
        true_rel = float(np.linalg.norm(f - A @ x)) / nf
        if not converged or true_rel <= tol or attempt == 1:
            break
        restarts += 1
        converged = False
    true_rel = float(np.linalg.norm(f - A @ x)) / nf
    return x, SolveInfo(it, rel, true_rel, converged and true_rel <= tol, restarts, hist)


class Breakdown(RuntimeError):
    pass


def bicgstab(A, f, precond, tol=1e-8, max_iter=500, x0=None):
    """Right-preconditioned BiCGStab (Barrett et al. 1994, "Templates").

    One iteration applies the preconditioner twice.  The test ||s|| <= tol
    ||f|| after the first half-step ends the iteration early (x += alpha
    p_hat); otherwise ||r|| <= tol ||f|| after the full step.  rho = 0 or
    omega = 0 is a breakdown.  Restart rule as in :func:`pcg`.
    """
    A = _as_csr(A)
    f = np.asarray(f, dtype=np.float64)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    nf = float(np.linalg.norm(f))
    if nf == 0.0:
        return np.zeros_like(f), SolveInfo(0, 0.0, 0.0, True)
    it = 0
    hist = []
    restarts = 0
    rel = 0.0
    converged = False
    for attempt in range(2):
        r = f - A @ x
        rel = float(np.linalg.norm(r)) / nf
        if rel <= tol:
            converged = True
        else:
            rt = r.copy()
            rho_old = alpha = omega = 1.0
            v = np.zeros_like(f)
            p = np.zeros_like(f)
            first = True
            while it < max_iter:
                rho = float(rt @ r)
                if rho == 0.0:
                    raise Breakdown("rho = 0")
                if first:
                    p = r.copy()
                    first = False
                else:
                    beta = (rho / rho_old) * (alpha / omega)
                    p = r + beta * (p - omega * v)
                p_hat = precond(p)
                v = A @ p_hat
                alpha = rho / float(rt @ v)
                s = r - alpha * v
                it += 1
                rel = float(np.linalg.norm(s)) / nf
                if rel <= tol:
                    x = x + alpha * p_hat
                    hist.append(rel)
                    converged = True
                    break
                s_hat = precond(s)
                t = A @ s_hat
                omega = float(t @ s) / float(t @ t)
                x = x + alpha * p_hat + omega * s_hat
                r = s - omega * t
                rel = float(np.linalg.norm(r)) / nf
                hist.append(rel)
                if rel <= tol:
                    converged = True
                    break
                if omega == 0.0:
                    raise Breakdown("omega = 0")
                rho_old = rho
        true_rel = float(np.linalg.norm(f - A @ x)) / nf
        if not converged or true_rel <= tol or attempt == 1:
            break
        restarts += 1
        converged = False
    true_rel = float(np.linalg.norm(f - A @ x)) / nf
    return x, SolveInfo(it, rel, true_rel, converged and true_rel <= tol, restarts, hist)


def arnoldi_cgs2(A, precond, V, j):
    """One Arnoldi step of flexible GMRES from the orthonormal basis V[0..j]:
    z = M v_j, w = A z, orthogonalised against every v_i by classical
    Gram-Schmidt applied twice (Giraud, Langou and Rozloznik 2005).  Returns
    (z, h, hn, w): the preconditioned vector, the coefficients h_i (the two
    passes added), hn = ||w|| and w (not normalised)."""
    z = precond(V[j])
    w = A @ z
    h = np.zeros(j + 1)
    for _ in range(2):
        c = np.array([float(V[i] @ w) for i in range(j + 1)])  # against the same w
        for i in range(j + 1):
            w = w - c[i] * V[i]
        h = h + c
    return z, h, float(np.sqrt(w @ w)), w


def gmres(A, f, precond, m=30, tol=1e-8, max_iter=500, x0=None):
    """Flexible restarted GMRES(m) (Saad 1993; Saad 2003, Alg. 9.6, restarted
    as in section 6.5.5), Arnoldi by :func:`arnoldi_cgs2`, Givens rotations
    for the least-squares problem.  The preconditioned vectors z_j = M v_j
    are kept, so the update x += Z_k y is exact also when M is linear only up
    to rounding (the FP32 V-cycle); for a fixed linear M this is right-
    preconditioned GMRES (Saad 2003, Alg. 9.5).

    One iteration is one Arnoldi step (one preconditioner application and
    one product with A).  After each step the least-squares residual |g_{j+1}|
    is tested against tol ||f||; a cycle ends on that test, on h_{j+1,j} = 0
    or after m steps, and then x += Z_k y.  Every cycle starts from the true
    residual f - A x, whose norm decides convergence, so a cycle whose
    estimate met tol but whose true residual does not simply continues.
    """
    A = _as_csr(A)
    f = np.asarray(f, dtype=np.float64)
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    nf = float(np.linalg.norm(f))
    if nf == 0.0:
        return np.zeros_like(f), SolveInfo(0, 0.0, 0.0, True)
    it = 0
    hist = []
    cycles = 0
    rel = 0.0
    converged = False
    while True:
        r = f - A @ x
        beta = float(np.sqrt(r @ r))
        rel = beta / nf
        if rel <= tol:
            converged = True
            break
        if it >= max_iter:
            break
        cycles += 1
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            z, h, hn, w = arnoldi_cgs2(A, precond, V, j)
            Z.append(z)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):  # earlier rotations
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            a, b = H[j, j], H[j + 1, j]
            d = float(np.sqrt(a * a + b * b))
            cs[j], sn[j] = a / d, b / d
            H[j, j], H[j + 1, j] = d, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            rel = abs(g[j + 1]) / nf
            hist.append(rel)
            if rel <= tol or hn == 0.0 or it >= max_iter:
                break
            V.append(w / hn)
        y = np.zeros(k)  # back substitution, H[:k, :k] upper triangular
        for i in range(k - 1, -1, -1):
            s_ = g[i]
            for c in range(i + 1, k):
                s_ = s_ - H[i, c] * y[c]
            y[i] = s_ / H[i, i]
        for i in range(k):
            x = x + y[i] * Z[i]
    true_rel = float(np.linalg.norm(f - A @ x)) / nf
    return x, SolveInfo(it, rel, true_rel, converged, max(cycles - 1, 0), hist)


def solve(A, f, params: Params | None = None, mixed: bool = False, h: Hierarchy | None = None):
    """Setup (unless ``h`` is given) and AMG-preconditioned Krylov solve.

    Returns (x, info, h).  ``mixed`` selects the FP32 V-cycle as preconditioner.
    """
    prm = params or Params()
    if h is None:
        h = setup(A, prm)
    if mixed:
        h32 = hierarchy_fp32(h)

        def M(r):
            return vcycle_fp32(h, r, h32)
    else:
        def M(r):
            return vcycle(h, r)
    if prm.solver == "gmres":
        x, info = gmres(h.levels[0].A, f, M, m=prm.gmres_m, tol=prm.tol, max_iter=prm.max_iter)
    else:
        krylov = pcg if prm.solver == "cg" else bicgstab
        x, info = krylov(h.levels[0].A, f, M, tol=prm.tol, max_iter=prm.max_iter)
    return x, info, h
