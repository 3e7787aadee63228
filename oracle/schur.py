"""Oracle for the Schur-complement pressure-correction field split.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain FP64 NumPy /
SciPy; SciPy's sparse products and LU are library primitives.

Where it comes from
-------------------
* Section 3, "Extensibility", and section 4 (the Navier-Stokes runs): the
  system of a velocity/pressure discretisation is split by field,
  ``A = [[K, G], [D, S]]`` (velocity unknowns first), and preconditioned in
  two steps; the pressure block is preconditioned with smoothed-aggregation
  AMG and the velocity block with SPAI-0.  The paper defers the method to its
  cited sources (Verfuerth 1984; Gmeiner et al. 2016).  Their two-step form
  is the block LU factorisation

      A = [[K, 0], [D, S_c]] [[I, K^-1 G], [0, I]],   S_c = S - D K^-1 G,

  whose inverse is applied to r = (r_u, r_p) as
      u* = K^-1 r_u,   p = S_c^-1 (r_p - D u*),   u = u* - K^-1 G p.
                                              -> :func:`field_split_apply`
  With exact inner solves this is A^-1 r (the pin of the step order).
* The approximate form: K^-1 is replaced by the SPAI-0 diagonal M_u of K;
  the Schur complement by the sparse S_hat = S - D diag(K)^-1 G (the
  classical SIMPLE choice); S_hat^-1 by one V-cycle of the smoothed
  aggregation hierarchy of S_hat (:mod:`oracle.sa_amg`).
                                        -> :func:`schur_matrix`, :func:`setup`,
  :func:`precond`
* The outer iteration is a nonsymmetric Krylov method (the preconditioner is
  not symmetric): BiCGStab or flexible GMRES from :mod:`oracle.sa_amg`.
                                                    -> :func:`solve`

Readings where the paper is silent (listed with their reasons in the design
notes): one V-cycle (no inner iteration) as the pressure solve; one
application of M_u as each velocity solve; diag(K) in S_hat; the
mixed-precision form runs only the pressure V-cycle in FP32.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import sa_amg


@dataclass
class Blocks:
    K: sp.csr_matrix  # velocity-velocity
    G: sp.csr_matrix  # velocity rows, pressure columns
    D: sp.csr_matrix  # pressure rows, velocity columns
    S: sp.csr_matrix  # pressure-pressure
    n_u: int


def split(A, n_u: int) -> Blocks:
    """The four field blocks of A, velocity unknowns 0..n_u-1 first."""
    A = sa_amg._as_csr(A)
    return Blocks(A[:n_u, :n_u].tocsr(), A[:n_u, n_u:].tocsr(), A[n_u:, :n_u].tocsr(),
                  A[n_u:, n_u:].tocsr(), n_u)


def schur_matrix(b: Blocks) -> sp.csr_matrix:
    """S_hat = S - D diag(K)^-1 G, the sparse approximate Schur complement.

    Each entry's products are summed in ascending velocity index k (the
    columns of D diag(K)^-1 are put in order before the product)."""
    dinv = sp.diags(1.0 / b.K.diagonal())
    Dk = (b.D @ dinv).tocsr()
    Dk.sort_indices()
    Sh = (b.S - Dk @ b.G).tocsr()
    Sh.sum_duplicates()
    Sh.sort_indices()
    return Sh


def field_split_apply(b: Blocks, r: np.ndarray, vel_solve, p_solve) -> np.ndarray:
    """One application of the two-step preconditioner with the given inner
    solves (vel_solve ~ K^-1, p_solve ~ S_c^-1)."""
    r_u, r_p = r[: b.n_u], r[b.n_u:]
    u_star = vel_solve(r_u)
    p = p_solve(r_p - b.D @ u_star)
    u = u_star - vel_solve(b.G @ p)
    return np.concatenate([u, p])


@dataclass
class SchurSetup:
    blocks: Blocks
    m_u: np.ndarray  # SPAI-0 diagonal of K
    S_hat: sp.csr_matrix
    h: sa_amg.Hierarchy  # smoothed-aggregation hierarchy of S_hat


def setup(A, n_u: int, params: sa_amg.Params | None = None) -> SchurSetup:
    b = split(A, n_u)
    Sh = schur_matrix(b)
    return SchurSetup(b, sa_amg.spai0_diagonal(b.K), Sh, sa_amg.setup(Sh, params))


def precond(ss: SchurSetup, mixed: bool = False):
    """The approximate field split as a function r -> z."""
    if mixed:
        h32 = sa_amg.hierarchy_fp32(ss.h)

        def p_solve(x):
            return sa_amg.vcycle_fp32(ss.h, x, h32)
    else:
        def p_solve(x):
            return sa_amg.vcycle(ss.h, x)

    def M(r):
        return field_split_apply(ss.blocks, r, lambda x: ss.m_u * x, p_solve)

    return M


def solve(A, f, n_u: int, params: sa_amg.Params | None = None, mixed: bool = False,
          ss: SchurSetup | None = None):
    """Setup (unless ``ss`` is given) and the field-split preconditioned
    BiCGStab or GMRES solve.  Returns (x, info, ss)."""
    prm = params or sa_amg.Params(solver="bicgstab")
    if prm.solver not in ("bicgstab", "gmres"):
        raise ValueError("the field split is not symmetric: BiCGStab or GMRES")
    if ss is None:
        ss = setup(A, n_u, prm)
    M = precond(ss, mixed)
    A = sa_amg._as_csr(A)
    if prm.solver == "gmres":
        x, info = sa_amg.gmres(A, f, M, m=prm.gmres_m, tol=prm.tol, max_iter=prm.max_iter)
    else:
        x, info = sa_amg.bicgstab(A, f, M, tol=prm.tol, max_iter=prm.max_iter)
    return x, info, ss
