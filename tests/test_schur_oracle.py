"""Pins of the field-split oracle (CPU only).

Each pin holds for reasons outside the oracle's own code: the block LU
identity (exact inner solves invert A), the element-by-element definition of
the approximate Schur complement on a tiny dense system, its stencil on the
Stokes grid worked out by hand, the closed form of SPAI-0 on the velocity
block, and a whole solve against a direct solve.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import sa_amg, schur
from problems.stokes import stokes3d, stokes_rhs


def _generic_blocks(seed=3, n_u=12, n_p=5):
    """A nonsymmetric two-field system whose D is not -G^T and whose K is not
    diagonal, so that a swapped or transposed block is seen."""
    rng = np.random.default_rng(seed)
    n = n_u + n_p
    M = np.zeros((n, n))
    K = rng.standard_normal((n_u, n_u)) * (rng.random((n_u, n_u)) < 0.3)
    K += np.diag(np.abs(K).sum(axis=1) + 2.0 + rng.random(n_u))
    G = rng.standard_normal((n_u, n_p)) * (rng.random((n_u, n_p)) < 0.4)
    D = rng.standard_normal((n_p, n_u)) * (rng.random((n_p, n_u)) < 0.4)
    S = rng.standard_normal((n_p, n_p)) * 0.1
    S += np.diag(3.0 + rng.random(n_p))
    M[:n_u, :n_u], M[:n_u, n_u:], M[n_u:, :n_u], M[n_u:, n_u:] = K, G, D, S
    return sp.csr_matrix(M), n_u


def test_exact_inner_solves_invert_the_system():
    """Block LU: with u* = K^-1 r_u, p = S_c^-1 (r_p - D u*), u = u* - K^-1 G p
    and S_c = S - D K^-1 G, the field split applies A^-1."""
    A, n_u = _generic_blocks()
    b = schur.split(A, n_u)
    Kd, Gd, Dd, Sd = (x.toarray() for x in (b.K, b.G, b.D, b.S))
    Sc = Sd - Dd @ np.linalg.solve(Kd, Gd)
    rng = np.random.default_rng(7)
    for _ in range(3):
        r = rng.standard_normal(A.shape[0])
        z = schur.field_split_apply(b, r, lambda x: np.linalg.solve(Kd, x), lambda y: np.linalg.solve(Sc, y))
        np.testing.assert_allclose(z, np.linalg.solve(A.toarray(), r), rtol=1e-11, atol=1e-12)


def test_schur_matrix_elementwise_definition():
    """S_hat_ij = S_ij - sum_k D_ik G_kj / K_kk, summed term by term."""
    A, n_u = _generic_blocks(seed=11)
    Ad = A.toarray()
    n_p = Ad.shape[0] - n_u
    want = np.zeros((n_p, n_p))
    for i in range(n_p):
        for j in range(n_p):
            acc = Ad[n_u + i, n_u + j]
            for k in range(n_u):
                acc -= Ad[n_u + i, k] * Ad[k, n_u + j] / Ad[k, k]
            want[i, j] = acc
    got = schur.schur_matrix(schur.split(A, n_u)).toarray()
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)


def test_schur_matrix_stencil_on_the_stokes_grid():
    """On the Stokes grid S_hat = beta L + G^T G / kappa (kappa = 6 + alpha,
    the velocity diagonal): -beta on the six neighbours, -h^2 / (4 kappa) two
    steps away along an axis when the midpoint is inside, and on the
    diagonal 6 beta plus h^2 / (4 kappa) per in-grid axis neighbour."""
    N, alpha = 5, 2.0
    A, n_u = stokes3d(N, alpha=alpha)
    h = 1.0 / (N + 1)
    beta, kappa = h * h / 12.0, 6.0 + alpha
    Sh = schur.schur_matrix(schur.split(A.to_scipy(), n_u)).toarray()
    want = np.zeros_like(Sh)

    def inside(c):
        return all(0 <= v < N for v in c)

    def idx(c):
        return c[0] + N * c[1] + N * N * c[2]

    for x in range(N):
        for y in range(N):
            for z in range(N):
                c = (x, y, z)
                i = idx(c)
                want[i, i] = 6.0 * beta
                for d in range(3):
                    for sgn in (1, -1):
                        e1 = list(c)
                        e1[d] += sgn
                        if not inside(e1):
                            continue
                        want[i, idx(e1)] -= beta
                        want[i, i] += h * h / (4.0 * kappa)
                        e2 = list(c)
                        e2[d] += 2 * sgn
                        if inside(e2):
                            want[i, idx(e2)] -= h * h / (4.0 * kappa)
    np.testing.assert_allclose(Sh, want, rtol=1e-13, atol=1e-17)


def test_diagonal_velocity_solve_with_exact_schur_inverts_the_lumped_system():
    """With vel_solve = diag(K)^-1 and the exact inverse of S_hat the split is
    the inverse of [[diag(K), G], [D, S]]: the SIMPLE factorisation."""
    A, n_u = _generic_blocks(seed=5)
    b = schur.split(A, n_u)
    Sh = schur.schur_matrix(b).toarray()
    dk = b.K.diagonal()
    Ahat = A.toarray().copy()
    Ahat[:n_u, :n_u] = np.diag(dk)
    r = np.random.default_rng(2).standard_normal(A.shape[0])
    z = schur.field_split_apply(b, r, lambda x: x / dk, lambda y: np.linalg.solve(Sh, y))
    np.testing.assert_allclose(Ahat @ z, r, rtol=1e-11, atol=1e-12)


def test_velocity_spai0_closed_form():
    """SPAI-0 of K = alpha I + L: kappa / (kappa^2 + #neighbours)."""
    N, alpha = 4, 2.0
    A, n_u = stokes3d(N, alpha=alpha)
    ss = schur.setup(A.to_scipy(), n_u)
    kappa = 6.0 + alpha
    n = N**3
    for comp in range(3):
        for i in range(n):
            c = (i % N, (i // N) % N, i // (N * N))
            nb = sum((v > 0) + (v < N - 1) for v in c)
            assert ss.m_u[comp * n + i] == pytest.approx(kappa / (kappa * kappa + nb), rel=1e-14)


@pytest.mark.parametrize("solver", ["bicgstab", "gmres"])
def test_whole_solve_vs_direct(solver):
    N = 8
    A, n_u = stokes3d(N)
    f = stokes_rhs(N)
    x, info, ss = schur.solve(A.to_scipy(), f, n_u, sa_amg.Params(solver=solver, tol=1e-10))
    assert info.converged
    want = spla.spsolve(A.to_scipy().tocsc(), f)
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-8 * np.abs(want).max())


def test_mixed_pressure_cycle_converges_to_the_same_solution():
    N = 10
    A, n_u = stokes3d(N)
    f = stokes_rhs(N)
    prm = sa_amg.Params(solver="bicgstab", coarse_enough=200)
    x64, i64, ss = schur.solve(A.to_scipy(), f, n_u, prm)
    x32, i32, _ = schur.solve(A.to_scipy(), f, n_u, prm, mixed=True, ss=ss)
    assert ss.h.nlevels >= 2
    assert i64.converged and i32.converged
    assert abs(i64.iters - i32.iters) <= 2
    np.testing.assert_allclose(x32, x64, rtol=0, atol=1e-6 * np.abs(x64).max())


def test_symmetric_krylov_refused():
    A, n_u = stokes3d(3)
    with pytest.raises(ValueError):
        schur.solve(A.to_scipy(), stokes_rhs(3), n_u, sa_amg.Params(solver="cg"))
