"""Pins for the oracle (CPU only).

Each test checks the oracle against something other than itself: the
hand-derived worked example, closed forms, invariants the mathematics fixes,
special cases that reduce to a dense solve, and brute force on tiny grids.
"""

import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import problems


def load_golden(path):
    out = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = [Fraction(v) for v in vals]
    return out


@pytest.fixture(scope="module")
def pw(golden_dir):
    return load_golden(os.path.join(golden_dir, "pw_1d_laplacian.txt"))


def _f(vals):
    return np.array([float(v) for v in vals])


def pw_hierarchy():
    A = problems.tridiag1d(9)
    return oracle.setup(A, oracle.Params(coarse_enough=3))


# ---------------------------------------------------------------- worked example


def test_worked_example_setup(pw):
    h = pw_hierarchy()
    assert h.nlevels == 2
    lv = h.levels[0]
    assert lv.agg.tolist() == [int(a) for a in pw["agg"]]
    assert lv.omega == pytest.approx(float(pw["omega"][0]), abs=1e-16)
    P = _f(pw["P"]).reshape(9, 3)
    assert np.max(np.abs(lv.P.toarray() - P)) <= 1e-15
    assert np.array_equal(lv.R.toarray(), lv.P.toarray().T)
    Ac = _f(pw["Ac"]).reshape(3, 3)
    assert np.max(np.abs(h.levels[1].A.toarray() - Ac)) <= 1e-15
    assert np.max(np.abs(lv.m - _f(pw["m"]))) <= 1e-16


def test_worked_example_vcycle(pw):
    h = pw_hierarchy()
    lv = h.levels[0]
    r = np.ones(9)
    z0 = lv.m * r
    f_c = lv.R @ (r - lv.A @ z0)
    assert np.max(np.abs(f_c - _f(pw["f_c"]))) <= 4e-15
    z_c = oracle.vcycle(h, f_c, 1)
    assert np.max(np.abs(z_c - _f(pw["z_c"]))) / 10.2 <= 1e-15
    V = oracle.vcycle(h, r)
    ref = _f(pw["V"])
    assert np.max(np.abs(V - ref)) / np.max(np.abs(ref)) <= 1e-15


# ---------------------------------------------------------------- closed forms


def test_spai0_closed_form_poisson():
    N = 6
    A = problems.poisson3d(N).to_scipy()
    m = oracle.spai0_diagonal(A)
    idx = np.arange(N**3)
    c = [idx % N, (idx // N) % N, idx // (N * N)]
    nb = sum(((ci > 0).astype(int) + (ci < N - 1).astype(int)) for ci in c)
    # a_ii = 6, sum_j a_ij^2 = 36 + (number of neighbours)
    expect = 6.0 / (36.0 + nb)
    assert np.array_equal(m, expect)
    assert m[idx[(nb == 6)][0]] == 6.0 / 42.0  # interior 1/7
    assert set(np.round(1.0 / m * 6).astype(int).tolist()) == {39, 40, 41, 42}


def test_jacobi_diagonal_closed_form():
    A = problems.poisson3d(4).to_scipy()
    m = oracle.jacobi_diagonal(A, 0.72)
    assert np.allclose(m, 0.12, rtol=0, atol=1e-17)


def test_level1_poisson_all_strong_and_filter_identity():
    A = problems.poisson3d(6).to_scipy()
    S = oracle.strength_graph(A, 0.08)
    off = A - sp.diags(A.diagonal())
    off.eliminate_zeros()
    assert (S != (off != 0)).nnz == 0
    A_F, d_F = oracle.filtered_matrix(A, S)
    assert abs(A_F - A).max() == 0
    isolated = np.diff(S.indptr) == 0
    assert oracle.prolongator_damping(A_F, d_F, isolated) == pytest.approx(2.0 / 3.0, abs=1e-16)


def test_strength_threshold_is_strict_and_squared():
    # 2x2 with a_01^2 exactly eps^2 a_00 a_11 is weak; slightly above is strong.
    eps = 0.25
    a00, a11 = 4.0, 1.0
    a01 = -eps * np.sqrt(a00 * a11)  # = -0.5, exact in binary
    for val, expect in ((a01, 0), (a01 * 1.0000001, 1)):
        A = sp.csr_matrix(np.array([[a00, val], [val, a11]]))
        S = oracle.strength_graph(A, eps)
        assert S.nnz == 2 * expect


def test_strength_symmetrised_for_nonsymmetric():
    A = sp.csr_matrix(np.array([[1.0, -0.5, 0.0], [-0.01, 1.0, -0.5], [0.0, -0.5, 1.0]]))
    S = oracle.strength_graph(A, 0.08).toarray()
    assert np.array_equal(S, S.T)
    assert S[0, 1] == 1 and S[1, 0] == 1  # 1->0 weak, but 0->1 strong


def test_filtered_matrix_lumps_weak_entries():
    A = sp.csr_matrix(np.array([[4.0, -1.0, -0.01], [-1.0, 4.0, -1.0], [-0.01, -1.0, 4.0]]))
    S = oracle.strength_graph(A, 0.08)
    A_F, d_F = oracle.filtered_matrix(A, S)
    D = A_F.toarray()
    assert D[0, 2] == 0 and D[2, 0] == 0
    assert D[0, 0] == pytest.approx(3.99) and D[1, 1] == 4.0
    assert np.allclose(D.sum(axis=1), A.toarray().sum(axis=1))


# ---------------------------------------------------------------- invariants


def _check_partition(S, agg):
    n = S.shape[0]
    isolated = np.diff(S.indptr) == 0
    assert np.all(agg[isolated] == -1)
    assert np.all(agg[~isolated] >= 0)
    nc = agg.max() + 1
    assert set(np.unique(agg[agg >= 0]).tolist()) == set(range(nc))
    # each aggregate is connected in the strong graph
    for a in range(nc):
        members = np.nonzero(agg == a)[0]
        sub = S[members][:, members]
        ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
        assert ncomp == 1
    return nc


@pytest.mark.parametrize("case", ["poisson", "diffusion", "convection"])
def test_aggregation_invariants(case):
    N = 10
    if case == "poisson":
        A = problems.poisson3d(N).to_scipy()
    elif case == "diffusion":
        A = problems.diffusion3d(N, problems.gaussian_field(N, 2.0, 8.0, 1)).to_scipy()
    else:
        A = problems.diffusion3d(N, problems.gaussian_field(N, 2.0, 8.0, 1),
                                 velocity=(50.0, 25.0, 12.5)).to_scipy()
    S = oracle.strength_graph(A, 0.08)
    agg = oracle.aggregate(S)
    nc = _check_partition(S, agg)
    assert 0 < nc < A.shape[0]
    assert np.array_equal(agg, oracle.aggregate(S))


def _graph(n, edges):
    r = [a for a, b in edges] + [b for a, b in edges]
    c = [b for a, b in edges] + [a for a, b in edges]
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))


def test_aggregation_phase1_natural_order():
    # path 0-...-6 plus isolated node 7: node 0 -> {0,1}; node 2 touches the
    # aggregated 1 -> skipped; node 3 -> {2,3,4}; node 5 skipped; node 6 -> {5,6}
    S = _graph(8, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 6)])
    assert oracle.aggregate(S).tolist() == [0, 0, 1, 1, 1, 2, 2, -1]


def test_aggregation_phase2_joins_lowest_index_neighbour():
    # node 4 touches node 1 (aggregate 0) and node 3 (aggregate 1): it joins the
    # aggregate of the lower-index neighbour, node 1
    S = _graph(5, [(0, 1), (2, 3), (1, 4), (3, 4)])
    assert oracle.aggregate(S).tolist() == [0, 0, 1, 1, 0]
    # and with the indices of the two aggregates' members swapped it follows them
    S = _graph(5, [(0, 3), (1, 2), (3, 4), (1, 4)])
    # phase 1: node 0 -> {0,3}; node 1 -> {1,2}; node 4 touches 1 and 3 -> lowest is 1
    assert oracle.aggregate(S).tolist() == [0, 1, 1, 0, 1]


def test_aggregation_partition_random_graphs():
    rng = np.random.default_rng(7)
    for _ in range(20):
        n = 60
        M = sp.random(n, n, density=0.05, random_state=rng, format="csr")
        S = ((M + M.T) > 0).astype(np.int8).tocsr()
        S.setdiag(0)
        S.eliminate_zeros()
        S.sort_indices()
        agg = oracle.aggregate(S)
        _check_partition(S, agg)


def test_prolongator_rowsum_invariant():
    N = 8
    A = problems.poisson3d(N).to_scipy()
    h = oracle.setup(A, oracle.Params(coarse_enough=50))
    P = h.levels[0].P
    rowsum = np.asarray(P.sum(axis=1)).ravel()
    zero_rows = np.abs(np.asarray(A.sum(axis=1)).ravel()) == 0
    assert zero_rows.sum() > 0
    assert np.max(np.abs(rowsum[zero_rows] - 1.0)) <= 1e-15
    # boundary rows lose mass (A row sum > 0) -> P row sums < 1
    assert np.all(rowsum[~zero_rows] < 1.0)


@pytest.mark.parametrize("case", ["poisson", "diffusion"])
def test_galerkin_symmetric_spd(case):
    N = 12
    if case == "poisson":
        A = problems.poisson3d(N).to_scipy()
    else:
        A = problems.diffusion3d(N, problems.gaussian_field(N, 2.0, 8.0, 1)).to_scipy()
    h = oracle.setup(A, oracle.Params(coarse_enough=30))
    assert h.nlevels >= 3
    for l in range(1, h.nlevels):
        Ac = h.levels[l].A.toarray()
        assert np.max(np.abs(Ac - Ac.T)) <= 1e-14 * np.max(np.abs(Ac))
        np.linalg.cholesky(Ac)
        # Galerkin identity against the dense triple product
        prev = h.levels[l - 1]
        dense = prev.P.toarray().T @ prev.A.toarray() @ prev.P.toarray()
        assert np.max(np.abs(Ac - dense)) <= 1e-13 * np.max(np.abs(dense))


def test_two_grid_closed_form():
    # npre = npost = 0, two levels: V(r) = P A_c^-1 R r
    A = problems.poisson3d(6).to_scipy()
    prm = oracle.Params(coarse_enough=100, npre=0, npost=0)
    h = oracle.setup(A, prm)
    assert h.nlevels == 2
    P = h.levels[0].P.toarray()
    Ac = h.levels[1].A.toarray()
    r = np.random.default_rng(1).standard_normal(A.shape[0])
    expect = P @ np.linalg.solve(Ac, P.T @ r)
    got = oracle.vcycle(h, r)
    assert np.max(np.abs(got - expect)) <= 1e-13 * np.max(np.abs(expect))


def _vcycle_matrix(h, n):
    return np.column_stack([oracle.vcycle(h, e) for e in np.eye(n)])


@pytest.mark.parametrize("relax", ["spai0", "jacobi"])
def test_vcycle_operator_symmetric_spd_linear(relax):
    N = 7
    A = problems.poisson3d(N).to_scipy()
    h = oracle.setup(A, oracle.Params(coarse_enough=10, relax=relax))
    assert h.nlevels >= 3
    B = _vcycle_matrix(h, A.shape[0])
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal((2, A.shape[0]))
    lhs = oracle.vcycle(h, 2.5 * x - 0.75 * y)
    rhs = 2.5 * oracle.vcycle(h, x) - 0.75 * oracle.vcycle(h, y)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14 * np.max(np.abs(rhs))


def test_single_level_is_exact():
    A = problems.poisson3d(10)  # 1000 unknowns <= 3000: one level, V = A^-1
    f = problems.rhs_ones(A.n)
    h = oracle.setup(A)
    assert h.nlevels == 1
    x, info, _ = oracle.solve(A, f, h=h)
    assert info.iters == 1
    xd = np.linalg.solve(A.to_scipy().toarray(), f)
    assert np.max(np.abs(x - xd)) / np.max(np.abs(xd)) < 1e-13
    x, info, _ = oracle.solve(A, f, oracle.Params(solver="bicgstab"), h=h)
    assert info.iters == 1


def _tiny_cases():
    out = []
    for N in (3, 5, 8):
        out.append(("poisson", N, problems.poisson3d(N), "cg", "spai0"))
    g = problems.gaussian_field(8, 2.0, 8.0, 1)
    out.append(("diffusion", 8, problems.diffusion3d(8, g), "cg", "spai0"))
    out.append(("diffusion-bicg", 8, problems.diffusion3d(8, g), "bicgstab", "jacobi"))
    out.append(("convection", 8, problems.diffusion3d(8, g, velocity=(50.0, 25.0, 12.5)),
                "bicgstab", "jacobi"))
    out.append(("convection-gmres", 8, problems.diffusion3d(8, g, velocity=(50.0, 25.0, 12.5)),
                "gmres", "jacobi"))
    out.append(("poisson-gmres", 5, problems.poisson3d(5), "gmres", "spai0"))
    return out


@pytest.mark.parametrize("name,N,A,solver,relax", _tiny_cases(), ids=lambda v: str(v) if isinstance(v, (str, int)) else "")
def test_whole_solve_vs_dense(name, N, A, solver, relax):
    f = problems.rhs_uniform(A.n, seed=0)
    prm = oracle.Params(solver=solver, relax=relax, coarse_enough=20)
    x, info, h = oracle.solve(A, f, prm)
    D = A.to_scipy().toarray()
    xd = np.linalg.solve(D, f)
    kappa = np.linalg.cond(D)
    assert info.converged
    assert info.true_rel_resid <= 1e-8
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= kappa * 1e-8


def test_mesh_independent_iterations():
    its = []
    for N in (16, 24, 32, 40, 48):
        A = problems.poisson3d(N)
        _, info, h = oracle.solve(A, problems.rhs_uniform(A.n, 0), oracle.Params())
        assert info.converged
        its.append(info.iters)
    assert max(its) / min(its) <= 1.5, its


def test_mixed_vcycle_is_fp32_close_but_not_fp64():
    A = problems.poisson3d(16)
    h = oracle.setup(A)
    r = problems.rhs_uniform(A.n, 0)
    z64 = oracle.vcycle(h, r)
    z32 = oracle.vcycle_fp32(h, r)
    rel = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 1e-9 < rel < 1e-5


def test_fp32_csr_product_accumulates_in_fp32():
    # The mixed oracle relies on SciPy's FP32 CSR product accumulating in FP32.
    n = 4000
    rng = np.random.default_rng(0)
    row = np.zeros(n, dtype=np.int64)
    col = np.arange(n)
    val = rng.random(n).astype(np.float32)
    x = rng.random(n).astype(np.float32)
    A = sp.csr_matrix((val, (row, col)), shape=(1, n))
    y = (A @ x)[0]
    assert y.dtype == np.float32
    acc = np.float32(0)
    for v, xx in zip(val, x):
        acc = np.float32(acc + np.float32(v * xx))
    assert y == acc


def test_pcg_and_bicgstab_report_iterations_and_zero_rhs():
    A = problems.poisson3d(16)
    f0 = np.zeros(A.n)
    x, info, _ = oracle.solve(A, f0)
    assert info.iters == 0 and not x.any()
    x, info, _ = oracle.solve(A, problems.rhs_ones(A.n), oracle.Params(max_iter=1))
    assert info.iters == 1 and not info.converged


def test_coarse_lu_solves_coarsest_system():
    A = problems.poisson3d(16)
    h = oracle.setup(A)
    Ac = h.levels[-1].A.toarray()
    b = np.random.default_rng(3).standard_normal(Ac.shape[0])
    z = oracle.vcycle(h, b, h.nlevels - 1)
    assert np.linalg.norm(Ac @ z - b) / np.linalg.norm(b) < 1e-13


# ---------------------------------------------------------------- Chebyshev smoother


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_chebyshev_residual_polynomial_closed_form(degree):
    # 1-D Laplacian, D = 2I: D^-1 A has eigenvalues mu_j = 1 - cos(j pi/(n+1)) with
    # eigenvectors sin(i j pi/(n+1)).  One sweep from zero multiplies the residual of
    # an eigenvector by T_k((theta - mu)/delta) / T_k(theta/delta).
    from numpy.polynomial import chebyshev as C

    n = 30
    A = problems.tridiag1d(n).to_scipy()
    hi = oracle.chebyshev_upper_bound(A)
    assert hi == 2.0  # interior rows (1 + 2 + 1) / 2
    lo = hi / 30.0
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    Tk = np.zeros(degree + 1)
    Tk[-1] = 1.0
    dinv = 1.0 / A.diagonal()
    idx = np.arange(1, n + 1)
    for j in (1, 3, 7, 15, 29):
        v = np.sin(idx * j * np.pi / (n + 1))
        mu = 1.0 - np.cos(j * np.pi / (n + 1))
        x, r = oracle.chebyshev_sweep(A, dinv, v, np.zeros(n), hi, lo, degree)
        expect = C.chebval((theta - mu) / delta, Tk) / C.chebval(theta / delta, Tk)
        assert np.max(np.abs(r - expect * v)) <= 1e-13
        assert np.max(np.abs((v - A @ x) - r)) <= 1e-13


def test_chebyshev_vcycle_symmetric_spd_linear_and_solve():
    N = 7
    A = problems.poisson3d(N).to_scipy()
    prm = oracle.Params(coarse_enough=10, relax="chebyshev")
    h = oracle.setup(A, prm)
    assert h.nlevels >= 3
    B = _vcycle_matrix(h, A.shape[0])
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal((2, A.shape[0]))
    lhs = oracle.vcycle(h, 1.5 * x - 2.0 * y)
    rhs = 1.5 * oracle.vcycle(h, x) - 2.0 * oracle.vcycle(h, y)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14 * np.max(np.abs(rhs))
    A8 = problems.poisson3d(8)
    f = problems.rhs_uniform(A8.n, 1)
    xs, info, _ = oracle.solve(A8, f, oracle.Params(relax="chebyshev", coarse_enough=20))
    xd = np.linalg.solve(A8.to_scipy().toarray(), f)
    assert info.converged and np.linalg.norm(xs - xd) / np.linalg.norm(xd) <= 1e-6
    # the FP32 V-cycle follows the same polynomial
    z64 = oracle.vcycle(h, x)
    z32 = oracle.vcycle_fp32(h, x)
    assert 1e-10 < np.linalg.norm(z32 - z64) / np.linalg.norm(z64) < 1e-5


# ------------------------------------------------------------------ GMRES


def _nonsym_small(n=40, seed=7):
    """Dense-backed nonsymmetric test matrix 3 I + B / sqrt(n), B Gaussian."""
    rng = np.random.default_rng(seed)
    return sp.csr_matrix(3.0 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n))


def test_gmres_minimal_residual_over_krylov_space():
    # k steps of one cycle minimise ||f - A x|| over x = M u, u in the Krylov
    # space K_k(A M, f): compare with a dense least-squares problem on an
    # orthonormal basis of that space (QR of [f, B f, ..., B^(k-1) f], B = A M)
    A = _nonsym_small()
    n = A.shape[0]
    dM = 1.0 + np.random.default_rng(8).random(n)  # a fixed diagonal preconditioner
    f = np.random.default_rng(9).standard_normal(n)
    B = A.toarray() * dM[None, :]
    nf = np.linalg.norm(f)
    for k in range(1, 9):
        x, info = oracle.gmres(A, f, lambda v: dM * v, m=50, tol=1e-300, max_iter=k)
        assert info.iters == k
        K = np.column_stack([np.linalg.matrix_power(B, i) @ f for i in range(k)])
        Q, _ = np.linalg.qr(K)
        c = np.linalg.lstsq(B @ Q, f, rcond=None)[0]
        best = np.linalg.norm(f - B @ (Q @ c))
        got = np.linalg.norm(f - A @ x)
        assert abs(got - best) <= 1e-10 * nf, (k, got, best)
        # the least-squares estimate of the last step is the true residual
        assert abs(info.history[-1] - got / nf) <= 1e-11


def test_gmres_arnoldi_relation_and_orthonormal_basis():
    A = _nonsym_small()
    n, k = A.shape[0], 10
    dM = 1.0 + np.random.default_rng(8).random(n)
    f = np.random.default_rng(10).standard_normal(n)
    V, Z = [f / np.linalg.norm(f)], []
    Hb = np.zeros((k + 1, k))
    for j in range(k):
        z, h, hn, w = oracle.arnoldi_cgs2(A, lambda v: dM * v, V, j)
        np.testing.assert_array_equal(z, dM * V[j])
        Z.append(z)
        Hb[: j + 1, j] = h
        Hb[j + 1, j] = hn
        V.append(w / hn)
    Vm, Zm = np.column_stack(V), np.column_stack(Z)
    assert np.abs(Vm.T @ Vm - np.eye(k + 1)).max() <= 1e-14
    assert np.abs(A @ Zm - Vm @ Hb).max() <= 1e-13 * np.abs(A).max()


def test_gmres_finite_termination_and_restarts():
    A = _nonsym_small(12, 3)
    f = np.random.default_rng(4).standard_normal(12)
    nf = np.linalg.norm(f)
    x, info = oracle.gmres(A, f, lambda v: v, m=12, tol=1e-12, max_iter=100)
    assert info.converged and info.iters <= 12 and info.restarts == 0
    assert np.linalg.norm(f - A @ x) <= 1e-12 * nf
    x3, info3 = oracle.gmres(A, f, lambda v: v, m=3, tol=1e-10, max_iter=500)
    assert info3.converged and info3.restarts > 0
    assert np.linalg.norm(f - A @ x3) <= 1e-10 * nf
    # each cycle minimises over a space that holds the zero correction, so
    # the residual never grows, also across restarts
    hist = np.array(info3.history)
    assert np.all(np.diff(hist) <= 1e-12)


def test_flexible_gmres_exact_with_fp32_vcycle():
    # the stored z_j make the update exact for the FP32 V-cycle: the solve
    # reaches tol in one cycle, like the FP64 one
    A = problems.poisson3d(16)
    f = problems.rhs_uniform(A.n, 0)
    x, info, h = oracle.solve(A, f, oracle.Params(solver="gmres"), mixed=True)
    x64, info64, _ = oracle.solve(A, f, oracle.Params(solver="gmres"), h=h)
    assert info.converged and info64.converged
    assert info.restarts == 0 and info64.restarts == 0
    assert abs(info.iters - info64.iters) <= 1


# ------------------------------------------------------------------ Krylov recurrences
#
# PCG and BiCGStab are pinned by what their iterates are in exact arithmetic,
# computed here by dense linear algebra on small systems with a fixed diagonal
# preconditioner M (Saad 2003, Prop. 9.1 / Thm. 6.6 for CG; van der Vorst 1992
# for BiCGStab's residual polynomial).


def _orth_krylov(apply, v, k):
    """Orthonormal basis (columns) of span{v, Bv, ..., B^(k-1) v}, B given by ``apply``:
    each new vector is B times the last basis vector, orthogonalised twice."""
    Q = []
    w = np.array(v, dtype=np.float64)
    for _ in range(k):
        for _pass in range(2):
            for q in Q:
                w = w - (q @ w) * q
        Q.append(w / np.linalg.norm(w))
        w = apply(Q[-1])
    return np.column_stack(Q)


def test_pcg_iterate_minimises_energy_error_over_krylov_space():
    # From x0 = 0, PCG's k-th iterate is the point of K_k(M A, M f) closest to
    # A^-1 f in the A-norm: x_k = Q (Q^T A Q)^-1 Q^T f for any basis Q of it.
    A = problems.poisson3d(4).to_scipy()
    n = A.shape[0]
    Ad = A.toarray()
    rng = np.random.default_rng(11)
    dM = 1.0 + rng.random(n)  # fixed SPD diagonal preconditioner
    f = rng.standard_normal(n)
    xs = np.linalg.solve(Ad, f)
    enorm = np.sqrt(xs @ Ad @ xs)
    nf = np.linalg.norm(f)
    for k in range(1, 9):
        x, info = oracle.pcg(A, f, lambda v: dM * v, tol=1e-300, max_iter=k)
        assert info.iters == k
        Q = _orth_krylov(lambda v: dM * (Ad @ v), dM * f, k)
        best = Q @ np.linalg.solve(Q.T @ Ad @ Q, Q.T @ f)
        e = x - best
        assert np.sqrt(e @ Ad @ e) <= 1e-12 * enorm, k
        # the recursively updated residual is the true one
        assert abs(info.rel_resid - np.linalg.norm(f - Ad @ x) / nf) <= 1e-12


def test_bicgstab_residual_is_product_of_stabilising_and_bicg_polynomials():
    # Right preconditioning, B = A M, x0 = 0, shadow vector r~ = r0 = f.  After
    # k steps r_k = psi_k(B) phi_k(B) r0, where phi_k(B) r0 is the BiCG
    # residual (in r0 + B K_k(B, r0), orthogonal to K_k(B^T, r~)) and
    # psi_k(t) = prod_j (1 - omega_j t), each omega_j minimising the 2-norm of
    # (I - omega B) psi_{j-1}(B) phi_j(B) r0.
    A = _nonsym_small()
    n = A.shape[0]
    Ad = A.toarray()
    rng = np.random.default_rng(12)
    dM = 1.0 + rng.random(n)
    f = rng.standard_normal(n)
    B = Ad * dM[None, :]
    r0 = f.copy()
    omegas = []
    for k in range(1, 7):
        Q = _orth_krylov(lambda v: B @ v, r0, k)
        Qs = _orth_krylov(lambda v: B.T @ v, r0, k)
        c = np.linalg.solve(Qs.T @ B @ Q, Qs.T @ r0)
        s = r0 - B @ (Q @ c)  # phi_k(B) r0
        for w in omegas:  # psi_{k-1}(B) phi_k(B) r0
            s = s - w * (B @ s)
        t = B @ s
        omega = (t @ s) / (t @ t)
        omegas.append(omega)
        rk = s - omega * t
        x, info = oracle.bicgstab(A, f, lambda v: dM * v, tol=1e-300, max_iter=k)
        assert info.iters == k
        assert np.linalg.norm((f - Ad @ x) - rk) <= 1e-12 * np.linalg.norm(f), k


# ------------------------------------------------------------------ FP32 V-cycle


def _is_nearest_fp32(v32, v64):
    """Every entry of v32 (float32) is a float32 nearest to the FP64 value."""
    v32 = np.asarray(v32)
    assert v32.dtype == np.float32
    up = np.nextafter(v32, np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(v32, np.float32(-np.inf)).astype(np.float64)
    d = np.abs(v32.astype(np.float64) - v64)
    return bool(np.all(d <= np.abs(up - v64)) and np.all(d <= np.abs(dn - v64)))


def test_hierarchy_fp32_is_the_rounded_fp64_hierarchy():
    A = problems.poisson3d(10)
    h = oracle.setup(A, oracle.Params(coarse_enough=100))
    assert h.nlevels >= 3
    h32 = oracle.hierarchy_fp32(h)
    assert len(h32) == h.nlevels - 1
    for lv, l32 in zip(h.levels[:-1], h32):
        for key in "APR":
            M64, M32 = getattr(lv, key), l32[key]
            assert M32.dtype == np.float32, key
            assert np.array_equal(M32.indptr, M64.indptr) and np.array_equal(M32.indices, M64.indices)
            assert _is_nearest_fp32(M32.data, M64.data), key
        assert l32["m"].dtype == np.float32 and _is_nearest_fp32(l32["m"], lv.m)


def test_fp32_vcycle_single_level_is_the_fp64_solve_rounded_once():
    # One level: the FP32 V-cycle is the FP64 direct solve of the FP32-rounded
    # right-hand side, rounded to FP32 once, so each entry is within half a
    # float32 ulp (<= 2^-24 |z|) of the dense FP64 solution (kappa ~ 1.6e4 here,
    # so an FP32 factorisation would be off by ~1e-3).
    A = problems.tridiag1d(200)
    h = oracle.setup(A)
    assert h.nlevels == 1
    f = np.random.default_rng(13).standard_normal(A.n)
    z = oracle.vcycle_fp32(h, f)
    ex = np.linalg.solve(A.to_scipy().toarray(), f.astype(np.float32).astype(np.float64))
    bound = 2.0 ** -24 * np.abs(ex) + 1e-10 * np.max(np.abs(ex))
    assert np.all(np.abs(z - ex) <= bound)


def test_fp32_two_grid_closed_form_within_rounding_bound():
    # npre = npost = 0, two levels: V32(r) = P32 fl32(A_c^-1 (R32 r32)) with
    # FP32 sums.  Against the same expression in exact arithmetic (FP64 dense,
    # the FP32 matrices' values, the FP64 coarse matrix), every entry is within
    # the componentwise rounding bound: gamma_k = k u / (1 - k u), u = 2^-24,
    # on the restriction and prolongation sums of at most k terms, propagated
    # through |A_c^-1|, plus one rounding of z_c.
    A = problems.poisson3d(6).to_scipy()
    h = oracle.setup(A, oracle.Params(coarse_enough=100, npre=0, npost=0))
    assert h.nlevels == 2
    h32 = oracle.hierarchy_fp32(h)
    P = h32[0]["P"].astype(np.float64).toarray()
    R = h32[0]["R"].astype(np.float64).toarray()
    Ac = h.levels[1].A.toarray()
    r = np.random.default_rng(14).standard_normal(A.shape[0])
    r32 = r.astype(np.float32).astype(np.float64)
    zc = np.linalg.solve(Ac, R @ r32)
    expect = P @ zc
    got = oracle.vcycle_fp32(h, r, h32)
    u = 2.0 ** -24

    def gamma(k):
        return k * u / (1.0 - k * u)

    kR = int(np.max(np.count_nonzero(R, axis=1)))
    kP = int(np.max(np.count_nonzero(P, axis=1)))
    dfc = gamma(kR) * (np.abs(R) @ np.abs(r32))
    dzc = np.abs(np.linalg.inv(Ac)) @ dfc
    dzc = dzc + u * (np.abs(zc) + dzc)
    bound = np.abs(P) @ dzc + gamma(kP) * (np.abs(P) @ (np.abs(zc) + dzc))
    assert np.all(np.abs(got - expect) <= bound + 1e-14 * np.max(np.abs(expect)))
    # and it is an FP32 result, not the FP64 one
    assert np.max(np.abs(got - oracle.vcycle(h, r))) > 1e-9 * np.max(np.abs(expect))
