"""Pins of the block-value oracle (CPU only).

Section 3, "Value types": a matrix whose entries are small dense blocks.
The block oracle (``oracle/block_amg.py``) is pinned by what mathematics and
the scalar method fix, not by itself:

* its block primitives against dense NumPy (inverse, products, transpose);
* block size 1 reduces it to the scalar oracle (same aggregates, operators
  and V-cycle up to rounding), which has its own pins;
* four decoupled fields (A_ij = a_ij diag(c)) give four scalar AMGs: the
  block V-cycle equals the scalar V-cycles of c_k A field by field;
* block SPAI-0 is the block-diagonal least-squares minimiser of
  ||I - M A||_F (computed here with a dense least-squares solve);
* Galerkin operators equal the dense P^T A P; with no sweeps the two-grid
  cycle is P A_c^-1 R; the V-cycle of a symmetric positive definite coupled
  system is symmetric, positive definite and linear;
* permuting the fields of every node permutes the V-cycle the same way;
* whole solves against a dense solve;
* planted mistakes (a missing transpose, a wrong tentative block, a skipped
  inverse, a swapped product) are caught by these pins.
"""

import inspect
import textwrap

import numpy as np
import pytest
import scipy.sparse as sp

import oracle.block_amg as ba
import oracle.sa_amg as sa
import problems


def _bsr(M: "problems.BSR") -> ba.Bsr:
    return ba.Bsr(M.row_ptr.astype(np.int64), M.col.astype(np.int64), M.blocks().copy(), M.nb)


def _scalar_as_bsr(A) -> ba.Bsr:
    return ba.Bsr(A.row_ptr.astype(np.int64), A.col.astype(np.int64), A.val.reshape(-1, 1, 1).copy(), A.n)


def _random_bsr(nb, b, density, seed, diag_shift=4.0):
    rng = np.random.default_rng(seed)
    mask = rng.random((nb, nb)) < density
    np.fill_diagonal(mask, True)
    rows, cols = np.nonzero(mask)
    data = rng.standard_normal((rows.size, b, b))
    data[rows == cols] += diag_shift * np.eye(b)
    indptr = np.zeros(nb + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    return ba.Bsr(np.cumsum(indptr), cols.astype(np.int64), data, nb)


# ------------------------------------------------------------------ primitives


def test_block_inverse_matches_dense_inverse():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((200, 4, 4))
    B[:50, 0, 0] = 0.0  # forces a row exchange
    inv = ba.block_inverse(B)
    ref = np.linalg.inv(B)
    assert np.max(np.abs(inv - ref) / np.max(np.abs(ref), axis=(1, 2))[:, None, None]) <= 1e-11
    assert np.allclose(np.einsum("nij,njk->nik", B, inv), np.eye(4), atol=1e-11)


def test_block_product_spgemm_and_transpose_match_dense():
    X = _random_bsr(30, 4, 0.15, 2)
    Y = _random_bsr(30, 4, 0.15, 3)
    C = ba.spgemm(X, Y)
    Xd, Yd = X.to_scipy().toarray(), Y.to_scipy().toarray()
    assert np.allclose(C.to_scipy().toarray(), Xd @ Yd, rtol=0, atol=1e-12)
    assert np.all(np.diff(C.indptr) >= 0) and C.indptr[-1] == C.indices.size
    for i in range(C.nb):
        assert np.all(np.diff(C.indices[C.indptr[i]:C.indptr[i + 1]]) > 0)
    T = ba.transpose(X)
    assert np.array_equal(T.to_scipy().toarray(), Xd.T)
    T2 = ba.block_product(X.data[:5], Y.data[:5])
    assert np.allclose(T2, X.data[:5] @ Y.data[:5], rtol=0, atol=1e-13)


def test_strength_closed_form_two_nodes():
    # ||t I||_F^2 = 4 t^2 and ||d I||_F^2 = 4 d^2: strong iff |t| > eps |d|
    for t, expect in ((0.081, 1), (0.079, 0)):
        data = np.stack([np.eye(4), -t * np.eye(4), -t * np.eye(4), np.eye(4)])
        A = ba.Bsr(np.array([0, 2, 4]), np.array([0, 1, 0, 1]), data, 2)
        S = ba.strength_graph(A, 0.08)
        assert S.nnz == 2 * expect


# ------------------------------------------------------------------ reductions


def _scalar_cases():
    return [
        (problems.poisson3d(12), {}),
        (problems.diffusion3d(10, problems.gaussian_field(10, 2.0, 8.0, 1)), {}),
        (problems.diffusion3d(10, problems.gaussian_field(10, 2.0, 8.0, 1), velocity=(50.0, 25.0, 12.5)),
         {"relax": "jacobi"}),
    ]


@pytest.mark.parametrize("case", range(3))
def test_block_size_one_is_the_scalar_method(case):
    A, kw = _scalar_cases()[case]
    prm = sa.Params(coarse_enough=100, **kw)
    hs = sa.setup(A, prm)
    hb = ba.setup(_scalar_as_bsr(A), prm)
    assert hb.nlevels == hs.nlevels >= 3
    for ls, lb in zip(hs.levels[:-1], hb.levels[:-1]):
        assert np.array_equal(ls.agg, lb.agg)
        assert abs(ls.omega - lb.omega) <= 1e-14 * ls.omega
        for a, b in ((ls.P, lb.Ps), (ls.R, lb.Rs)):
            assert abs(a - b).max() <= 1e-13 * abs(a).max()
        assert np.max(np.abs(ls.m - lb.Ms.diagonal())) <= 1e-13 * np.max(np.abs(ls.m))
    assert abs(hs.levels[-1].A - hb.levels[-1].As).max() <= 1e-12 * abs(hs.levels[-1].A).max()
    f = np.random.default_rng(4).standard_normal(A.n)
    zs, zb = sa.vcycle(hs, f), ba.vcycle(hb, f)
    assert np.linalg.norm(zs - zb) <= 1e-12 * np.linalg.norm(zs)


@pytest.mark.parametrize("npre,npost", [(1, 1), (2, 3), (0, 2), (3, 0)])
def test_decoupled_fields_are_four_scalar_amgs(npre, npost):
    N = 12
    g = problems.gaussian_field(N, 1.0, 8.0, 3)
    L = problems.diffusion3d(N, g)
    B = problems.decoupled_diffusion3d(N, g)
    c = np.diag(problems.blocks.DECOUPLED)
    hb = ba.setup(_bsr(B), sa.Params(coarse_enough=4 * 60, npre=npre, npost=npost))
    f = np.random.default_rng(5).standard_normal(B.n)
    zb = ba.vcycle(hb, f)
    for k in range(4):
        Ak = problems.CSR(L.n, L.row_ptr, L.col, c[k] * L.val)
        hs = sa.setup(Ak, sa.Params(coarse_enough=60, npre=npre, npost=npost))
        assert hs.nlevels == hb.nlevels >= 3
        for ls, lb in zip(hs.levels[:-1], hb.levels[:-1]):
            assert np.array_equal(ls.agg, lb.agg)
        zk = sa.vcycle(hs, f[k::4])
        assert np.linalg.norm(zb[k::4] - zk) <= 1e-12 * np.linalg.norm(zk), k


# ------------------------------------------------------------------ smoother


def test_block_spai0_is_the_least_squares_minimiser():
    A = _random_bsr(25, 4, 0.2, 6)
    M = ba.spai0_blocks(A)
    Ad = A.to_scipy().toarray()
    b = 4
    for i in range(A.nb):
        Bi = Ad[b * i:b * (i + 1), :]  # block row i of A
        Ei = np.zeros_like(Bi)
        Ei[:, b * i:b * (i + 1)] = np.eye(b)
        # min ||E_i - M_i B_i||_F  <=>  B_i^T M_i^T ~ E_i^T
        Mt, *_ = np.linalg.lstsq(Bi.T, Ei.T, rcond=None)
        assert np.allclose(M[i], Mt.T, rtol=0, atol=1e-10 * np.abs(Mt).max())


def test_block_jacobi_inverts_the_diagonal_blocks():
    A = _random_bsr(20, 4, 0.2, 7)
    M = ba.jacobi_blocks(A, 0.72)
    D = ba.diagonal_blocks(A)
    assert np.allclose(np.einsum("nij,njk->nik", M, D), 0.72 * np.eye(4), atol=1e-12)


# ------------------------------------------------------------------ hierarchy and cycle


def _coupled(N=8, **kw):
    return _bsr(problems.coupled_diffusion3d(N, problems.gaussian_field(N, 1.0, 8.0, 2), **kw))


def test_galerkin_is_dense_ptap_and_spd():
    h = ba.setup(_coupled(), sa.Params(coarse_enough=4 * 30))
    assert h.nlevels >= 3
    for l in range(h.nlevels - 1):
        lv, nxt = h.levels[l], h.levels[l + 1]
        A, P = lv.As.toarray(), lv.Ps.toarray()
        Ac = nxt.As.toarray()
        assert np.allclose(Ac, P.T @ A @ P, rtol=0, atol=1e-12 * np.abs(Ac).max())
        assert np.array_equal(lv.Rs.toarray(), P.T)
        assert np.max(np.abs(Ac - Ac.T)) <= 1e-13 * np.abs(Ac).max()
        assert np.linalg.eigvalsh(Ac).min() > 0


def test_tentative_blocks_are_identities_on_aggregates():
    A = _coupled()
    S = ba.strength_graph(A, 0.08)
    agg = sa.aggregate(S)
    Ph = ba.tentative_prolongator(agg, 4).to_scipy().toarray()
    ref = np.kron(sa.tentative_prolongator(agg).toarray(), np.eye(4))
    assert np.array_equal(Ph, ref)


def _dense_block_diag(D):
    n, b, _ = D.shape
    out = np.zeros((n * b, n * b))
    for i in range(n):
        out[b * i:b * (i + 1), b * i:b * (i + 1)] = D[i]
    return out


def test_prolongator_is_one_damped_block_jacobi_step_on_the_tentative_basis():
    """P = (I - omega D_F^-1 A_F) P_hat evaluated densely with LAPACK solves,
    and omega = (4/3) / rho with rho the dense Gershgorin bound of D_F^-1 A_F,
    which bounds its spectral radius."""
    A = _coupled(5)
    S = ba.strength_graph(A, 0.08)
    agg = sa.aggregate(S)
    A_F, D_F, iso = ba.filtered_matrix(A, S)
    omega = ba.prolongator_damping(A_F, D_F, iso)
    P = ba.smoothed_prolongator(A_F, D_F, ba.tentative_prolongator(agg, 4), omega)
    AFd, Dd = A_F.to_scipy().toarray(), _dense_block_diag(D_F)
    DinvA = np.linalg.solve(Dd, AFd)
    live = np.repeat(~iso, 4)
    rho = np.abs(DinvA).sum(axis=1)[live].max()
    assert abs(omega - (4.0 / 3.0) / rho) <= 1e-12 * omega
    assert np.max(np.abs(np.linalg.eigvals(DinvA))) <= rho * (1 + 1e-12)
    Ph = np.kron(sa.tentative_prolongator(agg).toarray(), np.eye(4))
    ref = Ph - omega * (DinvA @ Ph)
    assert np.allclose(P.to_scipy().toarray(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_two_grid_closed_form_without_sweeps():
    prm = sa.Params(coarse_enough=4 * 200, npre=0, npost=0)
    h = ba.setup(_coupled(), prm)
    assert h.nlevels == 2
    lv = h.levels[0]
    r = np.random.default_rng(8).standard_normal(lv.As.shape[0])
    P, R, Ac = lv.Ps.toarray(), lv.Rs.toarray(), h.levels[1].As.toarray()
    ref = P @ np.linalg.solve(Ac, R @ r)
    assert np.linalg.norm(ba.vcycle(h, r) - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("relax,sweeps", [("spai0", 1), ("jacobi", 1), ("spai0", 2), ("jacobi", 3)])
def test_vcycle_operator_symmetric_spd_linear(relax, sweeps):
    # equal pre- and post-sweep counts, the post-sweeps applying M^T: the
    # V-cycle is a symmetric positive definite linear operator
    A = _coupled(5)
    h = ba.setup(A, sa.Params(coarse_enough=24, relax=relax, npre=sweeps, npost=sweeps))
    assert h.nlevels >= 3
    n = A.nb * 4
    Bm = np.column_stack([ba.vcycle(h, e) for e in np.eye(n)])
    assert np.max(np.abs(Bm - Bm.T)) <= 1e-12 * np.abs(Bm).max()
    assert np.linalg.eigvalsh(0.5 * (Bm + Bm.T)).min() > 0
    rng = np.random.default_rng(9)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    lhs = ba.vcycle(h, 2.0 * x - 3.0 * y)
    assert np.linalg.norm(lhs - (2.0 * ba.vcycle(h, x) - 3.0 * ba.vcycle(h, y))) <= 1e-12 * np.linalg.norm(lhs)


def test_field_permutation_permutes_the_vcycle():
    A = _coupled()
    perm = np.array([2, 0, 3, 1])
    Q = np.eye(4)[perm]
    Ap = ba.Bsr(A.indptr, A.indices, np.einsum("ij,njk,lk->nil", Q, A.data, Q), A.nb)
    prm = sa.Params(coarse_enough=4 * 30)
    h, hp = ba.setup(A, prm), ba.setup(Ap, prm)
    f = np.random.default_rng(10).standard_normal(4 * A.nb)
    fp = f.reshape(-1, 4)[:, perm].reshape(-1)
    z, zp = ba.vcycle(h, f), ba.vcycle(hp, fp)
    assert np.linalg.norm(zp - z.reshape(-1, 4)[:, perm].reshape(-1)) <= 1e-12 * np.linalg.norm(z)


@pytest.mark.parametrize("kind", ["cg-spai0", "cg-jacobi", "bicgstab-jacobi-convection"])
def test_whole_block_solve_vs_dense(kind):
    solver, relax = kind.split("-")[:2]
    vel = (50.0, 25.0, 12.5) if kind.endswith("convection") else None
    A = _coupled(7, velocity=vel)
    f = problems.random_block_rhs(A.nb, 4, 11)
    prm = sa.Params(solver=solver, relax=relax, coarse_enough=4 * 20)
    x, info, h = ba.solve(A, f, prm)
    assert h.nlevels >= 3 and info.converged and info.true_rel_resid <= 1e-8
    xd = np.linalg.solve(A.to_scipy().toarray(), f)
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)


def test_fp32_vcycle_close_to_but_distinct_from_fp64():
    A = _coupled(10)
    h = ba.setup(A, sa.Params(coarse_enough=4 * 60))
    f = np.random.default_rng(12).standard_normal(4 * A.nb)
    z, z32 = ba.vcycle(h, f), ba.vcycle_fp32(h, f)
    e = np.linalg.norm(z - z32) / np.linalg.norm(z)
    assert 1e-9 < e < 1e-5


# ------------------------------------------------------------------ planted mistakes


def _one_edit(fn, old, new):
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, (fn.__name__, old)
    ns = dict(ba.__dict__)
    exec(compile(src.replace(old, new), "<mutant of %s>" % fn.__name__, "exec"), ns)
    return ns[fn.__name__]


def _pins_fail():
    checks = [
        test_block_inverse_matches_dense_inverse,
        test_block_product_spgemm_and_transpose_match_dense,
        lambda: test_block_size_one_is_the_scalar_method(0),
        lambda: test_decoupled_fields_are_four_scalar_amgs(1, 1),
        lambda: test_decoupled_fields_are_four_scalar_amgs(2, 3),
        test_block_spai0_is_the_least_squares_minimiser,
        test_galerkin_is_dense_ptap_and_spd,
        test_prolongator_is_one_damped_block_jacobi_step_on_the_tentative_basis,
        test_two_grid_closed_form_without_sweeps,
        lambda: test_vcycle_operator_symmetric_spd_linear("spai0", 1),
        lambda: test_vcycle_operator_symmetric_spd_linear("spai0", 2),
        test_field_permutation_permutes_the_vcycle,
        lambda: test_whole_block_solve_vs_dense("cg-spai0"),
    ]
    for chk in checks:
        try:
            chk()
        except (AssertionError, ValueError, np.linalg.LinAlgError, sa.Breakdown):
            return True
    return False


BLOCK_MUTATIONS = {
    "spai0_without_transpose": ("spai0_blocks", lambda: _one_edit(
        ba.spai0_blocks, "block_product(np.transpose(D, (0, 2, 1)), block_inverse(acc))",
        "block_product(D, block_inverse(acc))")),
    "spai0_gram_transposed": ("spai0_blocks", lambda: _one_edit(
        ba.spai0_blocks, "G = block_product(A.data, np.transpose(A.data, (0, 2, 1)))",
        "G = block_product(np.transpose(A.data, (0, 2, 1)), A.data)")),
    "tentative_ones_block": ("tentative_prolongator", lambda: _one_edit(
        ba.tentative_prolongator, "np.broadcast_to(np.eye(b), (int(live.sum()), b, b))",
        "np.broadcast_to(np.ones((b, b)) / b, (int(live.sum()), b, b))")),
    "prolongator_without_inverse": ("smoothed_prolongator", lambda: _one_edit(
        ba.smoothed_prolongator, "X = block_product(Dinv[rows], Y.data)", "X = Y.data / np.max(np.abs(D_F))")),
    "prolongator_inverse_on_the_right": ("smoothed_prolongator", lambda: _one_edit(
        ba.smoothed_prolongator, "X = block_product(Dinv[rows], Y.data)", "X = block_product(Y.data, Dinv[rows])")),
    "transpose_keeps_blocks": ("transpose", lambda: _one_edit(
        ba.transpose, "data = np.transpose(P.data[order], (0, 2, 1)).copy()", "data = P.data[order].copy()")),
    "spgemm_swapped_factors": ("spgemm", lambda: _one_edit(
        ba.spgemm, "prods = block_product(X.data[xk], Y.data[yk])", "prods = block_product(Y.data[yk], X.data[xk])")),
    "inverse_without_pivoting": ("block_inverse", lambda: _one_edit(
        ba.block_inverse, "p = c + np.argmax(np.abs(W[:, c:, c]), axis=1)", "p = np.full(m, c)")),
    "post_sweep_without_transpose": ("vcycle", lambda: _one_edit(
        ba.vcycle, "z = z + lv.Mts @ (f - lv.As @ z)", "z = z + lv.Ms @ (f - lv.As @ z)")),
    "damping_from_blocks_not_inverted": ("prolongator_damping", lambda: _one_edit(
        ba.prolongator_damping, "scaled = block_product(Dinv[rows], A_F.data)",
        "scaled = A_F.data / np.abs(D_F).max()")),
    "strength_without_diagonal_norms": ("strength_graph", lambda: _one_edit(
        ba.strength_graph, "s * s > e4 * (sd[rows] * sd[cols])", "s > e4 * (sd[rows] * sd[cols])")),
}


@pytest.mark.parametrize("name", sorted(BLOCK_MUTATIONS))
def test_planted_block_mistake_is_caught(name, monkeypatch):
    attr, make = BLOCK_MUTATIONS[name]
    monkeypatch.setattr(ba, attr, make())
    with np.errstate(all="ignore"):
        assert _pins_fail(), name


def test_block_pins_pass_unmutated():
    assert not _pins_fail()
