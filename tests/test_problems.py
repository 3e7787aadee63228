"""Pins for the seeded input generators (CPU)."""

import numpy as np
import pytest

import problems


def test_poisson_sizes_match_paper_150():
    # Section 4.1 quotes 3,375,000 unknowns and 23,490,000 nonzeros at 150^3.
    A = problems.poisson3d(150)
    assert A.n == 3_375_000
    assert A.nnz == 23_490_000
    assert problems.poisson3d_nnz(150) == 23_490_000


@pytest.mark.parametrize("N", [1, 2, 3, 7, 16, 32])
def test_poisson_nnz_closed_form(N):
    A = problems.poisson3d(N)
    assert A.nnz == 7 * N**3 - 6 * N**2
    assert A.row_ptr.dtype == np.int64 and A.col.dtype == np.int32


def test_other_sizes_closed_form():
    assert problems.poisson3d_nnz(32) == 223_232
    assert problems.poisson3d_nnz(128) == 14_581_760
    assert problems.poisson3d_nnz(200) == 55_760_000


def test_poisson_structure():
    N = 5
    A = problems.poisson3d(N)
    S = A.to_scipy()
    D = S.toarray()
    assert np.array_equal(D, D.T)
    assert np.all(np.diag(D) == 6.0)
    # columns strictly ascending per row and diagonal present
    for i in range(A.n):
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
        assert i in c
    # 7-point coupling: only unit-distance lexicographic neighbours
    i, j = np.nonzero(D)
    off = np.abs(i - j)
    assert set(off.tolist()) <= {0, 1, N, N * N}


def test_diffusion_unit_coefficient_is_poisson():
    N = 9
    P = problems.poisson3d(N)
    Dz = problems.diffusion3d(N, np.zeros(N**3))
    assert np.array_equal(P.row_ptr, Dz.row_ptr)
    assert np.array_equal(P.col, Dz.col)
    assert np.array_equal(P.val, Dz.val)


def test_diffusion_symmetric_and_m_matrix():
    N = 8
    g = problems.gaussian_field(N, sigma=2.0, ell=8.0, seed=1)
    A = problems.diffusion3d(N, g).to_scipy().toarray()
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0)
    # weak diagonal dominance with strict dominance on boundary rows
    assert np.all(np.diag(A) + off.sum(axis=1) >= -1e-12)
    np.linalg.cholesky(A)


def test_convection_m_matrix_zero_interior_rowsums():
    N = 7
    Pe = 50.0
    v = (1.0 * Pe, 0.5 * Pe, 0.25 * Pe)
    A = problems.diffusion3d(N, None, velocity=v).to_scipy().toarray()
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0)
    assert not np.allclose(A, A.T)
    idx = np.arange(N**3)
    i, j, k = idx % N, (idx // N) % N, idx // (N * N)
    interior = (i > 0) & (i < N - 1) & (j > 0) & (j < N - 1) & (k > 0) & (k < N - 1)
    rs = A.sum(axis=1)
    assert np.allclose(rs[interior], 0.0, atol=1e-12)
    assert np.all(rs[~interior] > 0)
    # upwind coefficient -v_x h on the -x neighbour of an interior node
    h = 1.0 / (N + 1)
    c = int(np.nonzero(interior)[0][0])
    assert A[c, c - 1] == pytest.approx(-1.0 - v[0] * h, rel=1e-14)
    assert A[c, c + 1] == pytest.approx(-1.0, rel=1e-14)


def test_gaussian_field_statistics_and_seed():
    N = 48
    g1 = problems.gaussian_field(N, sigma=1.0, ell=8.0, seed=3)
    g2 = problems.gaussian_field(N, sigma=1.0, ell=8.0, seed=3)
    g3 = problems.gaussian_field(N, sigma=1.0, ell=8.0, seed=4)
    assert np.array_equal(g1, g2)
    assert not np.array_equal(g1, g3)
    # variance is sigma^2 by construction (unit-norm kernel); sample estimate
    # over a correlated field is loose
    assert 0.3 < g1.var() < 2.0
    # correlation at lag ell along x is exp(-1/2) for the squared exponential
    G = g1.reshape(N, N, N)
    lag = 8
    a, b = G[:, :, :-lag].ravel(), G[:, :, lag:].ravel()
    rho = np.corrcoef(a, b)[0, 1]
    assert abs(rho - np.exp(-0.5)) < 0.15


def test_rhs_generators():
    assert np.array_equal(problems.rhs_ones(5), np.ones(5))
    u = problems.rhs_uniform(1000, seed=0)
    assert np.array_equal(u, np.random.default_rng(0).random(1000))
    assert u.min() >= 0.0 and u.max() < 1.0


def _check_csr_spd(A, dense=True):
    """Sorted unique columns, diagonal stored and positive, exact symmetry,
    weak diagonal dominance (with the matrices here: SPD)."""
    assert A.row_ptr.dtype == np.int64 and A.col.dtype == np.int32
    assert A.row_ptr[0] == 0 and np.all(np.diff(A.row_ptr) >= 1)
    for i in range(A.n):
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
        assert i in c
    S = A.to_scipy()
    assert (S != S.T).nnz == 0
    d = S.diagonal()
    assert np.all(d > 0)
    off = np.asarray(abs(S).sum(axis=1)).ravel() - d
    assert np.all(off <= d + 1e-12)
    if dense:
        assert np.linalg.eigvalsh(S.toarray()).min() > 0


def test_poisson27_stencil():
    N = 5
    A = problems.poisson3d_27(N)
    _check_csr_spd(A)
    rl = np.diff(A.row_ptr)
    # interior rows hold the full 3x3x3 box, corners 2x2x2
    assert rl.max() == 27 and rl.min() == 8
    assert A.nnz == (3 * N - 2) ** 3  # sum over axes of (3N - 2) per direction
    D = A.to_scipy().toarray()
    assert np.all(np.diag(D) == 26.0)
    assert set(np.unique(D[D != 0]).tolist()) == {-1.0, 26.0}


def test_anisotropic_couplings():
    N, eps = 6, 1e-3
    A = problems.anisotropic3d(N, eps)
    _check_csr_spd(A)
    D = A.to_scipy().toarray()
    i, j = np.nonzero(D - np.diag(np.diag(D)))
    gap = np.abs(i - j)
    assert set(gap.tolist()) == {1, N, N * N}
    assert np.all(D[i[gap == N * N], j[gap == N * N]] == -eps)
    assert np.all(D[i[gap < N * N], j[gap < N * N]] == -1.0)
    assert np.all(np.diag(D) == 4.0 + 2.0 * eps)


def test_decoupled_boundary_rows_are_identity():
    N = 4
    A = problems.decoupled_boundary(N)
    _check_csr_spd(A)
    M = N + 2
    assert A.n == M**3
    rl = np.diff(A.row_ptr)
    # (N+2)^3 - N^3 boundary rows hold only their unit diagonal
    assert int(np.sum(rl == 1)) == M**3 - N**3
    D = A.to_scipy().toarray()
    idx = np.arange(A.n)
    ii, jj, kk = idx % M, (idx // M) % M, idx // (M * M)
    interior = (ii > 0) & (ii < M - 1) & (jj > 0) & (jj < M - 1) & (kk > 0) & (kk < M - 1)
    assert np.all(np.diag(D)[~interior] == 1.0)
    # the interior block is the 7-point Poisson matrix of N^3
    P = problems.poisson3d(N).to_scipy().toarray()
    assert np.array_equal(D[np.ix_(interior, interior)], P)


def test_random_laplacian_structure():
    A = problems.random_laplacian(3000, hub_degree=1200, seed=5)
    _check_csr_spd(A, dense=False)
    S = A.to_scipy()
    rl = np.diff(A.row_ptr)
    assert rl.max() > 1024  # some rows longer than an FP64 stream block
    # row sums equal the shift exactly up to rounding (Laplacian + shift I)
    assert np.allclose(np.asarray(S.sum(axis=1)).ravel(), 0.05, atol=1e-9)
    B = problems.random_laplacian(3000, hub_degree=1200, seed=5)
    assert np.array_equal(A.val, B.val) and np.array_equal(A.col, B.col)



@pytest.mark.parametrize("N", [2, 4, 7])
def test_stokes_structure(N):
    from problems.stokes import stokes3d, stokes_rhs

    A, n_u = stokes3d(N)
    n = N**3
    assert A.n == 4 * n and n_u == 3 * n
    # K: three 7-point blocks; G and D: 2 N^2 (N-1) entries per axis; S: 7-point
    assert A.nnz == 40 * N**3 - 36 * N**2
    M = A.to_scipy()
    K, G, D, S = M[:n_u, :n_u], M[:n_u, n_u:], M[n_u:, :n_u], M[n_u:, n_u:]
    assert abs(K - K.T).max() == 0 and abs(D + G.T).max() == 0
    assert np.all(M.diagonal() > 0)
    h = 1.0 / (N + 1)
    assert set(np.unique(np.abs(G.data))) == {0.5 * h}
    assert np.allclose(S.diagonal(), 6 * h * h / 12)
    f = stokes_rhs(N)
    assert f.shape == (4 * n,) and f[:n_u].min() == 1.0 and not f[n_u:].any()


def test_oseen_p1_structure():
    """P1 tetrahedra on the Kuhn mesh: every interior node couples to its 14
    mesh neighbours; away from the boundary the rows of K sum to the lumped
    nodal volume over dt (h^3 / dt: stiffness, convection and streamline
    terms sum to zero), those of G_d and S to zero."""
    from problems.stokes import oseen_p1, oseen_rhs

    N = 6
    A, n_u = oseen_p1(N)
    n = N**3
    h = 1.0 / (N + 1)
    dt = 2.0 * h
    M = A.to_scipy()
    K, G, D, S = M[:n, :n], M[:n_u, n_u:], M[n_u:, :n_u], M[n_u:, n_u:]
    assert abs(D + G.T).max() == 0
    assert abs(K - K.T).max() > 0  # convection: nonsymmetric
    assert M[:n, n:n_u].nnz == 0  # velocity components uncoupled
    idx = np.arange(n)
    c = np.stack([idx % N, (idx // N) % N, idx // (N * N)], axis=1)
    deep = np.all((c >= 1) & (c <= N - 2), axis=1)
    rl = np.diff(K.indptr)
    assert np.all(rl[deep] == 15)
    assert np.allclose(np.asarray(K.sum(axis=1)).ravel()[deep], h**3 / dt, rtol=1e-12)
    for d in range(3):
        Gd = G[d * n:(d + 1) * n]
        assert np.allclose(np.asarray(Gd.sum(axis=1)).ravel()[deep], 0.0, atol=1e-14 * h * h)
        assert Gd.diagonal().max() == 0  # no self coupling in the gradient
    assert np.allclose(np.asarray(S.sum(axis=1)).ravel()[deep], 0.0, atol=1e-12 * S.diagonal().max())
    assert np.all(M.diagonal()[n_u:] > 0)
    f = oseen_rhs(N)
    assert f.shape == (4 * n,) and not f[n_u:].any()
