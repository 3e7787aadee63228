"""Field-split host setup of the library vs the oracle, and its C ABI error
paths (CPU only: the host-only entry point, no device compute)."""

import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import schur
import problems
from problems.grids import CSR

amg = pytest.importorskip("paper_1811_05704_amd.amg")


def _csr(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return CSR(M.shape[0], M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float64))


def _perturbed_stokes(N, seed=4):
    """Stokes with the divergence rows scaled entry by entry (D != -G^T)."""
    A, n_u = problems.stokes3d(N)
    M = A.to_scipy().tolil()
    M = sp.csr_matrix(M)
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    sel = (rows >= n_u) & (M.indices < n_u)
    M.data[sel] *= rng.uniform(0.8, 1.2, int(sel.sum()))
    return _csr(M), n_u


def _cases():
    return [
        ("stokes12",) + problems.stokes3d(12) + ({},),
        ("stokes20-coarse500",) + problems.stokes3d(20) + ({"coarse_enough": 500},),
        ("stokes10-unstabilised",) + problems.stokes3d(10, beta=0.0) + ({"coarse_enough": 200},),
        ("stokes14-perturbed-D",) + _perturbed_stokes(14) + ({"coarse_enough": 500},),
        ("stokes12-jacobi",) + problems.stokes3d(12) + ({"relax": "jacobi", "coarse_enough": 300},),
    ]


@pytest.mark.parametrize("case", _cases(), ids=[c[0] for c in _cases()])
def test_schur_hierarchy_matches_oracle(case):
    name, A, n_u, kw = case
    kw = dict(kw)
    kw.setdefault("solver", "bicgstab")
    H = amg.HostHierarchy(A, n_u=n_u, **kw)
    prm = oracle.Params(**kw)
    ss = schur.setup(A.to_scipy(), n_u, prm)
    assert H.nlevels == ss.h.nlevels
    # S_hat itself, bit for bit
    assert abs(H.level_scipy(0, "A") - ss.S_hat).max() == 0.0
    assert H.level_scipy(0, "A").nnz == ss.S_hat.nnz
    for l in range(H.nlevels):
        assert abs(H.level_scipy(l, "A") - ss.h.levels[l].A).max() == 0.0
        if l == H.nlevels - 1:
            continue
        assert np.array_equal(H.aggregates(l), ss.h.levels[l].agg)
        assert abs(H.level_scipy(l, "P") - ss.h.levels[l].P).max() == 0.0
        m, omega, _ = H.smoother(l)
        assert np.array_equal(m, ss.h.levels[l].m)
        assert omega == ss.h.levels[l].omega


def _setup_schur_host(A, n_u, **kw):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    p = amg.make_params(**kw)
    h = C.c_void_p()
    code = amg.lib().amg_setup_schur_host(int(A.n), rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                          col.ctypes.data_as(C.POINTER(C.c_int32)),
                                          val.ctypes.data_as(C.POINTER(C.c_double)), int(n_u), C.byref(p),
                                          C.byref(h))
    if h.value:
        amg.lib().amg_release(h)
    return code, h.value, amg.lib().amg_last_error().decode()


def test_schur_error_paths():
    A, n_u = problems.stokes3d(4)
    assert _setup_schur_host(A, n_u, solver="bicgstab")[0] == 0
    assert _setup_schur_host(A, n_u, solver="gmres")[0] == 0
    # CG: the split is not symmetric
    code, h, msg = _setup_schur_host(A, n_u, solver="cg")
    assert code == -1 and h is None and "symmetric" in msg
    for bad in (0, A.n, -3, A.n + 5):
        code, h, _ = _setup_schur_host(A, bad, solver="bicgstab")
        assert code == -1 and h is None
    # a zero velocity diagonal
    M = A.to_scipy().tolil()
    M[5, 5] = 0.0
    Z = _csr(M)
    code, h, msg = _setup_schur_host(Z, n_u, solver="bicgstab")
    assert code == -3 and h is None and "velocity row 5" in msg
    # a pressure Schur complement row without a positive diagonal: a pressure
    # unknown coupled to nothing
    M = A.to_scipy().tolil()
    p = n_u + 7
    M[p, :] = 0.0
    M[:, p] = 0.0
    code, h, msg = _setup_schur_host(_csr(M.tocsr()), n_u, solver="bicgstab")
    assert code == -3 and h is None and "row 7" in msg


def test_unstabilised_system_has_no_pressure_diagonal_and_is_accepted():
    A, n_u = problems.stokes3d(6, beta=0.0)
    M = A.to_scipy()
    assert M[n_u:, n_u:].nnz == 0
    code, h, _ = _setup_schur_host(A, n_u, solver="bicgstab")
    assert code == 0
    # the plain setup refuses the same matrix (missing diagonals)
    with pytest.raises(amg.AmgError):
        amg.HostHierarchy(A)


def interlaced(A, n_u):
    """The system renumbered node by node (u_x, u_y, u_z, p of node k at
    4k .. 4k+3) and its pressure mask; returns (CSR, pmask, new_of_old)."""
    n = A.n // 4
    old = np.arange(A.n)
    d, k = old // n, old % n
    new_of_old = 4 * k + d
    Q = sp.csr_matrix((np.ones(A.n), (new_of_old, old)), shape=(A.n, A.n))
    B = (Q @ A.to_scipy() @ Q.T).tocsr()
    pmask = np.zeros(A.n, dtype=np.uint8)
    pmask[3::4] = 1
    return _csr(B), pmask, new_of_old


def _setup_masked(A, pmask, **kw):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    m = np.ascontiguousarray(pmask, dtype=np.uint8)
    p = amg.make_params(**kw)
    h = C.c_void_p()
    code = amg.lib().amg_setup_schur_masked(int(A.n), rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                            col.ctypes.data_as(C.POINTER(C.c_int32)),
                                            val.ctypes.data_as(C.POINTER(C.c_double)),
                                            m.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(p), None, None,
                                            C.byref(h))
    if h.value:
        amg.lib().amg_release(h)
    return code, h.value, amg.lib().amg_last_error().decode()


def test_masked_setup_rejects_bad_masks_before_device_work():
    A, n_u = problems.stokes3d(3)
    B, pmask, _ = interlaced(A, n_u)
    for bad in (np.zeros(A.n, np.uint8), np.ones(A.n, np.uint8), np.where(pmask == 1, 2, 0).astype(np.uint8)):
        code, h, msg = _setup_masked(B, bad, solver="bicgstab")
        assert code == -1 and h is None and "pmask" in msg


def test_interlaced_system_is_the_permuted_one():
    A, n_u = problems.stokes3d(3)
    B, pmask, new_of_old = interlaced(A, n_u)
    M, N = A.to_scipy().toarray(), B.to_scipy().toarray()
    assert np.array_equal(N[np.ix_(new_of_old, new_of_old)], M)
    assert np.array_equal(np.flatnonzero(pmask), np.sort(new_of_old[n_u:]))
