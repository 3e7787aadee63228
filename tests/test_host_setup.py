"""Library host setup vs the oracle, and the C ABI contract (CPU only).

The library builds its hierarchy on the host (section 3: setup on the CPU,
then transfer to the device).  These tests call it through the C ABI's
host-only entry point and compare every level with the oracle; no device
compute is involved.
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import problems

amg = pytest.importorskip("paper_1811_05704_amd.amg")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return amg.lib()


def test_library_exports_every_declared_symbol(lib):
    header = open(os.path.join(ROOT, "include", "amg.h")).read()
    declared = set(re.findall(r"\b(amg_[a-z_0-9]+)\s*\(", header))
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(amg.exported_symbols())


def test_params_default_values():
    p = amg.make_params()
    assert (p.solver, p.relax, p.precision, p.npre, p.npost) == (0, 0, 0, 1, 1)
    assert (p.coarse_enough, p.max_levels, p.max_iter) == (3000, 30, 500)
    assert p.eps_strong == 0.08 and p.jacobi_omega == 0.72 and p.tol == 1e-8
    assert (p.cheb_degree, p.cheb_ratio) == (3, 30.0)


def _cases():
    g = problems.gaussian_field(24, 2.0, 8.0, 1)
    return [
        ("poisson32", problems.poisson3d(32), "spai0"),
        ("poisson40", problems.poisson3d(40), "spai0"),
        ("diffusion24", problems.diffusion3d(24, g), "spai0"),
        ("diffusion24-jacobi", problems.diffusion3d(24, g), "jacobi"),
        ("convection24", problems.diffusion3d(24, g, velocity=(50.0, 25.0, 12.5)), "jacobi"),
        ("diffusion24-chebyshev", problems.diffusion3d(24, g), "chebyshev"),
        # other structures: 27-point rows, weak (dropped) couplings, isolated
        # nodes, irregular rows with hubs longer than a stream block
        ("poisson27-16", problems.poisson3d_27(16), "spai0", {"eps_strong": 0.02}),
        ("anisotropic20", problems.anisotropic3d(20, 1e-3), "spai0"),
        ("decoupled14", problems.decoupled_boundary(14), "jacobi"),
        ("graph60k", problems.random_laplacian(60000, seed=2), "spai0"),
    ]


@pytest.mark.parametrize("case", _cases(), ids=[c[0] for c in _cases()])
def test_hierarchy_matches_oracle(case):
    name, A, relax = case[:3]
    kw = case[3] if len(case) > 3 else {}
    H = amg.HostHierarchy(A, relax=relax, **kw)
    h = oracle.setup(A, oracle.Params(relax=relax, **kw))
    assert H.nlevels == h.nlevels
    for l in range(H.nlevels):
        Al = H.level_scipy(l, "A")
        Ao = h.levels[l].A
        assert Al.shape == Ao.shape
        # values agree bit for bit (the oracle may drop exact zeros that the
        # library keeps as structural entries)
        assert abs(Al - Ao).max() == 0.0
        if l == H.nlevels - 1:
            continue
        assert np.array_equal(H.aggregates(l), h.levels[l].agg)
        P = H.level_scipy(l, "P")
        R = H.level_scipy(l, "R")
        assert abs(P - h.levels[l].P).max() == 0.0
        assert abs(R - P.T).max() == 0.0
        m, omega, hi = H.smoother(l)
        assert np.array_equal(m, h.levels[l].m)
        assert omega == h.levels[l].omega
        assert hi == (h.levels[l].cheb_hi or 0.0)
        # columns ascending in every row of the library's matrices
        for M in (Al, P, R):
            d = np.diff(M.indices)
            cross = M.indptr[1:-1] - 1  # positions in d that span two rows
            cross = cross[(cross >= 0) & (cross < d.size)]
            mask = np.ones(d.size, dtype=bool)
            mask[cross] = False
            assert np.all(d[mask] > 0)


def test_single_level_and_level_info():
    A = problems.poisson3d(10)
    H = amg.HostHierarchy(A)
    assert H.nlevels == 1
    n, na, npp = H.level_info(0)
    assert (n, na, npp) == (1000, A.nnz, 0)
    with pytest.raises(amg.AmgError):
        H.aggregates(0)


def test_worked_example_through_library(golden_dir):
    from tests.test_oracle import load_golden

    pw = load_golden(os.path.join(golden_dir, "pw_1d_laplacian.txt"))
    H = amg.HostHierarchy(problems.tridiag1d(9), coarse_enough=3)
    assert H.nlevels == 2
    assert H.aggregates(0).tolist() == [int(a) for a in pw["agg"]]
    P = H.level_scipy(0, "P").toarray()
    assert np.max(np.abs(P - np.array([float(v) for v in pw["P"]]).reshape(9, 3))) <= 1e-15
    Ac = H.level_scipy(1, "A").toarray()
    assert np.max(np.abs(Ac - np.array([float(v) for v in pw["Ac"]]).reshape(3, 3))) <= 1e-15


# ------------------------------------------------------------------ error paths


def _setup_host(n, rp, col, val, **kw):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    p = amg.make_params(**kw)
    h = C.c_void_p()
    code = amg.lib().amg_setup_host(n, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                    col.ctypes.data_as(C.POINTER(C.c_int32)),
                                    val.ctypes.data_as(C.POINTER(C.c_double)), C.byref(p), C.byref(h))
    if h.value:
        amg.lib().amg_release(h)
    return code, h.value


def _tri(n):
    A = problems.tridiag1d(n)
    return A.row_ptr.copy(), A.col.copy(), A.val.copy()


def test_error_bad_csr():
    rp, col, val = _tri(5)
    c = col.copy()
    c[1], c[0] = c[0], c[1]  # unsorted row 0
    assert _setup_host(5, rp, c, val) == (-2, None)
    c = col.copy()
    c[-1] = 7  # out of range
    assert _setup_host(5, rp, c, val) == (-2, None)
    r = rp.copy()
    r[0] = 1
    assert _setup_host(5, r, col, val)[0] == -2
    r = rp.copy()
    r[2], r[3] = r[3], r[2]  # decreasing
    assert _setup_host(5, r, col, val)[0] == -2


def test_error_zero_or_missing_diagonal():
    rp, col, val = _tri(5)
    v = val.copy()
    v[0] = 0.0
    assert _setup_host(5, rp, col, v)[0] == -3
    v = val.copy()
    v[0] = -2.0
    assert _setup_host(5, rp, col, v)[0] == -3
    # drop the diagonal of row 2
    keep = np.ones(col.size, dtype=bool)
    d2 = rp[2] + 1
    keep[d2] = False
    rp2 = rp.copy()
    rp2[3:] -= 1
    assert _setup_host(5, rp2, col[keep], val[keep])[0] == -3
    assert "diagonal" in amg.lib().amg_last_error().decode()


def test_error_non_finite_value():
    rp, col, val = _tri(5)
    v = val.copy()
    v[1] = np.nan
    assert _setup_host(5, rp, col, v)[0] == -9


def test_error_bad_params():
    rp, col, val = _tri(5)
    assert _setup_host(5, rp, col, val, solver=7)[0] == -1
    assert _setup_host(5, rp, col, val, npre=-1)[0] == -1
    assert _setup_host(5, rp, col, val, max_iter=0)[0] == -1
    assert _setup_host(0, rp, col, val)[0] == -1


def test_error_too_large():
    rp, col, val = _tri(5)
    assert _setup_host(1 << 31, rp, col, val)[0] == -8
    # coarsest level above the dense limit: no coarsening allowed
    A = problems.poisson3d(28)  # 21,952 rows
    assert _setup_host(A.n, A.row_ptr, A.col, A.val, max_levels=1)[0] == -8


def test_null_safety_and_host_handle_rejects_solve():
    L = amg.lib()
    L.amg_release(None)
    assert L.amg_num_levels(None) == 0
    assert L.amg_level_info(None, 0, None, None, None) == -1
    H = amg.HostHierarchy(problems.poisson3d(16))
    info = amg.Info()
    code = L.amg_solve(H._h, C.c_void_p(16), C.c_void_p(32), None, C.byref(info))
    assert code == -1
    assert L.amg_vcycle(H._h, C.c_void_p(16), C.c_void_p(32), None) == -1
    assert L.amg_setup(4, None, None, None, None, None, None, None) == -1


def test_level_schedules_by_row_length():
    """Every level matrix of the 7-point hierarchy gets the LDS-staged stream
    schedule; a band matrix whose rows are longer than 512 entries on average
    gets the 64-lanes-per-row vector schedule for A_1 and R_1 (in both value
    types), its prolongator (about two entries per row) the stream one.  The
    served path runs both schedules in its batched kernel."""
    H = amg.HostHierarchy(problems.poisson3d(32))
    for l in range(H.nlevels - 1):
        for which in "APR":
            for prec in ("fp64", "mixed"):
                k = H.level_kernel_info(l, which, prec)
                assert k["kind"] == "stream" and k["blocks"] > 0 and k["block_bytes"] > 0, (l, which, k)
    B = problems.banded_spd(6000, 600)
    Hb = amg.HostHierarchy(B, eps_strong=0.0005)
    assert Hb.nlevels == 2
    for prec in ("fp64", "mixed"):
        kA = Hb.level_kernel_info(0, "A", prec)
        kR = Hb.level_kernel_info(0, "R", prec)
        kP = Hb.level_kernel_info(0, "P", prec)
        assert kA == {"kind": "vector", "lanes": 64, "blocks": 6000 // 4, "block_bytes": 0}
        assert kR["kind"] == "vector" and kR["blocks"] == 2  # 5 rows, 4 per block
        assert kP["kind"] == "stream" and kP["lanes"] == 1
    with pytest.raises(amg.AmgError):
        Hb.level_kernel_info(1, "P")  # the coarsest level has no prolongator
