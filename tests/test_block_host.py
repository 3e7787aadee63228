"""Host block setup against the block oracle, and the block C ABI (CPU only).

The library's C++ block setup (``amg_setup_block_host``) must rebuild the
block oracle's hierarchy exactly: the same aggregates on every level and
bit-identical blocks of A_l, P_l, R_l and of the smoother, with the same
damping omega_l.  Settings the block path does not implement are refused.
"""

import numpy as np
import pytest

import oracle.block_amg as ba
import oracle.sa_amg as sa
import problems
from paper_1811_05704_amd import amg


def _oracle_bsr(B):
    return ba.Bsr(B.row_ptr.astype(np.int64), B.col.astype(np.int64), B.blocks().copy(), B.nb)


CASES = [
    ("coupled12", {}),
    ("coupled16-jacobi", {"relax": "jacobi"}),
    ("coupled12-3levels", {"coarse_enough": 200}),
    ("convection14-jacobi", {"relax": "jacobi", "solver": "bicgstab", "coarse_enough": 400}),
    ("decoupled12", {"coarse_enough": 240}),
]


def _matrix(name):
    if name.startswith("convection"):
        N = 14
        return problems.coupled_diffusion3d(N, problems.gaussian_field(N, 1.0, 8.0, 2), velocity=(50.0, 25.0, 12.5))
    if name.startswith("decoupled"):
        return problems.decoupled_diffusion3d(12, problems.gaussian_field(12, 1.0, 8.0, 3))
    N = int(name[len("coupled"):].split("-")[0])
    return problems.coupled_diffusion3d(N, problems.gaussian_field(N, 1.0, 8.0, 2))


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_host_block_hierarchy_bit_identical_to_oracle(name, kw):
    B = _matrix(name)
    H = amg.HostHierarchy(B, **kw)
    okw = {k: v for k, v in kw.items() if k in ("relax", "solver", "coarse_enough")}
    ho = ba.setup(_oracle_bsr(B), sa.Params(**okw))
    assert H.nlevels == ho.nlevels >= 2
    for l in range(H.nlevels - 1):
        lo = ho.levels[l]
        assert np.array_equal(H.aggregates(l), lo.agg)
        M, om = H.smoother_blocks(l)
        assert om == lo.omega
        assert np.array_equal(M, lo.M)
        for w, ob in (("A", lo.A), ("P", lo.P), ("R", lo.R)):
            _, _, rp, col, v = H.level_bsr(l, w)
            assert np.array_equal(rp, ob.indptr) and np.array_equal(col, ob.indices), (l, w)
            assert np.array_equal(v, ob.data), (l, w)
    _, _, rp, col, v = H.level_bsr(H.nlevels - 1, "A")
    assert np.array_equal(rp, ho.levels[-1].A.indptr) and np.array_equal(v, ho.levels[-1].A.data)
    H.release()


def test_block_settings_outside_the_path_are_refused():
    B = problems.coupled_diffusion3d(6)
    for kw in ({"relax": "chebyshev"}, {"npre": 17}, {"npost": -1}):
        with pytest.raises(amg.AmgError) as e:
            amg.HostHierarchy(B, **kw)
        assert e.value.code == -1, kw


def test_block_input_validation():
    B = problems.coupled_diffusion3d(4)
    bad_col = B.col.copy()
    bad_col[1], bad_col[2] = bad_col[2], bad_col[1]  # not ascending
    with pytest.raises(amg.AmgError) as e:
        amg.HostHierarchy(problems.BSR(B.nb, 4, B.row_ptr, bad_col, B.val))
    assert e.value.code == -2
    no_diag = problems.BSR(B.nb, 4, B.row_ptr, np.where(B.col == 0, 1, B.col).astype(np.int32), B.val)
    with pytest.raises(amg.AmgError):
        amg.HostHierarchy(no_diag)
    with pytest.raises(amg.AmgError) as e:
        amg.HostHierarchy(problems.BSR(B.nb, 3, B.row_ptr, B.col, B.val))
    assert e.value.code == -1
    # a scalar handle refuses the block queries and the other way round
    H = amg.HostHierarchy(B)
    with pytest.raises(amg.AmgError):
        H.level_csr(0, "A")
    S = amg.HostHierarchy(problems.poisson3d(16))
    with pytest.raises(amg.AmgError):
        S.level_bsr(0, "A")
