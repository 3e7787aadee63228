"""amg_vcycle_noalloc against amg_vcycle (GPU).

The allocation-free V-cycle keeps its work vectors in the library's fixed
device array; its result must be bitwise the one amg_vcycle computes with
the handle's own vectors, on consecutive calls whose second input is
smaller than the first (the array keeps the first call's contents), and
amg_vcycle must be unaffected afterwards.  A hierarchy whose work vectors
do not fit is refused.
"""

import numpy as np
import pytest

from tests.gpu_util import announce

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1811_05704_amd import amg  # noqa: E402

import problems  # noqa: E402


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


CASES = [
    ("poisson48", {}),                                  # then a smaller one
    ("poisson24", {}),
    ("poisson40", {"precision": "mixed"}),
    ("poisson20", {"precision": "mixed"}),
    ("poisson32", {"relax": "chebyshev"}),
    ("poisson16", {"npre": 2, "npost": 2}),
]


def _matrix(name):
    return problems.poisson3d(int(name[len("poisson"):]))


def test_noalloc_vcycle_equals_vcycle_on_consecutive_calls():
    for name, kw in CASES:
        A = _matrix(name)
        S = amg.Solver(A, **kw)
        r = np.random.default_rng(31).standard_normal(A.n)
        announce("noalloc vcycle", name, kw)
        ref = host(S.vcycle(dev(r)))
        for _ in range(2):
            z = S.vcycle_noalloc(dev(r))
            torch.cuda.synchronize()
            assert np.array_equal(host(z), ref), (name, kw)
        # the handle's own vectors are back in place
        assert np.array_equal(host(S.vcycle(dev(r))), ref)
        S.release()


def test_noalloc_refuses_work_vectors_beyond_the_array():
    A = problems.poisson3d(150)  # level-1 work vectors alone: 3 x 27 MB in FP64
    S = amg.Solver(A)
    announce("noalloc too large")
    r = dev(np.ones(A.n))
    with pytest.raises(amg.AmgError) as e:
        S.vcycle_noalloc(r)
    assert e.value.code == -8
    S.release()
