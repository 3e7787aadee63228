"""Fused coarse levels against the one-launch-per-step path and the oracle (GPU).

With ``fuse_coarse = 1`` the levels below level 1 whose operator
is small, and the coarse solve, run in one persistent launch separated by
grid-wide barriers.  Every block of that launch does what the per-step
kernel does for the same rows, so the V-cycle and whole solves must be
bitwise identical with and without fusion, and match the oracle as the
per-step path does.  A barrier wait that runs out of time (forced here by a
zero wait limit set from the host, so every workgroup still leaves at once)
must be reported as an error, and the next call must start clean.
"""

import numpy as np
import pytest

from tests.gpu_util import announce, rel_err

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1811_05704_amd import amg  # noqa: E402

import oracle  # noqa: E402
import problems  # noqa: E402
from tests.test_gpu_parity import max_rel, mixed_vcycle_tol  # noqa: E402


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _case(name):
    if name == "poisson32":
        return problems.poisson3d(32), {}
    if name == "poisson80":  # two levels below level 1 are fused
        return problems.poisson3d(80), {}
    if name == "diffusion40":
        return problems.diffusion3d(40, problems.gaussian_field(40, 2.0, 8.0, 1)), {}
    if name == "convection40":
        g = problems.gaussian_field(40, 2.0, 8.0, 1)
        return (problems.diffusion3d(40, g, velocity=(50.0, 25.0, 12.5)),
                {"solver": "bicgstab", "relax": "jacobi"})
    if name == "graph60k":
        return problems.random_laplacian(60000, seed=2), {}
    if name == "aniso32":
        return problems.anisotropic3d(32, 1e-3), {}
    if name == "decoupled30":
        return problems.decoupled_boundary(30), {}
    raise KeyError(name)


def _oracle_params(kw):
    keys = ("solver", "relax", "eps_strong")
    return oracle.Params(**{k: v for k, v in kw.items() if k in keys})


CASES = ["poisson32", "poisson80", "diffusion40", "convection40", "graph60k", "aniso32", "decoupled30"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", CASES)
def test_fused_tail_equals_per_step_and_oracle(name, precision):
    A, kw = _case(name)
    announce("fused tail", name, precision)
    S1 = amg.Solver(A, precision=precision, fuse_coarse=1, **kw)
    S0 = amg.Solver(A, precision=precision, fuse_coarse=0, **kw)
    first, grid = S1.tail_info()
    assert S0.tail_info() == (-1, 0)
    assert S1.nlevels >= 3 and 1 <= first <= S1.nlevels - 2 and grid > 0, (S1.nlevels, first, grid)
    if name == "poisson80":
        assert first == 1 and S1.nlevels == 4
    r = np.random.default_rng(21).standard_normal(A.n)
    z1 = host(S1.vcycle(dev(r)))
    z0 = host(S0.vcycle(dev(r)))
    assert np.array_equal(z1, z0)
    h = oracle.setup(A, _oracle_params(kw))
    if precision == "fp64":
        zo = oracle.vcycle(h, r)
        assert rel_err(z1, zo) <= 1e-12 and max_rel(z1, zo) <= 1e-12
    else:
        zo = oracle.vcycle_fp32(h, r)
        tol = mixed_vcycle_tol(S1.nlevels, kw)
        assert rel_err(z1, zo) <= tol and max_rel(z1, zo) <= 2 * tol
    print(f"[fused tail] {name} {precision}: levels {S1.nlevels}, fused from level {first}, "
          f"{grid} workgroups, vs oracle {rel_err(z1, zo):.2e}", flush=True)
    f = problems.rhs_ones(A.n)
    x1, i1 = S1.solve(dev(f))
    x1b, i1b = S1.solve(dev(f))  # replayed graphs
    x0, i0 = S0.solve(dev(f))
    assert i1["iters"] == i0["iters"] == i1b["iters"]
    assert np.array_equal(host(x1), host(x0)) and np.array_equal(host(x1), host(x1b))
    assert i1["true_rel_resid"] <= 1e-8
    S1.release()
    S0.release()


def test_fused_tail_barrier_timeout_is_reported_and_recovers():
    A, kw = _case("poisson32")
    S = amg.Solver(A, fuse_coarse=1)
    first, _ = S.tail_info()
    assert first >= 1
    r = np.random.default_rng(22).standard_normal(A.n)
    ref = host(S.vcycle(dev(r)))
    announce("fused tail: zero wait limit")
    S.set_tail_wait(0.0)
    with pytest.raises(amg.AmgError) as e:
        S.vcycle(dev(r))
    assert e.value.code == -6 and "ran out of time" in str(e.value)
    S.set_tail_wait(0.25)
    announce("fused tail: after the reported timeout")
    for _ in range(3):
        assert np.array_equal(host(S.vcycle(dev(r))), ref)
    x, info = S.solve(dev(problems.rhs_ones(A.n)))
    assert info["status"] == 0 and info["true_rel_resid"] <= 1e-8
    S.release()
