"""Block-value (4 x 4) solve phase on the device against the block oracle (GPU).

* One V-cycle on the same vector: within 1e-12 of the block oracle in FP64
  (2-norm and element by element); the FP32 V-cycle within the FP32 rounding
  bound of the oracle's FP32 V-cycle.  Cases cover 2 and 3 levels, both
  block smoothers, a nonsymmetric system, four decoupled fields and block
  rows long enough for the 4-lanes-per-component kernel.
* Whole solves: iterations within +-1 of the oracle, true relative residual
  <= 1e-8 recomputed on the CPU, solution within 1e-6 of the oracle's.
* A single-level block hierarchy is an exact solve; a zero right-hand side
  gives zero; graph replays are bitwise equal.
"""

import numpy as np
import pytest

from tests.gpu_util import announce, rel_err

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1811_05704_amd import amg  # noqa: E402

import oracle.block_amg as ba  # noqa: E402
import oracle.sa_amg as sa  # noqa: E402
import problems  # noqa: E402
from tests.test_gpu_parity import max_rel  # noqa: E402


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _oracle_bsr(B):
    return ba.Bsr(B.row_ptr.astype(np.int64), B.col.astype(np.int64), B.blocks().copy(), B.nb)


def _case(name):
    if name == "coupled12":
        return problems.coupled_diffusion3d(12, problems.gaussian_field(12, 1.0, 8.0, 2)), {}
    if name == "coupled16-3lev":
        return problems.coupled_diffusion3d(16, problems.gaussian_field(16, 1.0, 8.0, 2)), {"coarse_enough": 400}
    if name == "coupled20-jacobi":
        return (problems.coupled_diffusion3d(20, problems.gaussian_field(20, 2.0, 8.0, 1)),
                {"relax": "jacobi", "coarse_enough": 800})
    if name == "convection16":
        g = problems.gaussian_field(16, 1.0, 8.0, 2)
        return (problems.coupled_diffusion3d(16, g, velocity=(50.0, 25.0, 12.5)),
                {"relax": "jacobi", "solver": "bicgstab", "coarse_enough": 400})
    if name == "convection16-gmres":
        g = problems.gaussian_field(16, 1.0, 8.0, 2)
        return (problems.coupled_diffusion3d(16, g, velocity=(50.0, 25.0, 12.5)),
                {"relax": "jacobi", "solver": "gmres", "coarse_enough": 400})
    if name.startswith("coupled16-sweeps"):
        # sweep counts other than one pre- and one post-sweep (the unfused form)
        npre, npost = int(name[-2]), int(name[-1])
        return (problems.coupled_diffusion3d(16, problems.gaussian_field(16, 1.0, 8.0, 2)),
                {"coarse_enough": 400, "npre": npre, "npost": npost, "solver": "bicgstab"})
    if name == "convection16-sweeps21":
        g = problems.gaussian_field(16, 1.0, 8.0, 2)
        return (problems.coupled_diffusion3d(16, g, velocity=(50.0, 25.0, 12.5)),
                {"relax": "jacobi", "solver": "gmres", "coarse_enough": 400, "npre": 2, "npost": 1})
    if name == "decoupled16":
        return problems.decoupled_diffusion3d(16, problems.gaussian_field(16, 1.0, 8.0, 3)), {"coarse_enough": 400}
    if name == "coupled32":
        return problems.coupled_diffusion3d(32, problems.gaussian_field(32, 1.0, 8.0, 4)), {}
    raise KeyError(name)


def _oracle_params(kw):
    return sa.Params(**{k: v for k, v in kw.items() if k in ("relax", "solver", "coarse_enough", "npre", "npost")})


SWEEP_CASES = ["coupled16-sweeps22", "coupled16-sweeps03", "coupled16-sweeps10", "coupled16-sweeps32",
               "convection16-sweeps21"]
VCYCLE_CASES = ["coupled12", "coupled16-3lev", "coupled20-jacobi", "convection16", "decoupled16",
                "coupled32"] + SWEEP_CASES


@pytest.mark.parametrize("name", VCYCLE_CASES)
def test_block_vcycle_fp64_matches_oracle(name):
    B, kw = _case(name)
    announce("block vcycle fp64", name)
    S = amg.Solver(B, **kw)
    h = ba.setup(_oracle_bsr(B), _oracle_params(kw))
    assert S.nlevels == h.nlevels
    r = np.random.default_rng(41).standard_normal(B.n)
    z = host(S.vcycle(dev(r)))
    zo = ba.vcycle(h, r)
    e, m = rel_err(z, zo), max_rel(z, zo)
    print(f"[block vcycle fp64] {name}: levels {S.nlevels}, rel {e:.2e}, max {m:.2e}", flush=True)
    assert e <= 1e-12 and m <= 1e-12
    S.release()


@pytest.mark.parametrize("name", VCYCLE_CASES)
def test_block_vcycle_mixed_matches_fp32_oracle(name):
    B, kw = _case(name)
    announce("block vcycle mixed", name)
    S = amg.Solver(B, precision="mixed", **kw)
    h = ba.setup(_oracle_bsr(B), _oracle_params(kw))
    r = np.random.default_rng(42).standard_normal(B.n)
    z = host(S.vcycle(dev(r)))
    z32, z64 = ba.vcycle_fp32(h, r), ba.vcycle(h, r)
    # FP32 rounding bound: per level one product per sweep, the restriction
    # and the prolongation, each rounding to a few u; a 4 x 4 smoother block
    # adds a 4-term product per row to each sweep (counted as one more
    # product): 2 (npre + npost) + 2 products, 6 with one sweep each
    u = 2.0 ** -24
    tol = 2.0 * (2 * (kw.get("npre", 1) + kw.get("npost", 1)) + 2) * S.nlevels * u
    e32, m32, e64 = rel_err(z, z32), max_rel(z, z32), rel_err(z, z64)
    print(f"[block vcycle mixed] {name}: vs FP32 oracle rel {e32:.2e} max {m32:.2e}; vs FP64 oracle {e64:.2e}; "
          f"bound {tol:.2e}", flush=True)
    assert e32 <= tol and m32 <= 2 * tol and e64 <= tol
    S.release()


SOLVE_CASES = [("coupled12", "fp64"), ("coupled16-3lev", "fp64"), ("coupled16-3lev", "mixed"),
               ("coupled20-jacobi", "fp64"), ("convection16", "fp64"), ("convection16", "mixed"),
               ("coupled32", "fp64"), ("coupled32", "mixed"),
               ("convection16-gmres", "fp64"), ("convection16-gmres", "mixed"),
               ("coupled16-sweeps22", "fp64"), ("coupled16-sweeps03", "mixed"), ("coupled16-sweeps32", "mixed"),
               ("convection16-sweeps21", "fp64"), ("convection16-sweeps21", "mixed")]


@pytest.mark.parametrize("name,precision", SOLVE_CASES)
def test_block_solve_matches_oracle(name, precision):
    B, kw = _case(name)
    f = problems.random_block_rhs(B.nb, 4, 43)
    announce("block solve", name, precision)
    S = amg.Solver(B, precision=precision, **kw)
    x, info = S.solve(dev(f))
    x = host(x)
    xo, io, _ = ba.solve(_oracle_bsr(B), f, _oracle_params(kw), mixed=(precision == "mixed"))
    res = np.linalg.norm(f - B.to_scipy() @ x) / np.linalg.norm(f)
    print(f"[block solve] {name} {precision}: iters {info['iters']} (oracle {io.iters}), true res {res:.2e}, "
          f"vs oracle {rel_err(x, xo):.2e}", flush=True)
    assert info["status"] == 0
    assert abs(info["iters"] - io.iters) <= 1
    assert res <= 1e-8
    assert rel_err(x, xo) <= 1e-6
    # the captured iteration graph replays to the same result
    x2, info2 = S.solve(dev(f))
    assert info2["iters"] == info["iters"] and np.array_equal(host(x2), x)
    S.release()


def test_block_single_level_is_exact_and_zero_rhs_is_zero():
    B = problems.coupled_diffusion3d(6)
    S = amg.Solver(B, coarse_enough=4 * B.nb)
    assert S.nlevels == 1
    f = problems.random_block_rhs(B.nb, 4, 44)
    announce("block single level")
    z = host(S.vcycle(dev(f)))
    zr = np.linalg.solve(B.to_scipy().toarray(), f)
    assert rel_err(z, zr) <= 1e-10
    x, info = S.solve(dev(f))
    assert info["iters"] == 1 and info["true_rel_resid"] <= 1e-8
    x0, info0 = S.solve(dev(np.zeros(B.n)))
    assert info0["iters"] == 0 and not np.any(host(x0))
    S.release()


def test_block_vcycle_timing_reports_bytes():
    B, kw = _case("coupled32")
    S = amg.Solver(B, **kw)
    announce("block vcycle timing")
    us, by = S.time_kernel("vcycle", reps=5)
    assert us > 0 and by > 0
    with pytest.raises(amg.AmgError):
        S.time_kernel("restrict", reps=2)
    S.release()
    # the byte count covers one pre- and one post-sweep only
    B, kw = _case("coupled16-sweeps22")
    S = amg.Solver(B, **kw)
    with pytest.raises(amg.AmgError):
        S.time_kernel("vcycle", reps=2)
    S.release()


@pytest.mark.timeout(600)
def test_full_size_block96_properties():
    """The 96^3-node benchmark system (3,538,944 unknowns) in the benchmark's
    configuration, checked by properties that hold at any size: FP64 and
    mixed solves reach a true residual <= 1e-8 (recomputed on the CPU) with
    iteration counts within 1 of each other and solutions within 1e-6; the
    FP64 V-cycle is linear and, the post-sweep applying M^T, symmetric to
    rounding (<V a, b> = <a, V b> relative to |V a| |b|)."""
    A = problems.coupled_diffusion3d(96, problems.gaussian_field(96, 1.0, 8.0, 2))
    f = problems.rhs_uniform(A.n, 0)
    M = A.to_scipy()
    xs, its = {}, {}
    for precision in ("fp64", "mixed"):
        S = amg.Solver(A, precision=precision)
        announce("block96 solve", precision)
        x, info = S.solve(dev(f))
        x = host(x)
        tr = np.linalg.norm(f - M @ x) / np.linalg.norm(f)
        print(f"[block96] {precision}: iters {info['iters']} true {tr:.2e}", flush=True)
        assert info["status"] == 0 and tr <= 1e-8
        xs[precision], its[precision] = x, info["iters"]
        if precision == "fp64":
            rng = np.random.default_rng(21)
            a, b = rng.standard_normal(A.n), rng.standard_normal(A.n)
            announce("block96 V-cycle properties")
            Va, Vb = host(S.vcycle(dev(a))), host(S.vcycle(dev(b)))
            Vab = host(S.vcycle(dev(2.0 * a - 3.0 * b)))
            lin = np.linalg.norm(Vab - (2.0 * Va - 3.0 * Vb)) / np.linalg.norm(Vab)
            sym = abs(Va @ b - a @ Vb) / (np.linalg.norm(Va) * np.linalg.norm(b))
            print(f"[block96] linearity {lin:.2e} symmetry {sym:.2e}", flush=True)
            assert lin <= 1e-12 and sym <= 1e-12
        S.release()
    assert abs(its["fp64"] - its["mixed"]) <= 1
    assert rel_err(xs["mixed"], xs["fp64"]) <= 1e-6
