"""Device solve phase vs the oracle (GPU).

* One V-cycle on the same vector: relative error <= 1e-12 in FP64, also
  element by element; the FP32 V-cycle against the oracle's FP32 V-cycle
  (and against the FP64 one) within the FP32 rounding bound
  `mixed_vcycle_tol` (2-norm), twice that element by element.
* Whole solves: iteration counts within +-1 of the oracle and a true
  relative residual <= 1e-8, recomputed on the CPU from the returned x.
* Edge cases: zero right-hand side, single-level hierarchy, exact initial
  guess, iteration limit, singular coarsest matrix, other sweep counts,
  graph replay vs direct launches, run-to-run determinism.
"""

import os

import numpy as np
import pytest

from tests.gpu_util import announce, rel_err, true_rel_residual

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1811_05704_amd import amg  # noqa: E402

import oracle  # noqa: E402
import problems  # noqa: E402


def dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def max_rel(a, b):
    """Element-wise distance max|a - b| relative to max|b|."""
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def host(t):
    return t.detach().cpu().numpy()


def _problem(name):
    if name == "poisson32":
        return problems.poisson3d(32), {}
    if name == "poisson20":
        return problems.poisson3d(20), {}
    if name == "diffusion24":
        return problems.diffusion3d(24, problems.gaussian_field(24, 2.0, 8.0, 1)), {}
    if name == "convection24":
        g = problems.gaussian_field(24, 2.0, 8.0, 1)
        return problems.diffusion3d(24, g, velocity=(50.0, 25.0, 12.5)), {"relax": "jacobi"}
    # other structures: 27-point rows (4 lanes per row on level 1), weak
    # z-couplings dropped by the strength test, isolated identity rows, and an
    # irregular graph whose hub rows are longer than an FP64 stream block
    if name == "poisson27-16":
        return problems.poisson3d_27(16), {"eps_strong": 0.02}
    if name == "aniso20":
        return problems.anisotropic3d(20, 1e-3), {}
    if name == "decoupled14":
        return problems.decoupled_boundary(14), {}
    if name == "graph60k":
        return problems.random_laplacian(60000, seed=2), {}
    raise KeyError(name)


U32 = 2.0 ** -24  # FP32 unit roundoff


def mixed_vcycle_tol(levels, kw):
    """Rounding bound of an FP32 V-cycle against another evaluation of it.

    Each level applies p sparse products in FP32 (pre-sweeps, residual,
    restriction, prolongation, post-sweeps; a Chebyshev sweep is `degree`
    products), each of which, with its fused vector update, rounds its
    result to a relative error of a few u (u = 2^-24).  Both sides of a
    comparison (device and oracle, or FP32 and FP64) differ from the exact
    V-cycle by at most the sum over the levels, so the bound is
    2 * p * L * u for the 2-norm relative distance (and twice that for the
    largest element relative to the largest element).
    """
    sweeps = kw.get("npre", 1) + kw.get("npost", 1)
    per = kw.get("cheb_degree", 3) if kw.get("relax") == "chebyshev" else 1
    p = sweeps * per + 2
    return 2.0 * p * levels * U32


def _oracle_params(kw):
    keys = ("solver", "relax", "npre", "npost", "coarse_enough", "max_iter", "tol", "max_levels",
            "cheb_degree", "cheb_ratio", "gmres_m", "eps_strong", "jacobi_omega")
    return oracle.Params(**{k: v for k, v in kw.items() if k in keys})


# ------------------------------------------------------------------ V-cycle


VCYCLE_CASES = [
    ("poisson32", {}),
    ("diffusion24", {}),
    ("convection24", {}),
    ("poisson20", {"npre": 2, "npost": 2}),
    ("poisson20", {"npre": 0, "npost": 1}),
    ("poisson20", {"npre": 1, "npost": 0}),
    ("poisson20", {"npre": 3, "npost": 2, "relax": "jacobi"}),
    ("poisson20", {"coarse_enough": 50}),
    # Chebyshev relaxation: every sweep shape the device path distinguishes
    ("poisson32", {"relax": "chebyshev"}),
    ("diffusion24", {"relax": "chebyshev"}),
    ("convection24", {"relax": "chebyshev"}),
    ("diffusion24", {"relax": "chebyshev", "cheb_degree": 5, "cheb_ratio": 10.0}),
    ("poisson20", {"relax": "chebyshev", "cheb_degree": 1}),
    ("poisson20", {"relax": "chebyshev", "cheb_degree": 2}),
    ("poisson20", {"relax": "chebyshev", "cheb_degree": 2, "npre": 2, "npost": 2}),
    ("poisson20", {"relax": "chebyshev", "cheb_degree": 1, "npre": 2, "npost": 3}),
    ("poisson20", {"relax": "chebyshev", "cheb_degree": 3, "npre": 3, "npost": 2}),
    ("poisson20", {"relax": "chebyshev", "npre": 0, "npost": 1}),
    ("poisson20", {"relax": "chebyshev", "npre": 1, "npost": 0}),
    ("poisson20", {"relax": "chebyshev", "coarse_enough": 50}),
    ("poisson27-16", {}),
    ("aniso20", {}),
    ("decoupled14", {}),
    ("decoupled14", {"relax": "jacobi"}),
    ("graph60k", {}),
    ("graph60k", {"relax": "chebyshev"}),
]


@pytest.mark.parametrize("name,kw", VCYCLE_CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(VCYCLE_CASES)])
def test_vcycle_fp64_matches_oracle(name, kw):
    A, base = _problem(name)
    kw = {**base, **kw}
    S = amg.Solver(A, **kw)
    h = oracle.setup(A, _oracle_params(kw))
    assert S.nlevels == h.nlevels
    r = np.random.default_rng(11).standard_normal(A.n)
    announce("vcycle fp64", name, kw, "levels", S.nlevels)
    z = host(S.vcycle(dev(r)))
    zo = oracle.vcycle(h, r)
    e, m = rel_err(z, zo), max_rel(z, zo)
    print(f"[fp64 vcycle] {name} {kw}: rel {e:.2e}, max {m:.2e}", flush=True)
    assert e <= 1e-12
    assert m <= 1e-12
    S.release()


def test_vcycle_worked_example(golden_dir):
    from tests.test_oracle import load_golden

    pw = load_golden(os.path.join(golden_dir, "pw_1d_laplacian.txt"))
    S = amg.Solver(problems.tridiag1d(9), coarse_enough=3)
    announce("vcycle worked example")
    z = host(S.vcycle(dev(np.ones(9))))
    ref = np.array([float(v) for v in pw["V"]])
    assert np.max(np.abs(z - ref)) / np.max(np.abs(ref)) <= 1e-12
    S.release()


MIXED_CASES = [
    ("poisson32", {}),
    ("diffusion24", {}),
    ("convection24", {}),
    ("poisson32", {"relax": "chebyshev"}),
    ("diffusion24", {"relax": "chebyshev", "cheb_degree": 2}),
    ("poisson20", {"relax": "chebyshev", "cheb_degree": 1, "npre": 2, "npost": 2}),
    ("poisson27-16", {}),
    ("aniso20", {}),
    ("decoupled14", {}),
    ("graph60k", {}),
]


@pytest.mark.parametrize("name,extra", MIXED_CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(MIXED_CASES)])
def test_vcycle_mixed_matches_fp32_oracle(name, extra):
    A, kw = _problem(name)
    kw = {**kw, **extra}
    S = amg.Solver(A, precision="mixed", **kw)
    h = oracle.setup(A, _oracle_params(kw))
    r = np.random.default_rng(12).standard_normal(A.n)
    announce("vcycle mixed", name)
    z = host(S.vcycle(dev(r)))
    z32 = oracle.vcycle_fp32(h, r)
    z64 = oracle.vcycle(h, r)
    e32, m32 = rel_err(z, z32), max_rel(z, z32)
    e64, m64, o64 = rel_err(z, z64), max_rel(z, z64), rel_err(z32, z64)
    tol = mixed_vcycle_tol(S.nlevels, kw)
    print(f"[mixed vcycle] {name} {extra}: vs FP32 oracle rel {e32:.2e} max {m32:.2e}; "
          f"vs FP64 oracle rel {e64:.2e} max {m64:.2e}; FP32 oracle vs FP64 oracle {o64:.2e}; "
          f"bound {tol:.2e}", flush=True)
    assert e32 <= tol and m32 <= 2 * tol
    assert e64 <= tol and m64 <= 2 * tol
    S.release()


# ------------------------------------------------------------------ solves


SOLVE_CASES = [
    ("poisson32", "ones", {}),
    ("poisson32", "uniform", {"precision": "mixed"}),
    ("diffusion24", "ones", {}),
    ("diffusion24", "ones", {"solver": "bicgstab", "relax": "jacobi"}),
    ("convection24", "ones", {"solver": "bicgstab"}),
    ("convection24", "ones", {"solver": "bicgstab", "precision": "mixed"}),
    ("poisson32", "uniform", {"relax": "chebyshev"}),
    ("diffusion24", "ones", {"relax": "chebyshev", "precision": "mixed"}),
    ("diffusion24", "ones", {"relax": "chebyshev", "solver": "bicgstab"}),
    # flexible GMRES(m)
    ("poisson32", "uniform", {"solver": "gmres"}),
    ("convection24", "ones", {"solver": "gmres"}),
    ("convection24", "ones", {"solver": "gmres", "precision": "mixed"}),
    ("convection24", "ones", {"solver": "gmres", "gmres_m": 4}),
    ("diffusion24", "ones", {"solver": "gmres", "gmres_m": 2}),
    ("diffusion24", "uniform", {"solver": "gmres", "relax": "chebyshev", "check_every": 1}),
    ("poisson27-16", "uniform", {}),
    ("aniso20", "ones", {}),
    ("aniso20", "uniform", {"solver": "gmres"}),
    ("decoupled14", "ones", {"relax": "jacobi"}),
    ("graph60k", "uniform", {}),
    ("graph60k", "ones", {"solver": "bicgstab", "precision": "mixed"}),
]


@pytest.mark.parametrize("name,rhs,kw", SOLVE_CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(SOLVE_CASES)])
def test_solve_matches_oracle(name, rhs, kw):
    A, base = _problem(name)
    kw = {**base, **kw}
    f = problems.rhs_ones(A.n) if rhs == "ones" else problems.rhs_uniform(A.n, 0)
    S = amg.Solver(A, **kw)
    announce("solve", name, kw)
    x, info = S.solve(dev(f))
    x = host(x)
    xo, io, _ = oracle.solve(A, f, _oracle_params(kw), mixed=kw.get("precision") == "mixed")
    print("device iters", info["iters"], "oracle iters", io.iters, "true", info["true_rel_resid"])
    assert info["status"] == 0
    assert abs(info["iters"] - io.iters) <= 1
    tr = true_rel_residual(A, x, f)
    assert tr <= 1e-8
    assert abs(tr - info["true_rel_resid"]) <= 1e-3 * tr + 1e-15
    assert rel_err(x, xo) <= 1e-6
    S.release()


def _tridiag(n, lower, diag, upper):
    rows, cols, vals, rp = [], [], [], [0]
    for i in range(n):
        for j, v in ((i - 1, lower), (i, diag), (i + 1, upper)):
            if 0 <= j < n:
                cols.append(j)
                vals.append(v)
        rp.append(len(cols))
    return problems.CSR(n, np.array(rp, dtype=np.int64), np.array(cols, dtype=np.int32),
                        np.array(vals, dtype=np.float64))


COARSE_CASES = ([("spd", n) for n in (255, 383, 511, 895, 900, 1023, 2999)]
                + [("dense-spd", n) for n in (65, 383, 1000)]
                + [("nonsymmetric", n) for n in (255, 895, 2999)]
                + [("indefinite", n) for n in (255, 895, 2999)])


def _dense_spd(n):
    """B B^T / n + I with Gaussian B (seed n), stored as a full CSR matrix:
    every Gauss-Jordan block update meets nonzero entries."""
    B = np.random.default_rng(n).standard_normal((n, n))
    M = B @ B.T / n + np.eye(n)
    M = 0.5 * (M + M.T)
    rp = np.arange(0, n * n + 1, n, dtype=np.int64)
    cols = np.tile(np.arange(n, dtype=np.int32), n)
    return problems.CSR(n, rp, cols, M.reshape(-1).copy())


@pytest.mark.parametrize("kind,n", COARSE_CASES, ids=[f"{k}-{n}" for k, n in COARSE_CASES])
def test_coarse_inverse_every_order(kind, n):
    """Single-level hierarchy (the whole matrix is the coarsest level): the
    device's dense inverse applied to f equals a dense solve.  A symmetric
    positive definite matrix is factored without pivoting (every pivot comes
    out positive); a nonsymmetric one, and a symmetric indefinite one (whose
    unpivoted factorisation meets a non-positive pivot, so the LU with
    partial pivoting runs on a fresh copy), take LU with partial pivoting.  Orders of the form
    128k - 1 are included on purpose: an in-place LAPACK-style inversion of
    the ROCm stack was found wrong at those."""
    if kind == "spd":
        A = problems.tridiag1d(n)
    elif kind == "dense-spd":
        A = _dense_spd(n)
    elif kind == "nonsymmetric":
        A = _tridiag(n, -1.2, 2.5, -0.8)
    else:
        A = _tridiag(n, -2.0, 1.0, -2.0)
        assert np.linalg.eigvalsh(A.to_scipy().toarray()).min() < 0
    S = amg.Solver(A, coarse_enough=n, solver="cg" if kind.endswith("spd") else "bicgstab")
    assert S.nlevels == 1
    f = np.random.default_rng(n).standard_normal(n)
    announce("coarse inverse", kind, "order", n)
    z = host(S.vcycle(dev(f)))
    zr = np.linalg.solve(A.to_scipy().toarray(), f)
    assert rel_err(z, zr) <= 1e-8
    S.release()


def test_solve_with_coarsest_order_895():
    """Diffusion 45^3, k = exp(g), sigma 1, length 8, field seed 10332, f = 1:
    a three-level hierarchy whose coarsest order is 895.  Iterations within
    +-1 of the oracle and the true residual on the CPU."""
    A = problems.diffusion3d(45, problems.gaussian_field(45, 1.0, 8.0, 10332))
    f = problems.rhs_ones(A.n)
    h = oracle.setup(A)
    assert h.levels[-1].A.shape[0] == 895
    for precision in ("fp64", "mixed"):
        S = amg.Solver(A, precision=precision)
        announce("coarsest order 895 solve", precision)
        x, info = S.solve(dev(f))
        _, io, _ = oracle.solve(A, f, h=h, mixed=(precision == "mixed"))
        assert info["status"] == 0
        assert abs(info["iters"] - io.iters) <= 1
        assert true_rel_residual(A, host(x), f) <= 1e-8
        S.release()


@pytest.mark.parametrize("name", ["poisson32", "diffusion24", "convection24", "convection40", "poisson27-16",
                                  "aniso20", "decoupled14", "graph60k"])
def test_device_galerkin_matches_host_setup(name):
    """The device setup runs the strength graph, the smoothed prolongator,
    R = P^T, the smoother diagonal and the Galerkin products on the GPU;
    every level must be bit-identical to the host setup's (same arithmetic,
    same order)."""
    if name == "convection40":
        g = problems.gaussian_field(40, 2.0, 8.0, 3)
        A, kw = problems.diffusion3d(40, g, velocity=(50.0, 25.0, 12.5)), {"relax": "jacobi"}
    else:
        A, kw = _problem(name)
    S = amg.Solver(A, **kw)
    H = amg.HostHierarchy(A, **kw)
    announce("device galerkin", name, "levels", S.nlevels)
    assert S.nlevels == H.nlevels >= 2
    for l in range(S.nlevels):
        Ad, Ah = S.level_scipy(l, "A"), H.level_scipy(l, "A")
        assert np.array_equal(Ad.indptr, Ah.indptr) and np.array_equal(Ad.indices, Ah.indices)
        assert np.array_equal(Ad.data, Ah.data), l
    for l in range(S.nlevels - 1):
        assert np.array_equal(S.aggregates(l), H.aggregates(l))
        Pd, Ph = S.level_scipy(l, "P"), H.level_scipy(l, "P")
        assert np.array_equal(Pd.indptr, Ph.indptr) and np.array_equal(Pd.indices, Ph.indices)
        assert np.array_equal(Pd.data, Ph.data), l
        Rd, Rh = S.level_scipy(l, "R"), H.level_scipy(l, "R")
        assert np.array_equal(Rd.indptr, Rh.indptr) and np.array_equal(Rd.indices, Rh.indices)
        assert np.array_equal(Rd.data, Rh.data), l
        md, omd = S.smoother(l)[:2]
        mh, omh = H.smoother(l)[:2]
        assert np.array_equal(md, mh), l  # smoother diagonal
        assert omd == omh  # prolongator damping omega
    S.release()
    H.release()


def test_device_setup_structurally_nonsymmetric_falls_back():
    """A pattern without its transpose (row i holds i+37, row i+37 not i): the
    union of the strength graph then has entries A does not store, so that
    step runs on the host while the other steps stay on the device; the
    hierarchy must still equal the host setup's bit for bit."""
    n = 6000
    rp, cols, vals = [0], [], []
    for i in range(n):
        for j, v in ((i - 1, -1.0), (i, 4.0), (i + 37, -0.3)):
            if 0 <= j < n:
                cols.append(j)
                vals.append(v)
        rp.append(len(cols))
    A = problems.CSR(n, np.array(rp, dtype=np.int64), np.array(cols, dtype=np.int32), np.array(vals))
    S = amg.Solver(A, solver="bicgstab", relax="jacobi")
    H = amg.HostHierarchy(A, solver="bicgstab", relax="jacobi")
    announce("device setup nonsymmetric pattern, levels", S.nlevels)
    assert S.nlevels == H.nlevels >= 2
    for l in range(S.nlevels):
        Ad, Ah = S.level_scipy(l, "A"), H.level_scipy(l, "A")
        assert np.array_equal(Ad.indptr, Ah.indptr) and np.array_equal(Ad.indices, Ah.indices)
        assert np.array_equal(Ad.data, Ah.data), l
    for l in range(S.nlevels - 1):
        assert np.array_equal(S.aggregates(l), H.aggregates(l))
        assert abs(S.level_scipy(l, "P") - H.level_scipy(l, "P")).max() == 0.0
    f = problems.rhs_ones(n)
    x, info = S.solve(dev(f))
    assert info["status"] == 0 and true_rel_residual(A, host(x), f) <= 1e-8
    S.release()
    H.release()


@pytest.mark.parametrize("frac", [0.1, 0.35, 0.6, 0.85])
def test_setup_under_device_memory_limit(frac):
    """A device allocator that refuses requests past a byte limit (a fraction
    of the unlimited setup's peak).  Every setup step that cannot get its
    device memory runs on the host, after the host copies still in flight
    have landed, and when the solver's own storage does not fit beside the
    setup's level copies, those are let go and the storage is built again
    from the host hierarchy.  The setup then either succeeds with every level
    equal to the host setup's bit for bit and a converging solve, or reports
    out of memory, and nothing else happens."""
    A, kw = _problem("diffusion24")
    full = amg.Solver(A, **kw)
    peak = full.peak_bytes
    full.release()
    H = amg.HostHierarchy(A, **kw)
    announce("setup under a device memory limit", frac, "of", peak, "bytes")
    try:
        S = amg.Solver(A, alloc_limit=int(frac * peak), **kw)
    except amg.AmgError as e:
        assert e.code == -5, e  # AMG_ERR_OOM
        print(f"[limit] {frac:.2f} of {peak} bytes: out of memory", flush=True)
        H.release()
        return
    print(f"[limit] {frac:.2f} of {peak} bytes: set up, peak {S.peak_bytes}", flush=True)
    assert S.peak_bytes <= frac * peak
    assert S.nlevels == H.nlevels
    for l in range(S.nlevels):
        for which in (("A", "P", "R") if l + 1 < S.nlevels else ("A",)):
            Md, Mh = S.level_scipy(l, which), H.level_scipy(l, which)
            assert np.array_equal(Md.indptr, Mh.indptr) and np.array_equal(Md.indices, Mh.indices)
            assert np.array_equal(Md.data, Mh.data), (l, which)
    for l in range(S.nlevels - 1):
        assert np.array_equal(S.aggregates(l), H.aggregates(l))
        assert np.array_equal(S.smoother(l)[0], H.smoother(l)[0])
    f = problems.rhs_ones(A.n)
    x, info = S.solve(dev(f))
    assert info["status"] == 0 and true_rel_residual(A, host(x), f) <= 1e-8
    S.release()
    H.release()


@pytest.mark.parametrize("solver", ["cg", "bicgstab", "gmres"])
def test_zero_rhs_gives_zero(solver):
    A, _ = _problem("poisson20")
    S = amg.Solver(A, solver=solver)
    x, info = S.solve(dev(np.zeros(A.n)), x0=dev(np.ones(A.n)))
    assert info["iters"] == 0 and info["status"] == 0
    assert not host(x).any()
    S.release()


def test_single_level_is_exact():
    A = problems.poisson3d(10)
    for solver in ("cg", "bicgstab", "gmres"):
        S = amg.Solver(A, solver=solver)
        assert S.nlevels == 1
        f = problems.rhs_ones(A.n)
        x, info = S.solve(dev(f))
        assert info["iters"] == 1
        assert true_rel_residual(A, host(x), f) <= 1e-12
        S.release()


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("solver", ["cg", "bicgstab", "gmres"])
def test_tiny_systems(n, solver):
    """Degenerate sizes: the whole matrix is the coarsest level (dense inverse);
    every solver returns A^-1 f after one iteration."""
    A = problems.tridiag1d(n)
    f = np.arange(1.0, n + 1.0)
    S = amg.Solver(A, solver=solver)
    assert S.nlevels == 1
    announce("tiny system", n, solver)
    x, info = S.solve(dev(f))
    xr = np.linalg.solve(A.to_scipy().toarray(), f)
    assert info["status"] == 0 and info["iters"] == 1
    assert np.max(np.abs(host(x) - xr)) <= 1e-14 * np.max(np.abs(xr))
    S.release()


@pytest.mark.parametrize("solver", ["cg", "gmres"])
def test_exact_initial_guess_needs_no_iteration(solver):
    A, _ = _problem("poisson20")
    f = problems.rhs_ones(A.n)
    xs = np.linalg.solve(A.to_scipy().toarray(), f)
    S = amg.Solver(A, solver=solver)
    x, info = S.solve(dev(f), x0=dev(xs))
    assert info["iters"] == 0 and info["status"] == 0
    S.release()


@pytest.mark.parametrize("solver,limit", [("cg", 1), ("gmres", 1), ("gmres", 3)])
def test_iteration_limit_reports_not_converged(solver, limit):
    A, _ = _problem("poisson32")
    S = amg.Solver(A, max_iter=limit, solver=solver)
    x, info = S.solve(dev(problems.rhs_ones(A.n)), raise_on_error=False)
    assert info["status"] == amg.AMG_NOT_CONVERGED and info["iters"] == limit
    S.release()


def test_singular_coarse_level_is_reported():
    # 1-D Neumann Laplacian: singular (constant null space), positive diagonal;
    # n <= coarse_enough, so the whole matrix is the coarsest level.
    n = 6
    rows, cols, vals = [], [], []
    rp = [0]
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                cols.append(j)
                vals.append(-1.0 if j != i else (1.0 if i in (0, n - 1) else 2.0))
        rp.append(len(cols))
    A = problems.CSR(n, np.array(rp, dtype=np.int64), np.array(cols, dtype=np.int32), np.array(vals))
    with pytest.raises(amg.AmgError) as e:
        amg.Solver(A)
    assert e.value.code == -4


@pytest.mark.parametrize("solver", ["cg", "gmres"])
def test_graph_and_direct_launch_identical_and_deterministic(solver):
    A, _ = _problem("diffusion24")
    f = problems.rhs_ones(A.n)
    out = []
    for use_graph in (1, 0, 1):
        S = amg.Solver(A, use_graph=use_graph, solver=solver)
        x, info = S.solve(dev(f))
        out.append((host(x), info["iters"]))
        S.release()
    assert out[0][1] == out[1][1] == out[2][1]
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][0], out[2][0])


def test_repeated_solves_reuse_hierarchy():
    A, _ = _problem("poisson32")
    S = amg.Solver(A, check_every=1)
    f1 = problems.rhs_ones(A.n)
    f2 = problems.rhs_uniform(A.n, 3)
    x1, i1 = S.solve(dev(f1))
    x2, i2 = S.solve(dev(f2))
    x1b, i1b = S.solve(dev(f1))
    assert np.array_equal(host(x1), host(x1b)) and i1["iters"] == i1b["iters"]
    assert true_rel_residual(A, host(x2), f2) <= 1e-8
    S.release()


# ------------------------------------------------------------------ full size


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_poisson150(precision):
    """The 150^3 workload as the benchmark runs it: oracle-parity on one V-cycle
    and on the iteration count, and the true residual recomputed on the CPU."""
    A = problems.poisson3d(150)
    f = problems.rhs_uniform(A.n, 0)
    announce("full size 150^3 setup", precision)
    S = amg.Solver(A, precision=precision)
    h = oracle.setup(A)
    assert S.nlevels == h.nlevels
    for l in range(S.nlevels - 1):
        assert np.array_equal(S.aggregates(l), h.levels[l].agg)
    # coarse operators from the device Galerkin products: equal to the oracle's
    for l in range(1, S.nlevels):
        assert abs(S.level_scipy(l, "A") - h.levels[l].A).max() == 0.0, l
    announce("full size 150^3 vcycle", precision)
    z = host(S.vcycle(dev(f)))
    zo = oracle.vcycle(h, f) if precision == "fp64" else oracle.vcycle_fp32(h, f)
    e, m = rel_err(z, zo), max_rel(z, zo)
    print(f"[full size vcycle] {precision}: vs oracle rel {e:.2e} max {m:.2e}", flush=True)
    if precision == "fp64":
        assert e <= 1e-12 and m <= 1e-12
    else:
        tol = mixed_vcycle_tol(S.nlevels, {})
        assert e <= tol and m <= 2 * tol, (e, m, tol)
    announce("full size 150^3 solve", precision)
    x, info = S.solve(dev(f))
    x = host(x)
    _, io, _ = oracle.solve(A, f, mixed=(precision == "mixed"), h=h)
    print(precision, "device iters", info["iters"], "oracle", io.iters, "solve_s", info["solve_s"])
    assert abs(info["iters"] - io.iters) <= 1
    assert true_rel_residual(A, x, f) <= 1e-8
    S.release()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("variant", ["sym-cg-spai0", "sym-bicgstab-jacobi", "nonsym-bicgstab-jacobi",
                                     "sym-cg-chebyshev", "nonsym-gmres-jacobi"])
def test_full_size_diffusion128(variant):
    """128^3 variable-coefficient diffusion, k = exp(g), sigma 2, length 8
    (field seed 1), f = 1; the nonsymmetric form adds upwind convection
    (1, 0.5, 0.25) * 50.  Iterations within +-1 of the oracle, true residual
    <= 1e-8 recomputed on the CPU, one V-cycle within 1e-12 of the oracle."""
    N = 128
    g = problems.gaussian_field(N, 2.0, 8.0, 1)
    vel = (50.0, 25.0, 12.5) if variant.startswith("nonsym") else None
    A = problems.diffusion3d(N, g, velocity=vel)
    f = problems.rhs_ones(A.n)
    _, solver, relax = variant.split("-")
    announce("full size diffusion 128^3", variant)
    S = amg.Solver(A, solver=solver, relax=relax)
    prm = oracle.Params(solver=solver, relax=relax)
    h = oracle.setup(A, prm)
    assert S.nlevels == h.nlevels
    r = np.random.default_rng(13).standard_normal(A.n)
    z, zo = host(S.vcycle(dev(r))), oracle.vcycle(h, r)
    assert rel_err(z, zo) <= 1e-12 and max_rel(z, zo) <= 1e-12
    x, info = S.solve(dev(f))
    x = host(x)
    _, io, _ = oracle.solve(A, f, prm, h=h)
    print(variant, "device iters", info["iters"], "oracle", io.iters, "solve_s", info["solve_s"])
    assert info["status"] == 0
    assert abs(info["iters"] - io.iters) <= 1
    assert true_rel_residual(A, x, f) <= 1e-8
    S.release()


@pytest.mark.timeout(900)
def test_full_size_poisson200_mixed_and_fp64():
    """200^3 Poisson, f = U[0,1) seed 0: the mixed-precision solve (FP32
    V-cycle, FP64 Krylov and coarse solve) and the plain FP64 solve both reach
    a true FP64 relative residual <= 1e-8; iterations within +-1 of the oracle
    (FP64 and FP32-V-cycle oracles)."""
    A = problems.poisson3d(200)
    f = problems.rhs_uniform(A.n, 0)
    h = oracle.setup(A)
    out = {}
    for precision in ("fp64", "mixed"):
        announce("full size 200^3", precision)
        S = amg.Solver(A, precision=precision)
        x, info = S.solve(dev(f))
        x = host(x)
        _, io, _ = oracle.solve(A, f, mixed=(precision == "mixed"), h=h)
        print(precision, "device iters", info["iters"], "oracle", io.iters, "solve_s", info["solve_s"])
        assert abs(info["iters"] - io.iters) <= 1
        assert true_rel_residual(A, x, f) <= 1e-8
        out[precision] = x
        S.release()
    # both are solutions to 1e-8: they agree far below the discretisation scale
    assert rel_err(out["mixed"], out["fp64"]) <= 1e-6
