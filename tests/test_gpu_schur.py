"""Schur-complement field split on the device vs the oracle (GPU).

* One application of the preconditioner (amg_vcycle on a field-split
  handle) on the same vector: relative error <= 1e-12 in FP64, also element
  by element; with the FP32 pressure V-cycle, within the FP32 rounding bound
  of that V-cycle against the oracle's FP32 form.
* Whole BiCGStab / GMRES solves: iterations within +-1 of the oracle, true
  relative residual <= 1e-8 recomputed on the CPU, solution within 1e-6 of
  the oracle's.
* Edge cases: single-level pressure hierarchy, zero right-hand side, CG and
  the no-allocation entry point refused, repeated solves.
"""

import numpy as np
import pytest

from tests.gpu_util import announce, rel_err, true_rel_residual

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1811_05704_amd import amg  # noqa: E402

import oracle  # noqa: E402
from oracle import schur  # noqa: E402
import problems  # noqa: E402
from tests.test_gpu_parity import dev, host, max_rel, mixed_vcycle_tol  # noqa: E402
from tests.test_schur_host import _perturbed_stokes  # noqa: E402


def _problem(name):
    if name == "stokes7":  # pressure block of 343 rows: one level
        return problems.stokes3d(7) + ({},)
    if name == "stokes16":
        return problems.stokes3d(16) + ({"coarse_enough": 500},)
    if name == "stokes24":
        return problems.stokes3d(24) + ({},)
    if name == "stokes20-unstabilised":
        return problems.stokes3d(20, beta=0.0) + ({"coarse_enough": 500},)
    if name == "stokes14-perturbed":
        return _perturbed_stokes(14) + ({"coarse_enough": 500},)
    # equal-order P1 tetrahedra with convection (nonsymmetric K) and
    # stabilisation: the structure of the Navier-Stokes systems
    if name == "oseen16":
        return problems.oseen_p1(16) + ({"coarse_enough": 500},)
    if name == "oseen24":
        return problems.oseen_p1(24) + ({},)
    raise KeyError(name)


def _rhs(name, A):
    N = round((A.n // 4) ** (1 / 3))
    return problems.oseen_rhs(N) if name.startswith("oseen") else problems.stokes_rhs(N)


def _oracle_params(kw):
    keys = ("solver", "relax", "npre", "npost", "coarse_enough", "max_iter", "tol", "gmres_m", "eps_strong")
    return oracle.Params(**{k: v for k, v in kw.items() if k in keys})


APPLY_CASES = [("stokes7", {}), ("stokes16", {}), ("stokes24", {}), ("stokes20-unstabilised", {}),
               ("stokes14-perturbed", {}), ("stokes16", {"relax": "jacobi"}), ("stokes16", {"relax": "chebyshev"}),
               ("oseen16", {}), ("oseen24", {})]


@pytest.mark.parametrize("name,extra", APPLY_CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(APPLY_CASES)])
def test_split_apply_fp64_matches_oracle(name, extra):
    A, n_u, kw = _problem(name)
    kw = {**kw, **extra, "solver": "bicgstab"}
    S = amg.Solver(A, n_u=n_u, **kw)
    ss = schur.setup(A.to_scipy(), n_u, _oracle_params(kw))
    assert S.nlevels == ss.h.nlevels
    r = np.random.default_rng(5).standard_normal(A.n)
    announce("schur apply fp64", name, extra)
    z = host(S.vcycle(dev(r)))
    zo = schur.precond(ss)(r)
    e, m = rel_err(z, zo), max_rel(z, zo)
    print(f"[schur apply] {name} {extra}: levels {S.nlevels} rel {e:.2e} max {m:.2e}", flush=True)
    assert e <= 1e-12 and m <= 1e-12
    S.release()


@pytest.mark.parametrize("name", ["stokes16", "stokes24", "stokes14-perturbed", "oseen24"])
def test_split_apply_mixed_matches_fp32_oracle(name):
    A, n_u, kw = _problem(name)
    kw = {**kw, "solver": "bicgstab"}
    S = amg.Solver(A, n_u=n_u, precision="mixed", **kw)
    ss = schur.setup(A.to_scipy(), n_u, _oracle_params(kw))
    r = np.random.default_rng(6).standard_normal(A.n)
    announce("schur apply mixed", name)
    z = host(S.vcycle(dev(r)))
    z32 = schur.precond(ss, mixed=True)(r)
    z64 = schur.precond(ss)(r)
    tol = mixed_vcycle_tol(S.nlevels, kw)
    e32, m32, e64 = rel_err(z, z32), max_rel(z, z32), rel_err(z, z64)
    print(f"[schur apply mixed] {name}: vs FP32 oracle rel {e32:.2e} max {m32:.2e}; vs FP64 {e64:.2e}; "
          f"bound {tol:.2e}", flush=True)
    assert e32 <= tol and m32 <= 2 * tol and e64 <= tol
    S.release()


SOLVE_CASES = [
    ("stokes16", {"solver": "bicgstab"}),
    ("stokes16", {"solver": "gmres"}),
    ("stokes24", {"solver": "bicgstab"}),
    ("stokes24", {"solver": "bicgstab", "precision": "mixed"}),
    ("stokes24", {"solver": "gmres", "precision": "mixed"}),
    ("stokes24", {"solver": "gmres", "gmres_m": 8}),
    ("stokes7", {"solver": "bicgstab"}),
    ("stokes14-perturbed", {"solver": "bicgstab"}),
    ("stokes20-unstabilised", {"solver": "gmres"}),
    ("oseen16", {"solver": "bicgstab"}),
    ("oseen24", {"solver": "gmres"}),
    ("oseen24", {"solver": "bicgstab", "precision": "mixed"}),
    ("oseen16", {"solver": "gmres", "relax": "chebyshev"}),
    ("stokes16", {"solver": "bicgstab", "npre": 2, "npost": 2}),
    ("oseen16", {"solver": "bicgstab", "relax": "jacobi", "precision": "mixed"}),
]


@pytest.mark.parametrize("name,extra", SOLVE_CASES, ids=[f"{c[0]}-{i}" for i, c in enumerate(SOLVE_CASES)])
def test_split_solve_matches_oracle(name, extra):
    A, n_u, kw = _problem(name)
    kw = {**kw, **extra}
    f = _rhs(name, A)
    S = amg.Solver(A, n_u=n_u, **kw)
    announce("schur solve", name, extra)
    x, info = S.solve(dev(f))
    x = host(x)
    xo, io, _ = schur.solve(A.to_scipy(), f, n_u, _oracle_params(kw), mixed=kw.get("precision") == "mixed")
    print(f"[schur solve] {name} {extra}: device iters {info['iters']} oracle {io.iters} "
          f"true {info['true_rel_resid']:.2e}", flush=True)
    assert info["status"] == 0
    assert abs(info["iters"] - io.iters) <= 1
    tr = true_rel_residual(A, x, f)
    assert tr <= 1e-8
    assert abs(tr - info["true_rel_resid"]) <= 1e-3 * tr + 1e-15
    assert rel_err(x, xo) <= 1e-6
    S.release()


def test_split_zero_rhs_and_repeated_solves():
    A, n_u, kw = _problem("stokes16")
    S = amg.Solver(A, n_u=n_u, solver="bicgstab", **kw)
    x, info = S.solve(dev(np.zeros(A.n)))
    assert info["iters"] == 0 and not host(x).any()
    f = problems.stokes_rhs(16)
    x1, i1 = S.solve(dev(f))
    x2, i2 = S.solve(dev(f))
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(host(x1), host(x2))
    S.release()


def test_split_refuses_cg_and_noalloc():
    A, n_u, kw = _problem("stokes7")
    with pytest.raises(amg.AmgError):
        amg.Solver(A, n_u=n_u, solver="cg")
    S = amg.Solver(A, n_u=n_u, solver="gmres")
    with pytest.raises(amg.AmgError):
        S.vcycle_noalloc(dev(np.ones(A.n)))
    S.release()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_oseen56(precision):
    """The benchmark system (702,464 unknowns, 24.5M nonzeros) in the
    benchmark's configuration: one preconditioner application against the
    oracle's, and the whole solve against the oracle's solve."""
    A, n_u = problems.oseen_p1(56)
    f = problems.oseen_rhs(56)
    mixed = precision == "mixed"
    S = amg.Solver(A, n_u=n_u, solver="bicgstab", precision=precision)
    ss = schur.setup(A.to_scipy(), n_u, oracle.Params(solver="bicgstab"))
    assert S.nlevels == ss.h.nlevels
    r = np.random.default_rng(9).standard_normal(A.n)
    announce("oseen56 apply", precision)
    z = host(S.vcycle(dev(r)))
    zo = schur.precond(ss, mixed=mixed)(r)
    e, m = rel_err(z, zo), max_rel(z, zo)
    tol = mixed_vcycle_tol(S.nlevels, {}) if mixed else 1e-12
    print(f"[oseen56 apply] {precision}: rel {e:.2e} max {m:.2e} bound {tol:.2e}", flush=True)
    assert e <= tol and m <= 2 * tol
    announce("oseen56 solve", precision)
    x, info = S.solve(dev(f))
    x = host(x)
    xo, io, _ = schur.solve(A.to_scipy(), f, n_u, oracle.Params(solver="bicgstab"), mixed=mixed, ss=ss)
    tr = true_rel_residual(A, x, f)
    print(f"[oseen56 solve] {precision}: device iters {info['iters']} oracle {io.iters} true {tr:.2e}", flush=True)
    assert info["status"] == 0 and tr <= 1e-8
    assert abs(info["iters"] - io.iters) <= 1
    assert rel_err(x, xo) <= 1e-6
    S.release()


@pytest.mark.parametrize("name,precision", [("oseen16", "fp64"), ("oseen24", "fp64"), ("oseen24", "mixed")])
def test_masked_split_on_interlaced_system(name, precision):
    """The system numbered node by node (four unknowns per node) with a
    pressure mask: the library works in its velocity-first renumbering
    (each field in the caller's order), so the oracle on that renumbered
    system gives the reference; vectors go in and out in the caller's order."""
    from tests.test_schur_host import interlaced

    A, n_u, kw = _problem(name)
    B, pmask, _ = interlaced(A, n_u)
    order = np.concatenate([np.flatnonzero(pmask == 0), np.flatnonzero(pmask == 1)])
    Bp = B.to_scipy()[order][:, order]
    mixed = precision == "mixed"
    S = amg.Solver(B, pmask=pmask, solver="bicgstab", precision=precision, **kw)
    ss = schur.setup(Bp, n_u, _oracle_params({**kw, "solver": "bicgstab"}))
    assert S.nlevels == ss.h.nlevels
    assert abs(S.level_scipy(0, "A") - ss.S_hat).max() == 0.0
    r = np.random.default_rng(8).standard_normal(B.n)
    announce("masked apply", name, precision)
    z = host(S.vcycle(dev(r)))
    zo = np.empty(B.n)
    zo[order] = schur.precond(ss, mixed=mixed)(r[order])
    e, m = rel_err(z, zo), max_rel(z, zo)
    tol = mixed_vcycle_tol(S.nlevels, kw) if mixed else 1e-12
    print(f"[masked apply] {name} {precision}: rel {e:.2e} max {m:.2e}", flush=True)
    assert e <= tol and m <= 2 * tol
    f = _rhs(name, A)
    # the right-hand side in the caller's (interlaced) order
    n = A.n // 4
    old = np.arange(A.n)
    fB = np.empty(B.n)
    fB[4 * (old % n) + old // n] = f
    announce("masked solve", name, precision)
    x, info = S.solve(dev(fB))
    x = host(x)
    xo_p, io, _ = schur.solve(Bp, fB[order], n_u, _oracle_params({**kw, "solver": "bicgstab"}), mixed=mixed, ss=ss)
    xo = np.empty(B.n)
    xo[order] = xo_p
    tr = true_rel_residual(B, x, fB)
    print(f"[masked solve] {name} {precision}: device iters {info['iters']} oracle {io.iters} true {tr:.2e}",
          flush=True)
    assert info["status"] == 0 and tr <= 1e-8
    assert abs(info["iters"] - io.iters) <= 1
    assert rel_err(x, xo) <= 1e-6
    S.release()


def test_split_graph_and_direct_launch_identical():
    A, n_u, kw = _problem("oseen16")
    f = _rhs("oseen16", A)
    out = []
    for use_graph in (1, 0, 1):
        S = amg.Solver(A, n_u=n_u, solver="bicgstab", use_graph=use_graph, **kw)
        x, info = S.solve(dev(f))
        out.append((host(x), info["iters"]))
        S.release()
    assert out[0][1] == out[1][1] == out[2][1]
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][0], out[2][0])
