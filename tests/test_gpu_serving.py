"""Continuous-batching server (GPU).

Every served result must be bitwise identical to the single-solve path
(``amg_solve`` with the same parameters) and hence the same alone and in any
mix, and must match the oracle's solve of the same system (iterations within
one, solution within 1e-6 relative; the distance to the FP64 oracle's
solution is printed); admission under a small HBM budget must still complete
every request; a request that can never fit must fail cleanly.
"""

import time

import numpy as np
import pytest

from tests.gpu_util import announce, rel_err, true_rel_residual

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1811_05704_amd import amg  # noqa: E402

import oracle  # noqa: E402
import problems  # noqa: E402


def request(n, seed):
    g = problems.gaussian_field(n, 1.0, 8.0, seed)
    A = problems.diffusion3d(n, g)
    return A, problems.rhs_ones(A.n)


def serve(reqs, budget=2 << 30, slots=8, threads=4, timeout=120, together=False, **params):
    """Serve the requests; with `together`, wait until all are set up so that
    they are admitted in one step and run in one batch."""
    srv = amg.Server(budget, max_slots=slots, setup_threads=threads, **params)
    for rid, A, f in reqs:
        srv.submit(rid, A, f)
    if together and not srv.wait_ready(len(reqs), timeout):
        failed = [(r[0], r[3], r[2].get("error")) for r in srv.results()]
        srv.release()
        pytest.fail(f"not every request was set up; failed (id, status, error): {failed}")
    got = {}
    t0 = time.time()
    max_live = 0
    while len(got) < len(reqs):
        live, waiting = srv.step()
        max_live = max(max_live, live)
        for r in srv.results():
            got[r[0]] = r
        if live == 0:
            time.sleep(0.002)
        assert time.time() - t0 < timeout, "server did not finish"
    srv.release()
    return got, max_live


def single(A, f, **params):
    S = amg.Solver(A, **{"precision": "mixed", **params})
    x, info = S.solve(torch.tensor(f, device="cuda"))
    S.release()
    return x.cpu().numpy(), info


def oracle_check(rid, A, f, x, info, **params):
    """Served result vs the oracle's solve of the same system and parameters:
    iterations within one, ||x - x_o|| / ||x_o|| <= 1e-6 against the oracle in
    the served precision; the FP64 oracle's distance is printed as well."""
    prm = oracle.Params(relax=params.get("relax", "spai0"), eps_strong=params.get("eps_strong", 0.08))
    mixed = params.get("precision", "mixed") == "mixed"
    xo, io, h = oracle.solve(A, f, prm, mixed=mixed)
    err = rel_err(x, xo)
    err64 = err if not mixed else rel_err(x, oracle.solve(A, f, prm, h=h)[0])
    print(f"[oracle] request {rid} n={A.n}: iters {info['iters']} (oracle {io.iters}), "
          f"vs oracle {err:.2e}, vs FP64 oracle {err64:.2e}", flush=True)
    assert abs(info["iters"] - io.iters) <= 1, (rid, info["iters"], io.iters)
    assert err <= 1e-6, (rid, err)


def test_served_results_equal_single_solves():
    sizes = [16, 22, 18, 27, 20, 24, 17, 30]
    reqs = [(i, *request(n, 10000 + i)) for i, n in enumerate(sizes)]
    announce("serving", len(reqs), "requests")
    got, max_live = serve(reqs, together=True)
    assert max_live == len(reqs)  # all solves in one batch
    for rid, A, f in reqs:
        x_s, info_s = single(A, f)
        _, x, info, status, times = got[rid]
        assert status == 0, (rid, status, info.get("error"))
        assert info["iters"] == info_s["iters"]
        assert np.array_equal(x, x_s), rid
        assert true_rel_residual(A, x, f) <= 1e-8
        submit, ready, admit, done = times
        assert submit <= ready <= admit <= done
        oracle_check(rid, A, f, x, info)


def test_result_same_alone_and_in_mix():
    A, f = request(21, 10100)
    alone, _ = serve([(7, A, f)], slots=4)
    others = [(i, *request(n, 10200 + i)) for i, n in enumerate([19, 25, 16, 23])]
    mix, max_live = serve(others[:2] + [(7, A, f)] + others[2:], slots=8, together=True)
    assert max_live == 5
    assert np.array_equal(alone[7][1], mix[7][1])
    assert alone[7][2]["iters"] == mix[7][2]["iters"]


def test_admission_under_small_budget():
    reqs = [(i, *request(20, 10300 + i)) for i in range(6)]
    # a 20^3 request needs about 11 MiB of device memory: two fit at a time
    budget = 26 << 20
    announce("serving small budget")
    got, max_live = serve(reqs, budget=budget, slots=8, threads=3)
    assert 1 <= max_live < 6
    for rid, A, f in reqs:
        assert got[rid][3] == 0, (rid, got[rid][3], got[rid][2].get("error"))
        assert true_rel_residual(A, got[rid][1], f) <= 1e-8


def test_request_larger_than_budget_fails_cleanly():
    small = request(16, 10400)   # about 4 MiB
    big = request(28, 10401)     # about 63 MiB (dense coarse inverse of 2691 rows)
    got, _ = serve([(1, *small), (2, *big)], budget=24 << 20, slots=2, threads=2)
    assert got[1][3] == 0, got[1][2].get("error")
    assert got[2][3] == -5  # AMG_ERR_OOM: can never fit
    assert "budget" in got[2][2].get("error", "")  # the worker's reason reaches the caller


@pytest.mark.parametrize("params", [{"relax": "jacobi"}, {"precision": "fp64"}])
def test_served_results_equal_single_solves_other_settings(params):
    """Damped Jacobi smoothing and the FP64 V-cycle, served in one batch, give
    bitwise the single-solve results."""
    sizes = [18, 23, 16, 21]
    reqs = [(i, *request(n, 10500 + i)) for i, n in enumerate(sizes)]
    announce("serving", params)
    got, max_live = serve(reqs, together=True, **params)
    assert max_live == len(reqs)
    for rid, A, f in reqs:
        x_s, info_s = single(A, f, **params)
        _, x, info, status, _ = got[rid]
        assert status == 0, (rid, status, info.get("error"))
        assert info["iters"] == info_s["iters"]
        assert np.array_equal(x, x_s), rid
        assert true_rel_residual(A, x, f) <= 1e-8
        oracle_check(rid, A, f, x, info, **params)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_mix_of_structures_equals_single_solves(precision):
    """Requests of different structure in one batch: 27-point rows (four lanes
    per row), weak couplings dropped, isolated identity rows, and an irregular
    graph with hub rows longer than an FP64 stream block.  Every result is
    bitwise the single-solve result."""
    reqs = [
        (0, problems.poisson3d_27(16), problems.rhs_uniform(16**3, 1)),
        (1, problems.anisotropic3d(20, 1e-3), problems.rhs_ones(20**3)),
        (2, problems.decoupled_boundary(14), problems.rhs_ones(16**3)),
        (3, problems.random_laplacian(60000, seed=2), problems.rhs_uniform(60000, 2)),
        (4, *request(19, 10600)),
    ]
    params = {"precision": precision, "eps_strong": 0.02}
    announce("serving mix of structures", precision)
    got, max_live = serve(reqs, together=True, **params)
    assert max_live == len(reqs)
    for rid, A, f in reqs:
        x_s, info_s = single(A, f, **params)
        _, x, info, status, _ = got[rid]
        assert status == 0, (rid, status, info.get("error"))
        assert info["iters"] == info_s["iters"], rid
        assert np.array_equal(x, x_s), rid
        assert true_rel_residual(A, x, f) <= 1e-8
        oracle_check(rid, A, f, x, info, **params)


def test_submissions_from_a_client_thread():
    """Requests submitted from another thread while this one drives the
    server (amg_server_submit beside amg_server_step): every result is still
    bitwise the single-solve result."""
    import threading

    sizes = [17, 22, 19, 25, 16, 21]
    reqs = [(i, *request(n, 10700 + i)) for i, n in enumerate(sizes)]
    srv = amg.Server(2 << 30, max_slots=8, setup_threads=3)
    errors = []

    def client():
        try:
            for rid, A, f in reqs:
                srv.submit(rid, A, f)
                time.sleep(0.003)
        except Exception as e:  # reported below
            errors.append(e)

    announce("serving, client thread submits")
    th = threading.Thread(target=client)
    th.start()
    got = {}
    t0 = time.time()
    while len(got) < len(reqs):
        assert not errors, errors
        srv.step()
        for r in srv.results():
            got[r[0]] = r
        assert time.time() - t0 < 120, "server did not finish"
        time.sleep(0.001)
    th.join()
    srv.release()
    assert not errors, errors
    for rid, A, f in reqs:
        x_s, info_s = single(A, f)
        _, x, info, status, _ = got[rid]
        assert status == 0, (rid, status, info.get("error"))
        assert info["iters"] == info_s["iters"]
        assert np.array_equal(x, x_s), rid


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_long_rows_take_the_vector_schedule(precision):
    """A band matrix with rows of about 1,200 entries (mean row length above
    512: A_1 and R_1 get the 64-lanes-per-row schedule, which the host query
    confirms before anything runs) served beside a diffusion request: both
    results are bitwise the single-solve results and match the oracle."""
    B = problems.banded_spd(6000, 600)
    params = {"precision": precision, "eps_strong": 0.0005}
    H = amg.HostHierarchy(B, **params)
    assert H.nlevels == 2
    assert H.level_kernel_info(0, "A", precision)["kind"] == "vector"
    assert H.level_kernel_info(0, "R", precision)["kind"] == "vector"
    H.release()
    reqs = [(0, B, problems.rhs_ones(B.n)), (1, *request(18, 10800))]
    announce("serving long rows", precision)
    got, max_live = serve(reqs, together=True, **params)
    assert max_live == len(reqs)
    for rid, A, f in reqs:
        x_s, info_s = single(A, f, **params)
        _, x, info, status, _ = got[rid]
        assert status == 0, (rid, status, info.get("error"))
        assert info["iters"] == info_s["iters"], rid
        assert np.array_equal(x, x_s), rid
        assert true_rel_residual(A, x, f) <= 1e-8
        oracle_check(rid, A, f, x, info, **params)
