"""Benchmark: AMG-preconditioned CG on the 150^3 Poisson problem, one GPU.

One step is one complete FP64 solve (PCG + one V-cycle per iteration, to
relative residual 1e-8) of the 150^3 finite-difference Poisson system with a
uniform-random right-hand side, inputs resident in HBM; the hierarchy is set
up once beforehand (its time is reported separately), as in the paper's
shared-memory benchmark (section 4.1: 3,375,000 unknowns, 23,490,000
nonzeros, CG + smoothed aggregation + SPAI-0).  The same system is also
solved with the mixed-precision V-cycle (FP32 hierarchy inside FP64 CG).

Prints ONE JSON line.  Besides the solve time it reports the V-cycle's
achieved bandwidth against MI355X's 8 TB/s HBM peak, the dominant kernel's
roofline fraction (HIP-event timing of repeated launches on the solve
stream, algorithmic bytes), and the oracle timed on the host as a baseline.
The default line also carries a reduced served stream and two short legs:
the Schur field split on the 56^3-node P1 Oseen system and the 4 x 4 block
system of 96^3 nodes (5 timed solves each, FP64 and mixed).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solve s + V-cycle HBM GB/s, Poisson 150³ FP64 vs mixed; p50/p99 latency"

WORKLOADS = {
    # name: (grid N, rhs, matrix kind, solver, relax)
    "poisson150": (150, "uniform", "poisson", "cg", "spai0"),
    "poisson32": (32, "ones", "poisson", "cg", "spai0"),
    "poisson200": (200, "uniform", "poisson", "cg", "spai0"),
    "diffusion128": (128, "ones", "diffusion", "cg", "spai0"),
    "diffusion128-bicgstab": (128, "ones", "diffusion", "bicgstab", "jacobi"),
    "convection128-bicgstab": (128, "ones", "convection", "bicgstab", "jacobi"),
    "convection128-gmres": (128, "ones", "convection", "gmres", "jacobi"),
    "diffusion128-chebyshev": (128, "ones", "diffusion", "cg", "chebyshev"),
    # 4 unknowns per node, 4 x 4 blocks (96^3 nodes: 3,538,944 unknowns)
    "block96": (96, "uniform", "block", "cg", "spai0"),
    # velocity/pressure system of equal-order P1 tetrahedra, Schur pressure
    # correction (56^3 nodes: 702,464 unknowns; section 4's Navier-Stokes
    # system has 713,456)
    "oseen56": (56, "force", "oseen", "bicgstab", "spai0"),
    "oseen56-gmres": (56, "force", "oseen", "gmres", "spai0"),
    "oseen106": (106, "force", "oseen", "bicgstab", "spai0"),
}
KRYLOV_NAMES = {"cg": "PCG", "bicgstab": "BiCGStab", "gmres": "FGMRES(30)"}


def workload_matrix(kind, N):
    import problems

    if kind == "oseen":
        return problems.oseen_p1(N)[0]
    if kind == "poisson":
        return problems.poisson3d(N)
    if kind == "block":
        return problems.coupled_diffusion3d(N, problems.gaussian_field(N, 1.0, 8.0, 2))
    g = problems.gaussian_field(N, 2.0, 8.0, 1)
    vel = (50.0, 25.0, 12.5) if kind == "convection" else None
    return problems.diffusion3d(N, g, velocity=vel)


TRAFFIC_FILES = {w: os.path.join(ROOT, "profiles", f"hbm_traffic_{w}.json") for w in ("poisson150", "oseen56")}
# the kernels, their schedules and the V-cycle driver that picks their gathers and epilogues
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1811_05704_amd", "csrc", f)
                  for f in ("kernels.hpp", "device.hpp", "vcycle.hpp")]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, prec, kernel):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary of the
    workload, or None when there is none or the kernel sources changed since
    the counters were taken."""
    if workload not in TRAFFIC_FILES:
        return None
    try:
        with open(TRAFFIC_FILES[workload]) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch", {}).get(f"{prec}:{kernel}")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pct(v, q):
    import numpy as np

    return float(np.percentile(np.asarray(v), q))


def run_solves(S, f, steps, warmup, torch):
    for _ in range(warmup):
        S.solve(f)
    times, info = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        x, info = S.solve(f)
        times.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return x, info, times, wall


def kernel_table(S, reps, relax="spai0", block=False, split=False):
    """HIP-event timing of the level-1 kernels and of whole V-cycles.  The
    Chebyshev V-cycle runs other kernels than the four level-1 SPAI-0/Jacobi
    kernels, so for it only the outer SpMV and the V-cycle are timed; block
    values time the V-cycle only.  A field split times the SpMV with the
    whole system, the pressure hierarchy's level-1 kernels, its V-cycle and
    the whole preconditioner."""
    out = {}
    if block:
        names = ("vcycle",)
    elif split:
        names = ("split_outer_spmv_dot", "pre_smooth_residual", "post_smooth_dot", "restrict", "prolong", "vcycle",
                 "split_precond")
    else:
        names = ("outer_spmv_dot", "vcycle") if relax == "chebyshev" else S.KERNELS[:6]
    for k in names:
        us, by = S.time_kernel(k, reps=reps)
        out[k] = {"us": us, "bytes": by, "GBps": by / us / 1e3, "frac": by / us / 1e3 / HBM_PEAK_GBS}
    return out


def copy_bandwidth(torch, gib=2, reps=20):
    """Achievable HBM reference: device-to-device copy of `gib` GiB (read + write)."""
    n = (gib << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def cpu_baseline(A, f, x_gpu_by_prec, solver="cg", relax="spai0", n_u=None):
    """The oracle, single-threaded, on the host: one full FP64 solve at the
    benchmark size (the oracle hierarchy is built first and not timed); with
    n_u, the field-split oracle."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle import schur

    with threadpool_limits(limits=1):
        t = time.perf_counter()
        prm = oracle.Params(solver=solver, relax=relax)
        h = oracle.setup(A, prm) if n_u is None else schur.setup(A.to_scipy(), n_u, prm)
        t_setup = time.perf_counter() - t
        log(f"oracle setup {t_setup:.1f} s")
        t = time.perf_counter()
        if n_u is None:
            xo, io, _ = oracle.solve(A, f, prm, h=h)
        else:
            xo, io, _ = schur.solve(A.to_scipy(), f, n_u, prm, ss=h)
        t_solve = time.perf_counter() - t
    errs = {p: float(np.linalg.norm(x - xo) / np.linalg.norm(xo)) for p, x in x_gpu_by_prec.items()}
    return {
        "value": t_solve,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one full FP64 {'AMG' if n_u is None else 'Schur field-split'}-{KRYLOV_NAMES[solver]} solve of the "
                  f"same system (oracle hierarchy built first, {t_setup:.1f} s, untimed); NumPy/SciPy pinned to 1 "
                  f"thread",
        "iters": io.iters,
        "true_rel_resid": io.true_rel_resid,
        "setup_s": t_setup,
        "host_cpus": os.cpu_count(),
    }, errs


def pmc_probe(N, torch, amg, problems, kind="poisson"):
    """Counter calibration and hot-kernel dispatches for rocprofv3 --pmc runs.

    A device-to-device copy of exactly 1 GiB (read 1 GiB, write 1 GiB) gives
    the scale between the counters and bytes; then each level-1 kernel and
    the V-cycle are launched through amg_time_kernel (reps launches after one
    warm-up) in FP64 and mixed precision.  For the field split (kind
    "oseen"): the SpMV with the whole system and the pressure hierarchy's
    level-1 kernels.
    """
    torch.cuda.set_device(0)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    n_u = None
    if kind == "oseen":
        A, n_u = problems.oseen_p1(N)
        names = ("split_outer_spmv_dot", "pre_smooth_residual", "post_smooth_dot", "restrict", "prolong")
    else:
        A = problems.poisson3d(N)
        names = amg.Solver.KERNELS[:6]
    out = {"copy_bytes": src.numel() * 8, "kernel_source_hash": kernel_source_hash()}
    for prec in ("fp64", "mixed"):
        S = amg.Solver(A, precision=prec, n_u=n_u, solver="bicgstab" if n_u else "cg")
        for k in names:
            us, by = S.time_kernel(k, reps=3)
            out[f"{prec}:{k}"] = {"us": us, "bytes": by}
        S.release()
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ serving


def _gen_values(args):
    """Worker: coefficient values of request i (structure is shared per n)."""
    i, n, seed = args
    import problems

    g = problems.gaussian_field(n, 1.0, 8.0, seed)
    return i, problems.diffusion3d(n, g).val


def serving_schedule(count, seed_sizes=6, seed_gaps=5):
    """Request sizes n_i ~ U{16..96}, field seeds 10000 + i, unit-rate exponential gaps."""
    import numpy as np

    sizes = np.random.default_rng(seed_sizes).integers(16, 97, size=count)
    gaps = np.random.default_rng(seed_gaps).exponential(1.0, size=count)
    return sizes, gaps


def generate_requests(count):
    """Sizes, arrival gaps, per-size CSR structure and per-request values of the
    served stream (values computed by a process pool: run before any GPU use)."""
    import multiprocessing as mp

    import numpy as np

    import problems

    sizes, gaps = serving_schedule(count)
    log(f"serving: generating {count} requests (mean n^3 = {float(np.mean(sizes.astype(float) ** 3)):.0f})")
    t = time.perf_counter()
    structs = {}
    for n in sorted(set(int(v) for v in sizes)):
        P = problems.poisson3d(n)
        structs[n] = (P.row_ptr, P.col)
    vals = [None] * count
    with mp.get_context("fork").Pool(processes=max(1, min(16, os.cpu_count() or 1))) as pool:
        for i, v in pool.imap_unordered(_gen_values, [(i, int(sizes[i]), 10000 + i) for i in range(count)],
                                        chunksize=2):
            vals[i] = v
    log(f"serving: generated in {time.perf_counter() - t:.1f} s")
    return {"count": count, "sizes": sizes, "gaps": gaps, "structs": structs, "vals": vals}


def serving_runs(reqs, setup_threads, window, fracs=(0.5, 0.9, 1.2), small_budget=True, fp64_baseline=False,
                 check_every=10):
    """Serve the stream: closed loop (saturation rate mu), then Poisson
    arrivals at each fraction of mu, optionally once more at 0.9 mu under a
    2 GiB budget; optionally the same requests one at a time with plain FP64
    amg_setup + amg_solve (the unbatched baseline), and the served (mixed)
    solutions of every `check_every`-th request against that FP64 solve."""
    import numpy as np

    import problems
    import torch

    from paper_1811_05704_amd import amg

    count = reqs["count"]
    sizes, gaps, structs, vals = reqs["sizes"], reqs["gaps"], reqs["structs"], reqs["vals"]
    torch.cuda.set_device(0)
    torch.cuda.empty_cache()
    free, _total = torch.cuda.mem_get_info()

    class Req:
        __slots__ = ("n", "row_ptr", "col", "val")

    def req(i):
        r = Req()
        n = int(sizes[i])
        r.n = n ** 3
        r.row_ptr, r.col = structs[n]
        r.val = vals[i]
        return r

    ones = {int(n): np.ones(int(n) ** 3) for n in set(sizes.tolist())}
    kept = {}

    def one_run(arrivals, budget, window=None, label="", keep=False):
        """Serve all requests; arrivals = offsets in s (None: closed loop with `window` in flight)."""
        srv = amg.Server(budget, max_slots=64, setup_threads=setup_threads, precision="mixed")
        lat, iters, stat, setup_s, solve_s, queue_s = [], [], [], [], [], []
        failed = []
        t0 = time.perf_counter()
        sub_time = {}
        done = 0
        max_live = 0
        sub_error = []
        # Clients submit on their own thread while this thread drives the
        # server.  Open loop: each request at its arrival time (latency counts
        # from the arrival time).  Closed loop: a new request whenever fewer
        # than `window` are in flight (latency counts from its submission).
        permits = threading.Semaphore(window if arrivals is None else 0)
        if arrivals is not None:
            sub_time = {i: float(arrivals[i]) for i in range(count)}

        def submitter():
            try:
                for i in range(count):
                    if arrivals is None:
                        permits.acquire()
                        sub_time[i] = time.perf_counter() - t0
                    else:
                        wait = arrivals[i] - (time.perf_counter() - t0)
                        if wait > 0:
                            time.sleep(wait)
                    srv.submit(i, req(i), ones[int(sizes[i])])
            except Exception as e:  # reported by the driving loop
                sub_error.append(e)

        sub_thread = threading.Thread(target=submitter, daemon=True)
        sub_thread.start()
        last_progress = time.perf_counter()
        while done < count:
            if sub_error:
                raise sub_error[0]
            if time.perf_counter() - last_progress > 120.0:
                raise RuntimeError(f"serving made no progress for 120 s ({done}/{count} done)")
            live, waiting = srv.step()
            max_live = max(max_live, live)
            for rid, x, info, status, times in srv.results():
                tdone = time.perf_counter() - t0
                lat.append(tdone - sub_time.pop(rid))
                iters.append(info["iters"])
                stat.append(status)
                if keep and rid % check_every == 0:
                    kept[int(rid)] = (np.array(x, copy=True), info["iters"])
                if status != 0:
                    failed.append({"id": int(rid), "n": int(sizes[rid]), "status": int(status), "iters": info["iters"],
                                   "true_rel_resid": info["true_rel_resid"]})
                setup_s.append(info["setup_s"])
                solve_s.append(info["solve_s"])
                queue_s.append(times[2] - times[1])  # set up, waiting for a slot
                done += 1
                permits.release()
                last_progress = time.perf_counter()
            if live == 0:
                time.sleep(0.0005)
        wall = time.perf_counter() - t0
        sub_thread.join()
        srv.release()
        ok = sum(1 for s in stat if s == 0)
        res = {
            "solves_per_s": count / wall,
            "wall_s": wall,
            "latency_p50_s": pct(lat, 50),
            "latency_p99_s": pct(lat, 99),
            "latency_mean_s": float(np.mean(lat)),
            "max_live": max_live,
            "ok": ok,
            "iters_mean": float(np.mean(iters)),
            "iters_max": int(np.max(iters)),
            "setup_s_mean": float(np.mean(setup_s)),
            "device_solve_s_mean": float(np.mean(solve_s)),
            "slot_wait_s_mean": float(np.mean(queue_s)),
            "failed": failed[:32],
        }
        log(f"serving {label}: {res['solves_per_s']:.1f} solves/s, p50 {res['latency_p50_s']:.3f} s, "
            f"p99 {res['latency_p99_s']:.3f} s, max live {max_live}, ok {ok}/{count}")
        if failed:
            log(f"  not ok: {failed[:8]}")
        return res

    budget = int(0.8 * free)
    out = {"requests": count, "budget_bytes": budget, "setup_threads": setup_threads, "max_slots": 64}
    sat = one_run(None, budget, window=window, label="closed loop", keep=fp64_baseline)
    out["closed_loop"] = sat
    mu = sat["solves_per_s"]
    rates = {}
    for frac in fracs:
        lam = frac * mu
        arrivals = np.cumsum(gaps) / lam
        rates[f"{frac}mu"] = {"rate_per_s": lam, **one_run(arrivals, budget, label=f"{frac} mu")}
    out["rates"] = rates
    if small_budget:
        out["small_budget_0.9mu"] = one_run(np.cumsum(gaps) / (0.9 * mu), 2 << 30, label="0.9 mu, 2 GiB budget")
    if fp64_baseline:
        # the same requests, one at a time: plain FP64 setup + solve, no batching
        lat, iters, errs, ok = [], [], [], 0
        t0 = time.perf_counter()
        for i in range(count):
            ts = time.perf_counter()
            r = req(i)
            A = problems.CSR(r.n, r.row_ptr, r.col, r.val)
            S = amg.Solver(A, precision="fp64")
            x, info = S.solve(torch.tensor(ones[int(sizes[i])], device="cuda"))
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ts)
            iters.append(info["iters"])
            ok += int(info["status"] == 0)
            if i in kept:
                x64 = x.cpu().numpy()
                xs, its = kept[i]
                errs.append({"id": i, "n": int(sizes[i]), "served_iters": its, "fp64_iters": info["iters"],
                             "rel_err_vs_fp64": float(np.linalg.norm(xs - x64) / np.linalg.norm(x64))})
            S.release()
        wall = time.perf_counter() - t0
        out["fp64_one_at_a_time"] = {
            "solves_per_s": count / wall, "wall_s": wall, "latency_p50_s": pct(lat, 50),
            "latency_p99_s": pct(lat, 99), "iters_mean": float(np.mean(iters)), "ok": ok,
        }
        out["served_vs_fp64"] = {
            "checked": len(errs),
            "max_rel_err": max(e["rel_err_vs_fp64"] for e in errs) if errs else None,
            "max_iter_diff": max(abs(e["served_iters"] - e["fp64_iters"]) for e in errs) if errs else None,
            "cases": errs[:8],
        }
        log(f"serving fp64 one at a time: {out['fp64_one_at_a_time']['solves_per_s']:.1f} solves/s, "
            f"p50 {out['fp64_one_at_a_time']['latency_p50_s']:.3f} s; served vs FP64 max rel err "
            f"{out['served_vs_fp64']['max_rel_err']}")
    return out


def run_serving(args):
    reqs = generate_requests(args.serving_requests)
    if args.serving_closed_only:
        res = serving_runs(reqs, args.setup_threads, args.serving_window, fracs=(), small_budget=False)
        print(json.dumps({"closed_loop": res["closed_loop"]}), flush=True)
        return
    res = serving_runs(reqs, args.setup_threads, args.serving_window, fp64_baseline=True)
    line = {
        "metric": "served solves/s and p50/p99 latency (arrival -> result on host), mixed AMG-PCG",
        "value": res["rates"]["0.9mu"]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32 V-cycle / f64 Krylov",
        "data": "synthetic",
        "config": {
            "workload": SERVING_WORKLOAD.format(count=args.serving_requests),
            "budget_bytes": res["budget_bytes"],
            "setup_threads": args.setup_threads,
            "max_slots": 64,
        },
        **{k: v for k, v in res.items() if k not in ("requests", "budget_bytes", "setup_threads", "max_slots")},
    }
    print(json.dumps(line), flush=True)


SERVING_WORKLOAD = ("{count} diffusion systems n^3, n~U{{16..96}} (seed 6), k=exp(g), g Gaussian sigma 1 "
                    "length 8 (seed 10000+i), f=1, tol 1e-8, setup + mixed AMG-PCG per request, "
                    "Poisson arrivals (gaps seed 5)")


def measure(name, steps, warmup, reps, no_mixed=False, fuse_coarse=False):
    """Set up and time one workload in FP64 and mixed precision: (A, f_host,
    results per precision, solutions per precision, nnz)."""
    import numpy as np
    import torch

    import problems
    from paper_1811_05704_amd import amg

    N, rhs, kind, solver, relax = WORKLOADS[name]
    n_u = None
    if kind == "oseen":
        A, n_u = problems.oseen_p1(N)
        f_host = problems.oseen_rhs(N)
    else:
        A = workload_matrix(kind, N)
        f_host = problems.rhs_uniform(A.n, 0) if rhs == "uniform" else problems.rhs_ones(A.n)
    torch.cuda.set_device(0)
    f = torch.tensor(f_host, device="cuda")
    nnz = A.nnz if hasattr(A, "nnz") else A.nnzb * A.b * A.b
    log(f"workload {name}: n={A.n} nnz={nnz}")

    results = {}
    xs = {}
    precs = ["fp64"] if no_mixed else ["fp64", "mixed"]
    for prec in precs:
        log(f"setup {prec}")
        S = amg.Solver(A, precision=prec, solver=solver, relax=relax, fuse_coarse=1 if fuse_coarse else 0,
                       n_u=n_u)
        levels = [S.level_info(l) for l in range(S.nlevels)]
        fused_from, fused_grid = S.tail_info()
        log(f"{prec}: levels {levels}")
        x, info, times, wall = run_solves(S, f, steps, warmup, torch)
        xs[prec] = x.cpu().numpy()
        true_res = float(np.linalg.norm(f_host - A.to_scipy() @ xs[prec]) / np.linalg.norm(f_host))
        log(f"{prec}: {info['iters']} iters, solve {np.mean(times) * 1e3:.2f} ms, true res {true_res:.2e}")
        ktab = kernel_table(S, reps, relax, block=(kind == "block"), split=(kind == "oseen"))
        vc = ktab.pop("vcycle")
        pc = ktab.pop("split_precond", None)
        results[prec] = {
            "solve_s_mean": wall / steps,
            "solve_s_p50": pct(times, 50),
            "solve_s_p99": pct(times, 99),
            "iters": info["iters"],
            "true_rel_resid": true_res,
            "setup_s": info["setup_s"],
            "setup_profile_s": S.setup_profile(),
            "op_complexity": info["op_complexity"],
            "levels": [{"n": n, "nnz_A": a, "nnz_P": p} for n, a, p in levels],
            "vcycle_us": vc["us"],
            "vcycle_bytes": vc["bytes"],
            "vcycle_GBps": vc["GBps"],
            "vcycle_frac_of_peak": vc["frac"],
            "fused_from_level": fused_from,
            "fused_workgroups": fused_grid,
            "kernels": ktab,
        }
        if pc is not None:
            results[prec]["split_precond"] = pc
        S.release()

    return A, f_host, results, xs, nnz


def leg_summary(name, steps, warmup, reps):
    """A compact record of another workload for the default line."""
    A, _, res, _, nnz = measure(name, steps, warmup, reps)
    out = {"workload": name, "n": A.n, "nnz": nnz, "steps": steps, "warmup": warmup}
    for prec, r in res.items():
        out[prec] = {k: r[k] for k in ("solve_s_mean", "solve_s_p50", "solve_s_p99", "iters", "true_rel_resid",
                                       "setup_s", "vcycle_us", "vcycle_GBps") if k in r}
        if "split_precond" in r:
            out[prec]["split_precond"] = r["split_precond"]
        if r["kernels"]:
            out[prec]["kernels"] = r["kernels"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="poisson150", choices=sorted(WORKLOADS))
    ap.add_argument("--reps", type=int, default=50, help="launches per kernel / V-cycle timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--fuse-coarse", action="store_true",
                    help="run the small levels and the coarse solve as one persistent launch")
    ap.add_argument("--serving", action="store_true",
                    help="serving benchmark: Poisson arrivals of diffusion systems, continuous batching")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-window", type=int, default=64, help="in-flight requests of the closed loop")
    ap.add_argument("--setup-threads", type=int, default=12)
    ap.add_argument("--serving-closed-only", action="store_true")
    ap.add_argument("--serving-leg", type=int, default=300,
                    help="requests of the reduced served stream in the default line (0: none)")
    ap.add_argument("--legs", default=None,
                    help="comma-separated further workloads measured briefly (5 solves) for the same line "
                         "(default: oseen56,block96 with the poisson150 workload, none otherwise; '' for none)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch a 1 GiB copy and a few launches of each hot kernel (run under "
                         "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.serving:
        run_serving(args)
        return

    import numpy as np
    import torch

    import problems
    from paper_1811_05704_amd import amg

    N, rhs, kind, solver, relax = WORKLOADS[args.workload]
    if args.pmc_probe:
        pmc_probe(N, torch, amg, problems, kind)
        return
    # the served stream's inputs come from a process pool: before any GPU use
    reqs = generate_requests(args.serving_leg) if args.serving_leg > 0 else None
    A, f_host, results, xs, nnz = measure(args.workload, args.steps, args.warmup, args.reps, args.no_mixed,
                                          args.fuse_coarse)

    copy_gbps = copy_bandwidth(torch)
    log(f"device copy reference: {copy_gbps:.0f} GB/s")
    base = results["fp64"]
    cands = dict(base["kernels"])
    if relax == "chebyshev" or kind == "block":  # their per-step kernels are not timed one by one
        cands["vcycle"] = {"us": base["vcycle_us"], "GBps": base["vcycle_GBps"], "frac": base["vcycle_frac_of_peak"]}
    dom_name, dom = max(cands.items(), key=lambda kv: kv[1]["us"])
    line = {
        "metric": METRIC,
        "value": base["solve_s_mean"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": base["solve_s_mean"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"oseen P1 tetrahedra (Kuhn mesh) {N}^3 nodes x 4 fields (n={A.n}, nnz={nnz}), nu 0.01, "
                         f"dt 2h, rotating wind, ASGS-type stabilisation, f=(1,0.5,0.25) h^3, "
                         f"{KRYLOV_NAMES[solver]} with Schur pressure correction: SPAI-0 velocity, smoothed "
                         f"aggregation eps 0.08 spai0 1+1 V-cycle on S - D diag(K)^-1 G, coarse <= 3000 dense, "
                         f"tol 1e-8") if kind == "oseen" else
                        f"{kind}3d {N}^3 (n={A.n}, nnz={nnz}), f={'U[0,1) seed 0' if rhs == 'uniform' else 'ones'}, "
                        f"AMG-{KRYLOV_NAMES[solver]}: smoothed aggregation eps 0.08, "
                        f"{relax + ' degree 3' if relax == 'chebyshev' else relax} 1+1 sweeps, V-cycle, "
                        f"coarse <= 3000 dense, tol 1e-8"
                        + (", 4x4 blocks: coupled 4-field diffusion, k=exp(g) sigma 1 length 8 seed 2"
                           if kind == "block" else "")
                        + (", k=exp(g) sigma 2 length 8 seed 1" if kind not in ("poisson", "block") else "")
                        + (", upwind v=(1,0.5,0.25)*50" if kind == "convection" else ""),
            "n": A.n,
            "nnz": nnz,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom_name,
            "achieved": dom["GBps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["frac"],
            "traffic": measured_traffic(args.workload, "fp64", dom_name),
        },
        "vcycle_GBps": base["vcycle_GBps"],
        "vcycle_frac_of_peak": base["vcycle_frac_of_peak"],
        "copy_GBps": copy_gbps,
        "fp64": base,
    }
    if "mixed" in results:
        line["mixed"] = results["mixed"]
    if reqs is not None:
        log(f"serving leg: {args.serving_leg} requests")
        sv = serving_runs(reqs, args.setup_threads, args.serving_window, fracs=(0.9,), small_budget=False,
                          fp64_baseline=True)
        sv["workload"] = SERVING_WORKLOAD.format(count=args.serving_leg)
        line["serving"] = sv
    # the block and field-split oracles are sized for the parity tests
    legs = args.legs if args.legs is not None else ("oseen56,block96" if args.workload == "poisson150" else "")
    legs = [w for w in legs.split(",") if w]
    if legs:
        line["legs"] = {}
        for w in legs:
            log(f"leg {w}")
            line["legs"][w] = leg_summary(w, 5, 1, 20)
    # the block oracle is sized for the parity tests
    if not args.no_cpu_baseline and kind != "block":
        log("cpu baseline (oracle)")
        cb, errs = cpu_baseline(A, f_host, xs, solver, relax, n_u=3 * N**3 if kind == "oseen" else None)
        line["cpu_baseline"] = cb
        for p, e in errs.items():
            results[p]["err_vs_fp64_oracle"] = e
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
