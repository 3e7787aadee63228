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
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solve s + V-cycle HBM GB/s, Poisson 150³ FP64 vs mixed; p50/p99 latency"

WORKLOADS = {
    # name: (grid N, rhs)
    "poisson150": (150, "uniform"),
    "poisson32": (32, "ones"),
    "poisson200": (200, "uniform"),
}


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


def kernel_table(S, reps):
    out = {}
    for k in S.KERNELS:
        us, by = S.time_kernel(k, reps=reps)
        out[k] = {"us": us, "bytes": by, "GBps": by / us / 1e3, "frac": by / us / 1e3 / HBM_PEAK_GBS}
    return out


def cpu_baseline(A, f, x_gpu_by_prec):
    """The oracle, single-threaded, on the host: one full FP64 solve at the
    benchmark size (the oracle hierarchy is built first and not timed)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle

    with threadpool_limits(limits=1):
        t = time.perf_counter()
        h = oracle.setup(A)
        t_setup = time.perf_counter() - t
        log(f"oracle setup {t_setup:.1f} s")
        t = time.perf_counter()
        xo, io, _ = oracle.solve(A, f, h=h)
        t_solve = time.perf_counter() - t
    errs = {p: float(np.linalg.norm(x - xo) / np.linalg.norm(xo)) for p, x in x_gpu_by_prec.items()}
    return {
        "value": t_solve,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": "one full FP64 AMG-PCG solve of the same system (oracle hierarchy built first, "
                  f"{t_setup:.1f} s, untimed); NumPy/SciPy pinned to 1 thread",
        "iters": io.iters,
        "true_rel_resid": io.true_rel_resid,
        "setup_s": t_setup,
        "host_cpus": os.cpu_count(),
    }, errs


def pmc_probe(N, torch, amg, problems):
    """Counter calibration and hot-kernel dispatches for rocprofv3 --pmc runs.

    A device-to-device copy of exactly 1 GiB (read 1 GiB, write 1 GiB) gives
    the scale between the counters and bytes; then each level-1 kernel and
    the V-cycle are launched through amg_time_kernel (reps launches after one
    warm-up) in FP64 and mixed precision.
    """
    torch.cuda.set_device(0)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    A = problems.poisson3d(N)
    out = {"copy_bytes": src.numel() * 8}
    for prec in ("fp64", "mixed"):
        S = amg.Solver(A, precision=prec)
        for k in S.KERNELS:
            us, by = S.time_kernel(k, reps=3)
            out[f"{prec}:{k}"] = {"us": us, "bytes": by}
        S.release()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="poisson150", choices=sorted(WORKLOADS))
    ap.add_argument("--reps", type=int, default=50, help="launches per kernel / V-cycle timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only launch a 1 GiB copy and a few launches of each hot kernel (run under "
                         "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU path is "
              "not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import problems
    from paper_1811_05704_amd import amg

    N, rhs = WORKLOADS[args.workload]
    if args.pmc_probe:
        pmc_probe(N, torch, amg, problems)
        return
    A = problems.poisson3d(N)
    f_host = problems.rhs_uniform(A.n, 0) if rhs == "uniform" else problems.rhs_ones(A.n)
    torch.cuda.set_device(0)
    f = torch.tensor(f_host, device="cuda")
    log(f"workload {args.workload}: n={A.n} nnz={A.nnz}")

    results = {}
    xs = {}
    precs = ["fp64"] if args.no_mixed else ["fp64", "mixed"]
    for prec in precs:
        log(f"setup {prec}")
        S = amg.Solver(A, precision=prec)
        levels = [S.level_info(l) for l in range(S.nlevels)]
        log(f"{prec}: levels {levels}")
        x, info, times, wall = run_solves(S, f, args.steps, args.warmup, torch)
        xs[prec] = x.cpu().numpy()
        true_res = float(np.linalg.norm(f_host - A.to_scipy() @ xs[prec]) / np.linalg.norm(f_host))
        log(f"{prec}: {info['iters']} iters, solve {np.mean(times) * 1e3:.2f} ms, true res {true_res:.2e}")
        ktab = kernel_table(S, args.reps)
        vc = ktab.pop("vcycle")
        results[prec] = {
            "solve_s_mean": wall / args.steps,
            "solve_s_p50": pct(times, 50),
            "solve_s_p99": pct(times, 99),
            "iters": info["iters"],
            "true_rel_resid": true_res,
            "setup_s": info["setup_s"],
            "op_complexity": info["op_complexity"],
            "levels": [{"n": n, "nnz_A": a, "nnz_P": p} for n, a, p in levels],
            "vcycle_us": vc["us"],
            "vcycle_bytes": vc["bytes"],
            "vcycle_GBps": vc["GBps"],
            "vcycle_frac_of_peak": vc["frac"],
            "kernels": ktab,
        }
        S.release()

    base = results["fp64"]
    dom_name, dom = max(base["kernels"].items(), key=lambda kv: kv[1]["us"])
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
            "workload": f"poisson3d {N}^3 (n={A.n}, nnz={A.nnz}), f={'U[0,1) seed 0' if rhs == 'uniform' else 'ones'}, "
                        "AMG-PCG: smoothed aggregation eps 0.08, SPAI-0 1+1 sweeps, V-cycle, "
                        "coarse <= 3000 dense, tol 1e-8",
            "n": A.n,
            "nnz": A.nnz,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom_name,
            "achieved": dom["GBps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["frac"],
            "traffic": None,
        },
        "vcycle_GBps": base["vcycle_GBps"],
        "vcycle_frac_of_peak": base["vcycle_frac_of_peak"],
        "fp64": base,
    }
    if "mixed" in results:
        line["mixed"] = results["mixed"]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cb, errs = cpu_baseline(A, f_host, xs)
        line["cpu_baseline"] = cb
        for p, e in errs.items():
            results[p]["err_vs_fp64_oracle"] = e
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
