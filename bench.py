"""Benchmark: NMPC solves/s to KKT residual 1e-6 on the 64x64 grid, N = 40.

One step = one batch of 256 synthetic heat-process instances (64x64 interior
nodes, 4x4 Gaussian actuator lattice, horizon 40, seeded x0 and reference),
solved from the cold start to r_scaled <= 1e-6 by the double-layer Jacobi
method on one GPU. Inputs for every step are generated and copied to HBM
before the timed region; each step uses its own seeds.

Prints one JSON line with the metric, the roofline of the dominant kernel
(the fused upper-iteration kernel, measured with HIP events on the library's
stream over the timed region) and the CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
KERNEL_SRC = os.path.join(ROOT, "paper_2004_02484_amd", "csrc", "nmpc_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_iterate_c1_b256_traffic.json")
EVAL_SEED0 = 1_000_000         # disjoint from any training seeds


def bytes_per_unit(n: int, m: int, N: int, word: int = 8) -> float:
    """Algorithmic HBM bytes of one (instance, stage) unit of one upper
    iteration: read s_i^k, write s_i^{k+1} (2n + m values each) and the
    instance's x0 and xref once per iteration (2n values shared by N stages)."""
    return word * (2.0 * (2 * n + m) + 2.0 * n / N)


def kernel_digest() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_per_launch(units_per_launch: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_digest") != kernel_digest():
        return None
    return t["bytes_per_unit"] * units_per_launch


def cpu_baseline(P, x0s, xrefs, budget_s: float):
    """The oracle (plain C, FP64, OpenMP over stages) on a bounded sample of
    the first timed batch: cold start, same tolerance and schedule."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    done = 0
    iters = []
    for b in range(x0s.shape[0]):
        o = oracle.solve(P, x0s[b], xrefs[b], tol=1e-6, max_iter=5000)
        iters.append(o["iters"])
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "solves/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{done} of the 256 instances of the first timed batch, 64x64 N=40, "
                      f"cold start, tol 1e-6, iterations {min(iters)}..{max(iters)}, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0 disables)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_2004_02484_amd as nm
    from nmpc_inputs import make_batch, make_problem

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    P = make_problem("c1")
    B = args.batch
    prec = nm.NMPC_FP32_SWEEP if args.precision == "fp32" else nm.NMPC_FP64
    solver = nm.Solver(P, max_batch=B, precision=prec, tol=1e-6, max_iter=5000,
                       check_every=16)

    nb = args.warmup + args.steps
    host = [make_batch(P, range(EVAL_SEED0 + s * B, EVAL_SEED0 + (s + 1) * B)) for s in range(nb)]
    dev_in = [(torch.tensor(x, device=dev), torch.tensor(r, device=dev)) for x, r in host]
    out = (torch.empty((B, P.N, P.n), dtype=torch.float64, device=dev),
           torch.empty((B, P.N, P.m), dtype=torch.float64, device=dev),
           torch.empty((B, P.N, P.n), dtype=torch.float64, device=dev))
    torch.cuda.synchronize()

    for s in range(args.warmup):
        solver.solve_batch(*dev_in[s], out=out)
    torch.cuda.synchronize()

    solver.timing_enable(True)
    iters = []
    worst = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warmup, nb):
        rc, X, U, L, infos = solver.solve_batch(*dev_in[s], out=out)
        worst = max(worst, rc)
        iters += [i["iters"] for i in infos]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = solver.timing_read()
    solver.timing_enable(False)
    elapsed = t1 - t0

    if args.copy_calibration:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)   # 512 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    solves = B * args.steps
    value = solves / elapsed
    avg_launch_s = tm["kernel_ms"] * 1e-3 / max(tm["launches"], 1)
    units_per_launch = tm["units"] / max(tm["launches"], 1)
    bpu = bytes_per_unit(P.n, P.m, P.N)
    achieved = bpu * units_per_launch / avg_launch_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_per_launch(units_per_launch),
            "kernel": "k_iterate (fused upper iteration)",
            "avg_launch_us": round(avg_launch_s * 1e6, 1),
            "units_per_launch": round(units_per_launch, 1),
            "bytes_per_unit": bpu}

    result = {
        "metric": "NMPC solves/s to KKT res 1e-6, 64x64 grid N=40 (batch 256, cold start)",
        "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 sweeps, f64 state/residual" if prec == nm.NMPC_FP32_SWEEP else "f64",
        "data": "synthetic",
        "config": {"workload": "2D nonlinear heat 64x64, N=40, 16 Gaussian inputs, "
                               "batch 256, cold start, tol 1e-6",
                   "global_batch": B, "grid": "64x64", "horizon": P.N,
                   "iters_min": int(min(iters)), "iters_max": int(max(iters)),
                   "iters_mean": round(float(np.mean(iters)), 1), "status_worst": worst},
        "roofline": roof,
    }
    if args.cpu_budget > 0:
        result["cpu_baseline"] = cpu_baseline(P, host[args.warmup][0], host[args.warmup][1],
                                              args.cpu_budget)
    print(json.dumps(result), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
