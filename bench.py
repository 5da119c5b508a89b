"""Benchmark: NMPC solves/s to KKT residual 1e-6 on the 64x64 grid, N = 40,
learned warm start vs the plain (cold) start.

One step = one batch of 256 synthetic heat-process instances (64x64 interior
nodes, 4x4 Gaussian actuator lattice, horizon 40, seeded x0 and reference)
solved to r_scaled <= 1e-6 by the double-layer Jacobi method on one GPU. With
the learned start (the timed value) a step is: network inference on the
matrix cores (by default the per-actuator linear map on second-order window
features alone; --mlp 1 adds the bf16 hidden path, which leaves the held-out
error and the iteration counts unchanged on this workload) -> predicted
input trajectories -> states by the backward-Euler
rollout and costates by the adjoint recursion -> per-instance fallback to the
cold start if that start's residual is worse -> Jacobi refinement. The same
batches are then solved from the cold start for the comparison. Inputs for
every step are generated and copied to HBM before the timed region; each step
uses its own seeds, disjoint from the network's training seeds.

The upper layer is the stage-parallel Jacobi iteration (eq. 1st_jacobi) by
default (--upper jacobi|fgs|bgs|sgs; the paper's own experiment used SGS,
eq. sgs). Prints one JSON line with the metric, the roofline of the dominant
kernel (the fused Jacobi iteration kernel, or the persistent Gauss-Seidel
kernel, measured with HIP events on the library's stream over the timed
region), the network's matrix-core rate, the per-result FP32-vs-FP64 error,
the FP64-sweep variant on the same batches and the CPU oracle timed on a
bounded sample of the same workload.

--workload selects other workloads for the same kind of line (the default,
64x64 N=40 batch 256, is the headline): "c2" solves single 256x256, N=100
instances (8x8 actuator lattice) on the streaming marching-strip path, "c3"
solves batches of 512 instances of mixed grids {32, 48, 64, 96}^2 and horizons
{20, 40, 60} in the ragged kernel.
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
CSRC = os.path.join(ROOT, "paper_2004_02484_amd", "csrc")
UPPER = {"jacobi": 0, "fgs": 1, "bgs": 2, "sgs": 3}
# dominant kernel per upper layer: (name, sources it is built from, counter summary)
KERNELS = {
    "jacobi": ("k_iterate (fused upper iteration, all stages in parallel)",
               ("nmpc_kernels.hip", "nmpc_stage.h"), "k_iterate_c1_b256_traffic.json"),
    "gs": ("k_gs (persistent Gauss-Seidel sweeps, one workgroup per instance)",
           ("nmpc_gs.hip", "nmpc_stage.h"), "k_gs_c1_b256_traffic.json"),
    "stream": ("streaming upper iteration (marching-strip passes k_st_*, one captured graph)",
               ("nmpc_stream.hip",), "stream_c2_traffic.json"),
    "ragged": ("k_iterate_rg (ragged batch; one upper iteration = one launch per tile case)",
               ("nmpc_ragged.hip", "nmpc_stage.h"), "k_iterate_rg_c3_b512_traffic.json"),
}
WEIGHTS = os.path.join(ROOT, "paper_2004_02484_amd", "weights", "c1_patchnet.npz")
MFMA_BF16_PEAK_TFLOPS = 2500.0
MFMA_F32_PEAK_TFLOPS = 157.3
EVAL_SEED0 = 1_000_000         # disjoint from any training seeds


def bytes_per_unit(n: int, m: int, N: int, word: int = 8, sweeps: int = 1) -> float:
    """Algorithmic HBM bytes of one (instance, stage) unit: each stage sweep
    reads s_i and writes its new value (2n + m values each); the instance's x0
    and xref are read once per sweep (2n values shared by N stages). The
    library counts one unit per stage sweep (a Jacobi iteration is one sweep,
    an SGS iteration two), so the rooflines take sweeps = 1."""
    return word * (sweeps * 2.0 * (2 * n + m) + 2.0 * n / N)


def eval_bytes_per_unit(n: int, m: int, N: int, word: int = 8) -> float:
    """Algorithmic HBM bytes of an evaluation-only unit (the residual check of
    the FP64-corrected iterate): it reads s_i and its share of x0 and xref and
    writes no new iterate."""
    return word * ((2 * n + m) + 2.0 * n / N)


def extra_flags(src: str):
    """The per-source compiler flags the library build adds to this source."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_nmpc_build", os.path.join(ROOT, "paper_2004_02484_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.EXTRA.get(src, [])


def kernel_digest(sources) -> str:
    """Digest of a kernel's sources and of the per-source flags they are built
    with (a counter summary is valid only for the binary it was taken on)."""
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(CSRC, src), "rb") as f:
            h.update(f.read())
        flags = extra_flags(src)
        if flags:
            h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def traffic_per_launch(kind: str, units_per_launch: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source (else None)."""
    _, sources, fname = KERNELS[kind]
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_digest") != kernel_digest(sources):
        return None
    return t["bytes_per_unit"] * units_per_launch


def oracle_native():
    """The oracle built for this host's CPU (-march=native) and loaded."""
    import oracle
    oracle.use_native()
    return oracle


def single_core_ns(oracle, P, x0, xr, seconds: float = 3.0) -> float:
    """The oracle's time per stage-point per upper iteration on one core
    (cold-start iterations of one instance)."""
    oracle.set_threads(1)
    X, U, L = oracle.cold_start(P, x0)
    t = time.perf_counter()
    k = 0
    while time.perf_counter() - t < seconds:
        X, U, L, _, _ = oracle.iterate(P, x0, xr, X, U, L)
        k += 1
    dt = (time.perf_counter() - t) / k
    oracle.set_threads(oracle.threads())
    return dt / (P.N * P.n) * 1e9


def cpu_baseline(P, x0s, xrefs, budget_s: float, upper: str, u_pred=None):
    """The oracle (plain C, FP64, built for the host CPU; OpenMP over stages in
    its KKT evaluation and, for Jacobi, its stage solves) on a bounded sample
    of the first timed batch, same upper layer, tolerance and schedule.

    With u_pred (the network's predicted inputs of that batch, [B][N][m]) the
    value is the refinement from the learned start, the work the GPU's
    solves/s counts after inference: the start's states and costates are
    built from u_pred by the oracle's own input-start construction (sparse LU,
    untimed, as many instances as about a third of the budget allows), then
    the oracle's upper iteration is timed from it. The cold-start rate, and
    the single-core time per stage-point per iteration, are reported beside
    it."""
    oracle = oracle_native()
    threads = oracle.threads()
    oracle.set_threads(threads)
    out = {"unit": "solves/s", "cores": threads, "kind": "oracle"}
    t0 = time.perf_counter()
    done, iters = 0, []
    cold_budget = budget_s / 3 if u_pred is not None else budget_s
    for b in range(x0s.shape[0]):
        o = oracle.solve(P, x0s[b], xrefs[b], tol=1e-6, max_iter=5000, upper=upper)
        iters.append(o["iters"])
        done += 1
        if time.perf_counter() - t0 >= cold_budget:
            break
    dt = time.perf_counter() - t0
    cold = {"solves_per_s": done / dt, "instances": done,
            "iters": f"{min(iters)}..{max(iters)}", "seconds": round(dt, 2)}
    ns = single_core_ns(oracle, P, x0s[0], xrefs[0])
    out["single_core_ns_per_stage_point_iteration"] = round(ns, 1)
    out["paper_single_core_ns_per_stage_point_iteration"] = {
        "value": 123, "hardware": "Intel Core i5-8265U laptop core, C implementation, SGS upper "
                                  "layer, 13x13 copper plate, N = 20 (0.416 ms per iteration)",
        "note": "context only: other problem, machine and upper layer"}
    if u_pred is None:
        out["value"] = cold["solves_per_s"]
        out["sample"] = (f"{done} of the {x0s.shape[0]} instances of the first timed batch, "
                         f"64x64 N=40, cold start, {upper} upper layer, tol 1e-6, iterations "
                         f"{cold['iters']}, {dt:.1f} s")
        return out
    from oracle.start import input_start
    starts, t1 = [], time.perf_counter()
    while len(starts) < x0s.shape[0] and (time.perf_counter() - t1 < budget_s / 3
                                          or len(starts) < 2):
        b = len(starts)
        starts.append(input_start(P, x0s[b], xrefs[b], u_pred[b]))
    reps = 0
    lit = []
    t2 = time.perf_counter()
    while True:
        for b, S in enumerate(starts):
            o = oracle.solve(P, x0s[b], xrefs[b], start=tuple(a.copy() for a in S), tol=1e-6,
                             max_iter=5000, upper=upper)
            if reps == 0:
                lit.append(o["iters"])
        reps += 1
        if time.perf_counter() - t2 >= budget_s / 3:
            break
    dt2 = time.perf_counter() - t2
    out["value"] = reps * len(starts) / dt2
    out["sample"] = (f"refinement from the learned start: the first {len(starts)} instances of "
                     f"the first timed batch (64x64 N=40), start states and costates built by the "
                     f"oracle from the network's predicted inputs (untimed), {upper} upper "
                     f"layer to tol 1e-6 ({min(lit)}..{max(lit)} iterations), solved {reps} "
                     f"times in {dt2:.1f} s; inference and start construction not counted")
    out["cold_start"] = cold
    return out


def net_flops(net, count: int):
    """Flops of one inference over `count` instances (2 per MAC): the bf16
    hidden layers and the fp32 per-actuator linear map."""
    rows = count * net.m
    return (2.0 * rows * (net.K0p * net.H + 2 * net.H * net.H + net.H * net.N),
            2.0 * rows * net.K0p * net.N)


def timed_steps(solver, batches, out, net=None, ubuf=None, errs=None):
    """Solve each batch once (learned start if `net` is given); return per-step
    wall times, iteration counts, starts used and the worst status (errs, if
    given, receives each result's err_vs_fp64)."""
    import torch
    times, iters, used, worst = [], [], [], 0
    torch.cuda.synchronize()
    for x0, xr in batches:
        t = time.perf_counter()
        if net is not None:
            up = net.predict(x0, xr, out=ubuf)
            rc, X, U, L, infos = solver.solve_batch(x0, xr, warm=(None, up, None), out=out)
        else:
            rc, X, U, L, infos = solver.solve_batch(x0, xr, out=out)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        worst = max(worst, rc)
        iters += infos["iters"].tolist()
        used += infos["start_used"].tolist()
        if errs is not None:
            errs += infos["err_vs_fp64"].tolist()
    return times, iters, used, worst


def closed_loop(solver, net, P, x0, xr, steps: int, ubuf):
    """Closed loop of `steps` NMPC steps per instance of one batch (the plant
    is one explicit-Euler step of the model with the applied first input).
    Step 1 starts cold; steps 2..steps are solved three ways on the same
    states: cold, shifted previous solution, learned. Returns per start kind
    solves/s and iterations over steps 2..steps."""
    import torch
    B = x0.shape[0]
    rc, X, U, L, _ = solver.solve_batch(x0, xr)
    X, U, L = X.clone(), U.clone(), L.clone()
    out = {k: {"t": 0.0, "it": []} for k in ("cold", "shifted", "learned")}
    xs = x0.clone()
    for _ in range(2, steps + 1):
        xs = solver.plant_step_batch(xs, U, P.h)
        warm = solver.shift_batch(X, U, L)
        torch.cuda.synchronize()
        for kind in ("cold", "learned", "shifted"):
            t = time.perf_counter()
            if kind == "cold":
                rc, Xo, Uo, Lo, inf = solver.solve_batch(xs, xr)
            elif kind == "learned":
                up = net.predict(xs, xr, out=ubuf)
                rc, Xo, Uo, Lo, inf = solver.solve_batch(xs, xr, warm=(None, up, None))
            else:
                rc, Xo, Uo, Lo, inf = solver.solve_batch(xs, xr, warm=warm)
            torch.cuda.synchronize()
            out[kind]["t"] += time.perf_counter() - t
            out[kind]["it"] += inf["iters"].tolist()
        X, U, L = Xo.clone(), Uo.clone(), Lo.clone()   # the shifted solve's trajectory
    n = B * (steps - 1)
    return {k: {"solves_per_s": round(n / v["t"], 1), "iters_mean": round(float(np.mean(v["it"])), 1),
                "iters_max": int(max(v["it"]))} for k, v in out.items()}


def copy_calibration(dev):
    """A plain 512 MiB device copy (three times): the known-size reference for
    scaling the HBM counters of the same run."""
    import torch
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def roofline(kind: str, tm, bpu: float, bpu_eval: float = 0.0):
    """HBM roofline of the dominant kernel from the library's HIP-event timing
    (kernel_ms, launches, units updated, evaluation-only units) and the
    algorithmic bytes of an updated and of an evaluation-only unit."""
    avg_launch_s = tm["kernel_ms"] * 1e-3 / max(tm["launches"], 1)
    units_per_launch = tm["units"] / max(tm["launches"], 1)
    eval_per_launch = tm.get("eval_units", 0) / max(tm["launches"], 1)
    achieved = (bpu * units_per_launch + bpu_eval * eval_per_launch) / avg_launch_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_per_launch(kind, units_per_launch),
            "kernel": KERNELS[kind][0],
            "avg_launch_us": round(avg_launch_s * 1e6, 1),
            "units_per_launch": round(units_per_launch, 1),
            "bytes_per_unit": round(bpu, 1),
            "eval_units_per_launch": round(eval_per_launch, 1),
            "eval_bytes_per_unit": round(bpu_eval, 1)}


def line(metric, value, args, elapsed, dtype, cfg, roof, cpu=None):
    out = {"metric": metric, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(elapsed / args.steps * 1e3, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic", "config": cfg, "roofline": roof}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def bench_c2(args):
    """Single 256x256, N=100 instances (one per step, own seeds) on the
    streaming path, Jacobi upper layer, FP32 sweeps, tol 1e-6."""
    import torch
    import paper_2004_02484_amd as nm
    from nmpc_inputs import make_instance, make_problem
    dev = torch.device("cuda:0")
    P = make_problem("c2")
    solver = nm.Solver(P, max_batch=1, precision=nm.NMPC_FP32_SWEEP, tol=1e-6, max_iter=5000,
                       check_every=16, upper=nm.NMPC_UPPER_JACOBI)
    cfg_path = solver.kernel_config()
    nb = args.warmup + args.steps
    host = [make_instance(P, EVAL_SEED0 + s) for s in range(nb)]
    dev_in = [(torch.tensor(x, device=dev)[None], torch.tensor(r, device=dev)[None])
              for x, r in host]
    timed_steps(solver, dev_in[:args.warmup], None)
    solver.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, iters, _, worst = timed_steps(solver, dev_in[args.warmup:], None)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = solver.timing_read()
    solver.timing_enable(False)
    if args.copy_calibration:
        copy_calibration(dev)
    # one streaming "launch" is one upper iteration of all N stages
    roof = roofline("stream", tm, bytes_per_unit(P.n, P.m, P.N))
    cfg = {"workload": "2D nonlinear heat 256x256, N=100, 64 Gaussian inputs (8x8 lattice), "
                       "single instance per step, cold start, Jacobi upper layer, streaming "
                       "marching-strip path, tol 1e-6",
           "global_batch": 1, "grid": "256x256", "horizon": P.N, "path": cfg_path,
           "iters_min": int(min(iters)), "iters_max": int(max(iters)),
           "status_worst": worst, "step_ms_median": round(1e3 * float(np.median(times)), 2)}
    cpu = None
    if args.cpu_budget > 0:
        oracle = oracle_native()
        x0, xr = host[args.warmup]
        X, U, L = oracle.cold_start(P, x0)
        t = time.perf_counter()
        k = 0
        while time.perf_counter() - t < args.cpu_budget:
            X, U, L, _, _ = oracle.iterate(P, x0, xr, X, U, L)
            k += 1
        per_it = (time.perf_counter() - t) / k
        it = float(np.mean(iters))
        cpu = {"value": 1.0 / (per_it * it), "unit": "solves/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"{k} cold-start Jacobi upper iterations of the first timed instance "
                         f"({per_it:.2f} s each), scaled by the {it:.0f} iterations the "
                         f"instance takes to tol 1e-6"}
    line("NMPC solves/s to KKT res 1e-6, 256x256 grid N=100, single instance",
         len(times) / elapsed, args, elapsed, "f32 sweeps, f64 state/residual", cfg, roof, cpu)
    solver.close()


def bench_c3(args):
    """Batches of 512 instances of mixed grids and horizons (one batch per
    step, own seeds) in the ragged kernel, Jacobi upper layer, FP32 sweeps."""
    import torch
    import paper_2004_02484_amd as nm
    from nmpc_inputs import make_instance, make_problem, ragged_specs
    dev = torch.device("cuda:0")
    grids, horizons, B = (32, 48, 64, 96), (20, 40, 60), 512
    keys = [(g, h) for g in grids for h in horizons]
    classes = [make_problem("grid", ns=g, N=h, lattice=4) for g, h in keys]
    solver = nm.RaggedSolver(classes, max_instances=B, tol=1e-6, max_iter=5000,
                             precision=nm.NMPC_FP32_SWEEP)
    nb = args.warmup + args.steps
    batches = []
    for s in range(nb):
        specs = ragged_specs(B, seed=EVAL_SEED0 + s, grids=grids, horizons=horizons)
        cls = [keys.index((g, h)) for g, h, _ in specs]
        inst = [make_instance(classes[c], sd) for c, (_, _, sd) in zip(cls, specs)]
        x0 = torch.cat([torch.tensor(x, device=dev) for x, _ in inst])
        xr = torch.cat([torch.tensor(r, device=dev) for _, r in inst])
        batches.append((cls, x0, xr, inst))
    waves = solver.autotune(batches[0][0], batches[0][1], batches[0][2], iters=4)

    def run(bs):
        ts, its, worst = [], [], 0
        torch.cuda.synchronize()
        for cls, x0, xr, _ in bs:
            t = time.perf_counter()
            rc, _, infos, _ = solver.solve(cls, x0, xr)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            its.append(infos["iters"].tolist())
            worst = max(worst, rc)
        return ts, its, worst

    run(batches[:args.warmup])
    solver.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, its, worst = run(batches[args.warmup:])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = solver.timing_read()
    solver.timing_enable(False)
    if args.copy_calibration:
        copy_calibration(dev)
    # algorithmic bytes per unit, weighted over the instances' stage-iterations
    wsum = bsum = esum = ewsum = 0.0
    for (cls, _, _, _), it in zip(batches[args.warmup:], its):
        for c, k in zip(cls, it):
            P = classes[c]
            w = float(k + 1) * P.N
            wsum += w
            bsum += w * bytes_per_unit(P.n, P.m, P.N)
            ewsum += P.N
            esum += P.N * eval_bytes_per_unit(P.n, P.m, P.N)
    roof = roofline("ragged", tm, bsum / wsum, esum / ewsum)
    allit = np.concatenate([np.asarray(i) for i in its])
    cfg = {"workload": "512 independent 2D heat instances per step, grids {32,48,64,96}^2 and "
                       "horizons {20,40,60} drawn uniformly, 4x4 Gaussian lattice, cold start, "
                       "Jacobi upper layer, ragged kernel (LPT-balanced over 8 XCDs, hipGraph "
                       "captured, autotuned waves), tol 1e-6",
           "global_batch": B, "waves": waves,
           "iters_min": int(allit.min()), "iters_max": int(allit.max()),
           "iters_mean": round(float(allit.mean()), 1), "status_worst": worst,
           "step_ms_median": round(1e3 * float(np.median(times)), 2)}
    cpu = None
    if args.cpu_budget > 0:
        oracle = oracle_native()
        cls, _, _, inst = batches[args.warmup]
        t = time.perf_counter()
        done, grids = 0, {}
        for c, (x0, xr) in zip(cls, inst):
            oracle.solve(classes[c], x0, xr, tol=1e-6, max_iter=5000)
            done += 1
            grids[classes[c].nsx] = grids.get(classes[c].nsx, 0) + 1
            if time.perf_counter() - t >= args.cpu_budget:
                break
        dt = time.perf_counter() - t
        mix = ", ".join(f"{k}x{k}: {v}" for k, v in sorted(grids.items()))
        cpu = {"value": done / dt, "unit": "solves/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"the first {done} instances of the first timed batch ({mix}; horizons "
                         f"as drawn), cold start, Jacobi, tol 1e-6, {dt:.1f} s"}
    line("NMPC solves/s to KKT res 1e-6, 512 ragged instances (mixed grids and horizons)",
         B * args.steps / elapsed, args, elapsed, "f32 sweeps, f64 state/residual", cfg, roof, cpu)
    solver.close()


def bench_model(args):
    """The model engine's workloads: the paper's copper plate (13 x 13 Neumann
    grid, 16 actuator nodes as inputs, box [T_a, T_a + 400] with tau = 100,
    gamma = 0.5, N = 20, T = 100 s, SGS upper layer, two sweeps and two Schur
    steps, stop at |K|_inf < 1) or the second-order damped membrane (24 x 24,
    N = 30, 4 x 4 Gaussian actuators, Jacobi upper layer, r_scaled <= 1e-6).
    One step = one batch of instances with their own seeded references
    (plate) or initial states and references (wave), one workgroup per
    instance. For the plate the paper's own scenario is also timed: one
    instance, closed loop of 200 steps of 5 s from the ambient temperature,
    reference a slope for 500 s and a V shape after, each step warm-started
    from the previous solution shifted by one stage (nominal loop: the next
    initial state is the solution's first state)."""
    import torch
    import paper_2004_02484_amd as nm
    from nmpc_inputs import (make_plate_instance, make_plate_problem, make_wave_instance,
                             make_wave_problem)
    dev = torch.device("cuda:0")
    plate = args.workload == "plate"
    P = make_plate_problem() if plate else make_wave_problem()
    inst = make_plate_instance if plate else make_wave_instance
    B = args.batch
    # both models default to SGS, the paper's upper layer (the membrane from a
    # cold start: 26.5 SGS iterations against 345 Jacobi ones); --upper
    # jacobi|fgs|bgs|sgs given explicitly overrides it
    upper = UPPER[args.upper if args.upper_given else "sgs"]
    opts = dict(tol=1.0, residual=nm.NMPC_RES_PAPER) if plate else dict(tol=1e-6)
    solver = nm.ModelSolver(P, max_batch=B, max_iter=5000, upper=upper, **opts)
    nb = args.warmup + args.steps
    host = []
    for s in range(nb):
        xs, rs = zip(*(inst(P, EVAL_SEED0 + s * B + b) for b in range(B)))
        host.append((np.stack(xs), np.stack(rs)))
    dev_in = [(torch.tensor(x, device=dev), torch.tensor(r, device=dev)) for x, r in host]

    def run(batches):
        ts, its, worst = [], [], 0
        torch.cuda.synchronize()
        for x0, xr in batches:
            t = time.perf_counter()
            rc, X, U, L, infos = solver.solve_batch(x0, xr)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            its += infos["iters"].tolist()
            worst = max(worst, rc)
        return ts, its, worst

    run(dev_in[:args.warmup])
    solver.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, iters, worst = run(dev_in[args.warmup:])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = solver.timing_read()
    solver.timing_enable(False)
    # algorithmic bytes of one stage visit: read s_i, write its new value, the
    # neighbours' x_{i-1}, lambda_{i+1} and the reference once per stage
    nx = 2 * P.nodes if P.model == "wave" else P.nodes
    bpu = 8.0 * (2 * (2 * nx + P.m) + 2 * nx + P.nodes)
    roof = roofline_model(tm, bpu)
    uname = [k for k, v in UPPER.items() if v == upper][0]
    cfg = {"global_batch": B, "grid": f"{P.nsx}x{P.nsy}", "horizon": P.N, "upper": uname,
           "iters_min": int(min(iters)), "iters_max": int(max(iters)),
           "iters_mean": round(float(np.mean(iters)), 1), "status_worst": worst,
           "step_ms_median": round(1e3 * float(np.median(times)), 2)}
    if plate:
        cfg["workload"] = ("copper plate of the paper's experiment: 13x13 nodes, zero Neumann "
                           "boundary, 16 actuator nodes as inputs boxed to [T_a, T_a+400] (tau "
                           "100), gamma 0.5, Q = I, R = 0.1 I, N = 20, T = 100 s, SGS upper "
                           "layer, 2 Jacobi sweeps + 2 Schur steps, stop at |K|_inf < 1; batch "
                           "of seeded slope / V references, cold start")
        cfg["paper_scenario"] = plate_closed_loop(nm, P, dev)
    else:
        cfg["workload"] = ("second-order-in-time damped nonlinear membrane 24x24 interior nodes "
                           "(W_tt + 2 W_t = (1 + 0.5 W) Lap W + B u, state (W, W_t)), 4x4 "
                           f"Gaussian actuators, N = 30, {uname.upper()} upper layer, the v6 "
                           "elimination of the lower layer, r_scaled <= 1e-6, cold start")
    cpu = None
    if args.cpu_budget > 0:
        import oracle.models as om
        ops = om.Ops(P)
        x0s, xrs = host[args.warmup]
        name = uname
        t = time.perf_counter()
        if plate:
            done, its = 0, []
            while done < B and (time.perf_counter() - t < args.cpu_budget or done == 0):
                o = om.solve(ops, om.state_x0(ops, x0s[done]), xrs[done], upper=name,
                             tol=opts["tol"], residual_kind="paper", max_iter=5000)
                its.append(o["iters"])
                done += 1
            dt = time.perf_counter() - t
            value = done / dt
            sample = (f"the first {done} instances of the first timed batch solved by the numpy "
                      f"oracle ({name}, {min(its)}..{max(its)} iterations), {dt:.1f} s")
        else:
            S = om.cold_start(ops, om.state_x0(ops, x0s[0]))
            k = 0
            while time.perf_counter() - t < args.cpu_budget or k == 0:
                S = om.iterate(ops, om.state_x0(ops, x0s[0]), xrs[0], S, name)
                k += 1
            per_it = (time.perf_counter() - t) / k
            it = float(np.mean(iters))
            value = 1.0 / (per_it * it)
            sample = (f"{k} cold-start {name} iterations of the first timed instance by the numpy "
                      f"oracle ({per_it:.2f} s each), scaled by the GPU's mean {it:.0f} "
                      f"iterations per solve")
        cpu = {"value": value, "unit": "solves/s", "cores": 1, "kind": "oracle", "sample": sample}
    line(f"NMPC solves/s, {'copper plate 13x13 N=20 (|K|_inf < 1)' if plate else 'damped membrane 24x24 N=30 (r_scaled <= 1e-6)'}",
         B * args.steps / elapsed, args, elapsed, "f64", cfg, roof, cpu)
    solver.close()


def roofline_model(tm, bpu: float):
    """HBM roofline of the model engine's persistent kernel: algorithmic bytes
    per stage visit times the visits of a launch, over the launch time."""
    avg_launch_s = tm["kernel_ms"] * 1e-3 / max(tm["launches"], 1)
    units_per_launch = tm["units"] / max(tm["launches"], 1)
    achieved = bpu * units_per_launch / avg_launch_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_model (persistent, one workgroup per instance)",
            "avg_launch_us": round(avg_launch_s * 1e6, 1),
            "units_per_launch": round(units_per_launch, 1), "bytes_per_unit": round(bpu, 1)}


def plate_closed_loop(nm, P, dev, steps: int = 200):
    """The paper's closed loop (Sec. 5): 1000 s at 5 s sampling from the
    ambient temperature; the reference is a slope for the first 500 s and a V
    shape after it, fed in over 50 s. Each step starts from the previous
    solution shifted by one stage (the last stage repeated) and solves to
    |K|_inf < 1 with SGS; the plant is the model (the next initial state is
    the solution's first stage)."""
    import torch
    from nmpc_inputs import plate_reference
    rng = np.random.default_rng(2020)
    ref1 = plate_reference(P, "slope", rng)
    ref2 = plate_reference(P, "v", rng)
    s = nm.ModelSolver(P, max_batch=1, tol=1.0, residual=nm.NMPC_RES_PAPER, max_iter=5000,
                       upper=UPPER["sgs"])
    s.timing_enable(True)
    x = torch.full((1, P.nodes), P.t_amb, dtype=torch.float64, device=dev)
    warm = None
    its, ts = [], []
    for k in range(steps):
        t_now = 5.0 * k
        w = min(max((t_now - 500.0) / 50.0, 0.0), 1.0)
        xr = torch.tensor(((1 - w) * ref1 + w * ref2)[None], device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, X, U, L, infos = s.solve_batch(x, xr, warm=warm)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
        its.append(int(infos[0]["iters"]))
        x = X[:, 0].clone()
        warm = (torch.cat([X[:, 1:], X[:, -1:]], 1).contiguous(),
                torch.cat([U[:, 1:], U[:, -1:]], 1).contiguous(),
                torch.cat([L[:, 1:], L[:, -1:]], 1).contiguous())
    tm = s.timing_read()
    s.close()
    kernel_ms = tm["kernel_ms"]
    return {"steps": steps, "iters_mean": round(float(np.mean(its)), 2), "iters_max": int(max(its)),
            "ms_per_iteration_kernel": round(kernel_ms / max(sum(its), 1), 4),
            "ms_per_step_median_wall": round(1e3 * float(np.median(ts)), 3),
            "paper_ms_per_iteration": {"value": 0.416, "hardware": "Intel Core i5-8265U laptop, "
                                       "one core, C implementation", "note": "context only"},
            "note": "single instance, one workgroup: latency-bound; iterations count SGS "
                    "iterations (a backward and a forward sweep each)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "plate", "wave"], default="c1",
                    help="c1: 64x64 N=40 batch 256 (headline); c2: 256x256 N=100 single "
                         "instance; c3: 512 ragged instances; plate: the paper's copper plate "
                         "(batch and closed loop); wave: second-order damped membrane")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--upper", choices=list(UPPER), default="jacobi",
                    help="upper-layer splitting: Jacobi (every stage in parallel; the default "
                         "of c1, c2, c3), or the Gauss-Seidel sweeps SGS (the default of plate "
                         "and wave, as in the paper's experiment), FGS, BGS")
    ap.add_argument("--n-sweep", type=int, default=2,
                    help="point-Jacobi sweeps per lower-layer solve (the paper's 2)")
    ap.add_argument("--n-schur", type=int, default=2,
                    help="Schur input iterations of the lower layer (the paper's 2)")
    ap.add_argument("--fp32-finish", type=int, choices=[0, 1], default=0,
                    help="FP32 sweeps: 0 (default) ends with the final FP64 correction step; "
                         "1 returns the iterate whose FP64-evaluated test passed in the FP32 "
                         "phase (same test, same tolerance, no FP64 step)")
    ap.add_argument("--warm-sweeps", type=int, default=10,
                    help="sweeps per stage (point-Jacobi, Chebyshev weights) when the library "
                         "builds the learned start's states")
    ap.add_argument("--warm-sweeps-lambda", type=int, default=14,
                    help="the same for the learned start's costates")
    ap.add_argument("--start", choices=["learned", "cold"], default="learned",
                    help="start timed for the value (the other one is reported beside it)")
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--mlp", type=int, choices=[0, 1], default=0,
                    help="1: the network's hidden path adds to the per-actuator linear map; "
                         "0: the linear map alone (network built with hidden = 0)")
    ap.add_argument("--closed-loop-steps", type=int, default=10,
                    help="closed loop per instance of the first timed batch after the timed "
                         "region: cold vs shifted vs learned starts at steps 2.. (0 disables)")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0 disables)")
    ap.add_argument("--fp64-variant", type=int, choices=[0, 1], default=1,
                    help="also time the FP64-sweep variant (learned and plain start) on the "
                         "same batches")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for counter scaling)")
    args = ap.parse_args()
    args.upper_given = any(a == "--upper" or a.startswith("--upper=") for a in sys.argv[1:])
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_2004_02484_amd as nm
    from nmpc_inputs import make_batch, make_problem

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "c2":
        return bench_c2(args)
    if args.workload == "c3":
        return bench_c3(args)
    if args.workload in ("plate", "wave"):
        return bench_model(args)
    P = make_problem("c1")
    B = args.batch
    prec = nm.NMPC_FP32_SWEEP if args.precision == "fp32" else nm.NMPC_FP64
    # warm_sweeps / warm_sweeps_lambda: Chebyshev-weighted point-Jacobi sweeps
    # per stage when the library builds the states / the costates from the
    # predicted inputs. On this grid and step the states keep the iteration
    # counts down to 8 sweeps (6 cost three times the iterations), the
    # costates down to 12 (10 cost half again as many): 10 and 14 keep a margin
    inner = dict(n_sweep=args.n_sweep, n_schur=args.n_schur)
    fin = args.fp32_finish if prec == nm.NMPC_FP32_SWEEP else 0
    solver = nm.Solver(P, max_batch=B, precision=prec, tol=1e-6, max_iter=5000,
                       check_every=16, fallback=1, upper=UPPER[args.upper],
                       warm_sweeps=args.warm_sweeps, warm_sweeps_lambda=args.warm_sweeps_lambda,
                       fp32_finish=fin, **inner)
    kind = "jacobi" if args.upper == "jacobi" else "gs"
    net = None
    if args.start == "learned":
        if not os.path.exists(args.weights):
            raise SystemExit(f"{args.weights}: no trained network; run "
                             f"python -m paper_2004_02484_amd.train_warmstart --out {args.weights}")
        from paper_2004_02484_amd.warmstart import PatchNet
        net = PatchNet.load(args.weights, device="cuda", mlp=bool(args.mlp))

    nb = args.warmup + args.steps
    host = [make_batch(P, range(EVAL_SEED0 + s * B, EVAL_SEED0 + (s + 1) * B)) for s in range(nb)]
    dev_in = [(torch.tensor(x, device=dev), torch.tensor(r, device=dev)) for x, r in host]
    out = (torch.empty((B, P.N, P.n), dtype=torch.float64, device=dev),
           torch.empty((B, P.N, P.m), dtype=torch.float64, device=dev),
           torch.empty((B, P.N, P.n), dtype=torch.float64, device=dev))
    ubuf = torch.empty((B, P.N, P.m), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    # warmup: graphs, network buffers, both starts; the timed kind last, so
    # the handle enters the timed region as in steady operation (its first
    # graph is sized from the previous solve of the same kind)
    if net is not None:
        timed_steps(solver, dev_in[:args.warmup], out)
    timed_steps(solver, dev_in[:args.warmup], out, net, ubuf)

    # timed region: exactly K steps with the selected start
    solver.timing_enable(True)
    errs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, iters, used, worst = timed_steps(solver, dev_in[args.warmup:], out, net, ubuf, errs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tm = solver.timing_read()
    solver.timing_enable(False)

    if args.copy_calibration:
        copy_calibration(dev)

    solves = B * args.steps
    value = solves / elapsed
    # one unit per stage sweep for every upper layer (an SGS iteration is two)
    roof = roofline(kind, tm, bytes_per_unit(P.n, P.m, P.N), eval_bytes_per_unit(P.n, P.m, P.N))

    start_desc = ("learned warm start (network" + (" with hidden path" if net.H else ": linear map on "
                  "second-order features") + " + rollout + adjoint, cold fallback)") \
        if net is not None else "cold start"
    cfg = {"workload": "2D nonlinear heat 64x64, N=40, 16 Gaussian inputs, batch 256, "
                       f"{start_desc}, {args.upper.upper()} upper layer, tol 1e-6",
           "global_batch": B, "grid": "64x64", "horizon": P.N, "start": args.start,
           "upper": args.upper, "n_sweep": args.n_sweep, "n_schur": args.n_schur,
           "fp32_finish": fin, "iters_min": int(min(iters)), "iters_max": int(max(iters)),
           "iters_mean": round(float(np.mean(iters)), 1), "status_worst": worst,
           "step_ms_median": round(1e3 * float(np.median(times)), 2),
           "step_ms_min": round(1e3 * min(times), 2)}
    if prec == nm.NMPC_FP32_SWEEP:
        e = np.asarray(errs)
        e = e[e >= 0]
        cfg["err_vs_fp64"] = {
            "per_result": "FP64 correction step from the FP32-phase iterate, max|du| / max|u| "
                          "(nmpc_info.err_vs_fp64)",
            "median": float(np.median(e)) if e.size else None,
            "max": float(e.max()) if e.size else None, "results": int(e.size)}
    if net is not None:
        # the plain (cold) start on the same batches, same solver settings
        ct, citers, _, cworst = timed_steps(solver, dev_in[args.warmup:], out)
        plain = solves / sum(ct)
        cfg.update({"starts_used": {k: int(v) for k, v in
                                    zip(("cold", "given", "from_inputs"),
                                        np.bincount(used, minlength=3))},
                    "plain_solves_per_s": round(plain, 2),
                    "plain_iters_mean": round(float(np.mean(citers)), 1),
                    "plain_iters_max": int(max(citers)),
                    "plain_status_worst": cworst,
                    "speedup_vs_plain": round(value / plain, 3)})
        # the plain start under every upper splitting (same batches): the
        # learned start against the fastest plain configuration
        best = (args.upper, plain)
        for up in UPPER:
            if up == args.upper or up in ("fgs", "bgs"):
                continue
            s2 = nm.Solver(P, max_batch=B, precision=prec, tol=1e-6, max_iter=5000,
                           check_every=16, fallback=1, upper=UPPER[up], fp32_finish=fin,
                           **inner)
            timed_steps(s2, dev_in[:1], out)
            t2, it2, _, w2 = timed_steps(s2, dev_in[args.warmup:], out)
            r2 = solves / sum(t2)
            cfg[f"plain_{up}_solves_per_s"] = round(r2, 2)
            cfg[f"plain_{up}_iters_mean"] = round(float(np.mean(it2)), 1)
            if r2 > best[1]:
                best = (up, r2)
            s2.close()
        cfg["speedup_vs_best_plain"] = {"upper": best[0], "value": round(value / best[1], 3)}
        # network rate on the matrix cores (inference only)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            net.predict(*dev_in[args.warmup], out=ubuf)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        fb, f32 = net_flops(net, B)
        tf = (fb + f32) / (ms * 1e-3) / 1e12
        pk = MFMA_BF16_PEAK_TFLOPS if net.H else MFMA_F32_PEAK_TFLOPS
        cfg["network"] = {"inference_ms": round(ms, 3), "params": net.num_params(),
                          "gflop": {"bf16_layers": round(fb / 1e9, 2), "fp32_map": round(f32 / 1e9, 2)},
                          "mfma": {"bound": "mfma", "achieved": round(tf, 2),
                                   "peak": pk, "unit": "TFLOP/s", "frac": round(tf / pk, 4),
                                   "note": "both parts over the bf16 peak" if net.H else
                                           "fp32 map over the fp32 matrix peak"},
                          "weights": os.path.relpath(args.weights, ROOT),
                          "hidden_path": bool(net.H),
                          "val_rel_err_median": net.meta.get(
                              "val_rel_err_median" if net.H else "linear_val_rel_err_median")}

    if net is not None and prec == nm.NMPC_FP32_SWEEP and args.fp64_variant:
        # the FP64-sweep variant of the same workload, learned and plain start
        # on the same batches (the FP32-sweep variant is the timed value)
        s64 = nm.Solver(P, max_batch=B, precision=nm.NMPC_FP64, tol=1e-6, max_iter=5000,
                        check_every=16, fallback=1, upper=UPPER[args.upper],
                        warm_sweeps=args.warm_sweeps, warm_sweeps_lambda=args.warm_sweeps_lambda,
                        **inner)
        timed_steps(s64, dev_in[:1], out)
        timed_steps(s64, dev_in[:1], out, net, ubuf)
        t64, it64, _, w64 = timed_steps(s64, dev_in[args.warmup:], out, net, ubuf)
        p64, pit64, _, pw64 = timed_steps(s64, dev_in[args.warmup:], out)
        cfg["fp64_variant"] = {
            "solves_per_s": round(solves / sum(t64), 2),
            "iters_mean": round(float(np.mean(it64)), 1), "iters_max": int(max(it64)),
            "status_worst": w64,
            "plain_solves_per_s": round(solves / sum(p64), 2),
            "plain_iters_mean": round(float(np.mean(pit64)), 1), "plain_status_worst": pw64,
            "speedup_vs_plain": round(sum(p64) / sum(t64), 3),
            "note": "all sweeps FP64, learned start, same batches as the timed value"}
        s64.close()

    u_pred = None
    if net is not None and args.cpu_budget > 0:
        x0f, xrf = dev_in[args.warmup]
        u_pred = net.predict(x0f, xrf, out=ubuf).cpu().numpy()
        # control error of sampled results of the timed configuration against
        # the oracle's exact solution (r_scaled <= 1e-12)
        rc, X, U, L, infos = solver.solve_batch(x0f, xrf, warm=(None, ubuf, None), out=out)
        Uh = U.cpu().numpy()
        oracle = oracle_native()
        smp = {}
        for b in (0, B // 2, B - 1):
            ex = oracle.solve(P, host[args.warmup][0][b], host[args.warmup][1][b], tol=1e-12,
                              max_iter=20000)
            smp[str(b)] = {"control_rel_err_vs_oracle_exact":
                           float(np.abs(Uh[b] - ex["U"]).max() / np.abs(ex["U"]).max()),
                           "err_vs_fp64": float(infos[b]["err_vs_fp64"]),
                           "iters": int(infos[b]["iters"])}
        cfg["sampled_vs_oracle"] = {"instances_of_first_timed_batch": smp,
                                    "bar": 1e-4 if prec == nm.NMPC_FP32_SWEEP else 1e-6}

    if net is not None and args.closed_loop_steps >= 2:
        cfg["closed_loop"] = dict(
            closed_loop(solver, net, P, *dev_in[args.warmup], args.closed_loop_steps, ubuf),
            steps=f"2..{args.closed_loop_steps}", plant="explicit Euler, dt = h",
            instances=B)

    result = {
        "metric": "NMPC solves/s to KKT res 1e-6, 64x64 grid N=40: learned warm start vs plain",
        "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 sweeps, f64 state/residual" if prec == nm.NMPC_FP32_SWEEP else "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": roof,
    }
    if args.cpu_budget > 0:
        result["cpu_baseline"] = cpu_baseline(P, host[args.warmup][0], host[args.warmup][1],
                                              args.cpu_budget, args.upper, u_pred)
    print(json.dumps(result), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
