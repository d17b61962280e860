#!/usr/bin/env python3
"""Benchmark of the APG solver for scenario-tree SMPC on one MI355X.

Default workload (`value`): the Barcelona-shaped plain method in float64 --
63 tanks, 114 flows, 88 demands, 17 junctions, horizon N = 24, branching 7 at
the first three stages (343 scenarios, 7260 decision nodes), log-normal
demands around a 24-periodic profile, cold start, tolerance 1e-3.  One step =
one solve to tolerance; `value` is APG iterations per second over the timed
steps (inputs resident in HBM; each solve uploads p and q, ~1.4 kB, and reads
back u0).

Further legs (one JSON line in all):
- batched: 64 trees of uneven size (horizons 12/18/24, 16..512 scenarios,
  ~260k nodes) in one batch with float32 solve steps on a float64 dual and
  20 float64 polish iterations, then the same 64 trees solved one at a time
  by the plain float64 solver;
  solves/s of both, per-tree u0 and cost differences and duality gaps, and
  the roofline of the float32 batch launch;
- table1_sweep: runtime against scenario count over the controllers of
  Table 1 (N = 24, 1..493 scenarios) in float64 and float32 + float64;
- closed_loop: 168 closed-loop steps (Alg. 2, 500 float64 iterations each)
  of the controllers CE-MPC..SMPC6 with the KPIs of Sec. V-B;
- serving: the closed loop of Alg. 2 for 256 controllers driven at a Poisson
  arrival rate for a fixed window, then drained;
- cpu_baseline: the float64 NumPy oracle on the host cores.

The roofline's `achieved` uses the algorithmic bytes of one APG iteration
(the dual iterates y^nu, y^(nu-1) read and y^(nu+1) written, beta, uhat, e
and pi read once: (3 (2 nx + nu) + nv + nu + nx + 1) values per node, with
nv = nu - ne the size of beta in the reduced variables).  `traffic` comes
from the rocprofv3 FETCH_SIZE / WRITE_SIZE summary committed under
profiles/; it is reported only while the kernel source still has the hash
recorded there (null otherwise).

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
PMC_SUMMARY = os.path.join(ROOT, "profiles", "apg_iteration_hbm_traffic_tree7260_batch64.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1604_01074_amd", "csrc", "smpc_kernels.hip")
METRIC = "APG iters/s + solves/s to tol 1e-3 (FP32 batched vs FP64 plain); p50/p99 latency"


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or
    None when the summary is absent or the kernel source has changed since."""
    import hashlib
    import re

    try:
        text = open(PMC_SUMMARY).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"kernel source sha256: ([0-9a-f]{64})", text)
    t = re.search(rf"traffic per launch {re.escape(kernel)}: (\d+) bytes", text)
    if not m or not t or m.group(1) != src:
        return None
    return int(t.group(1))


def algorithmic_bytes(nx: int, nu: int, ne: int, elem: int, dual_elem: int | None = None) -> int:
    """Bytes one APG iteration must move per node: y^nu, y^(nu-1) read and
    y^(nu+1) written (3 D, D = 2 nx + nu, in the dual's precision), beta
    (nv = nu - ne values in the reduced variables), uhat (nu), e (nx) and pi
    read once (in the solve step's precision)."""
    D = 2 * nx + nu
    return (dual_elem or elem) * 3 * D + elem * ((nu - ne) + nu + nx + 1)


def kernel_bytes(kernel: str, nx: int, nu: int, elem: int, dual_elem: int | None = None) -> int:
    """Bytes per node that one launch of the library's kernel reads and writes
    as implemented (each array it touches counted once): the backward half
    reads y^nu, y^(nu-1), beta, pi and the scaling and writes du; the forward
    half reads du, uhat, e, pi, the scaling, y^nu, y^(nu-1) and writes
    y^(nu+1)."""
    D = 2 * nx + nu
    de = dual_elem or elem
    bwd = de * 2 * D + elem * (nu + 1 + 3 + nu)
    fwd = elem * (2 * nu + nx + 1 + 3) + de * 3 * D
    if kernel.startswith("backward"):
        return bwd
    if kernel.startswith("forward"):
        return fwd
    if kernel.startswith("iter"):
        return bwd + fwd
    return 0


def roofline_entry(kernel: str, avg_ms: float, nodes: int, nx: int, nu: int, ne: int, elem: int, traffic,
                   dual_elem: int | None = None) -> dict:
    per = algorithmic_bytes(nx, nu, ne, elem, dual_elem)
    alg = per * nodes
    achieved = alg / (avg_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
           "avg_launch_us": round(avg_ms * 1e3, 2), "nodes_per_launch": nodes,
           "algorithmic_bytes_per_node": per, "bytes_per_launch": alg,
           "kernel_bytes_per_launch": kernel_bytes(kernel, nx, nu, elem, dual_elem) * nodes}
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / alg, 3)
    return out


def cpu_baseline(inst, seconds: float, precond_scale, lam) -> dict:
    """The float64 oracle on the host: iterations/s on the 7260-node tree with
    every BLAS thread, then with one."""
    import oracle as O

    try:
        from threadpoolctl import threadpool_info, threadpool_limits

        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        blas = sorted({p.get("internal_api", "?") for p in threadpool_info()})
    except Exception:
        threadpool_limits = None
        threads, blas = os.cpu_count() or 1, []
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)

    def rate(sec):
        t0 = time.perf_counter()
        O.apg(P, lam, 2, F, scale=precond_scale)
        per = (time.perf_counter() - t0) / 2
        iters = max(2, int(sec / max(per, 1e-6)))
        t0 = time.perf_counter()
        O.apg(P, lam, iters, F, scale=precond_scale)
        return iters, time.perf_counter() - t0

    iters, dt = rate(seconds)
    out = {"value": iters / dt, "unit": "APG iterations/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{iters} FP64 iterations of the 7260-node Barcelona-shaped tree (no stop test)",
           "seconds": round(dt, 2), "cpu_model": model, "blas": blas, "nproc": os.cpu_count()}
    if threadpool_limits is not None:
        with threadpool_limits(1):
            i1, d1 = rate(seconds / 3)
        out["one_thread"] = {"value": i1 / d1, "iterations": i1, "seconds": round(d1, 2)}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch-steps", type=int, default=1)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-batch64", action="store_true", help="skip the per-tree float64 solves of the batch trees")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the Table 1 runtime sweep")
    ap.add_argument("--max-iter", type=int, default=50000, help="iteration cap of the float64 solves")
    ap.add_argument("--batch-max-iter", type=int, default=30000, help="iteration cap of the batched solves")
    ap.add_argument("--only-batch", action="store_true", help="run only the batched legs (profiling aid)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate of the served loop, req/s")
    ap.add_argument("--serve-window", type=float, default=20.0, help="seconds of arrivals (0: skip serving)")
    ap.add_argument("--serve-drain", type=float, default=40.0, help="seconds allowed to drain after the window")
    ap.add_argument("--serve-controllers", type=int, default=256)
    ap.add_argument("--serve-max-iter", type=int, default=20000)
    ap.add_argument("--serve-max-active", type=int, default=64)
    ap.add_argument("--serve-warm", type=int, default=1, help="0: cold starts; 1: warm starts from the shifted resident dual")
    ap.add_argument("--only-serve", action="store_true", help="run only the served closed loop")
    ap.add_argument("--only-sweep", action="store_true", help="run only the Table 1 sweep")
    ap.add_argument("--closed-loop-hours", type=int, default=168,
                    help="closed-loop steps per controller for the KPIs (0: skip)")
    ap.add_argument("--closed-loop-iters", type=int, default=500, help="APG iterations per closed-loop step")
    ap.add_argument("--closed-loop-warm", type=int, default=0,
                    help="0: cold starts (Alg. 2); 1: warm starts from the shifted dual")
    ap.add_argument("--only-closed-loop", action="store_true", help="run only the closed-loop KPI leg")
    ap.add_argument("--chunk64", default="", metavar="BWD,FWD",
                    help="fixed float64 chunk lengths of the plain leg instead of tuning them (counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device a few times (scales HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X and has no multi-GPU path "
              "(trees would shard across GPUs whole, with no per-iteration exchange).", file=sys.stderr)
        return 2

    import torch

    import dwn_synth as ds
    from paper_1604_01074_amd import solver

    torch.cuda.set_device(0)
    if a.copy_calibration:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                          "launches": 5}), flush=True)
        return 0
    if a.only_serve or a.only_batch or a.only_sweep or a.only_closed_loop:
        ctx = solver.Context(0)
        out = {}
        if a.only_serve:
            out["serving"] = serving_leg(ctx, a.serve_controllers, a.serve_rate, a.serve_window, a.serve_drain,
                                         a.serve_max_iter, a.serve_max_active, a.serve_warm)
        if a.only_batch:
            out["batched"] = batched_leg(ctx, a.batch_steps, a.batch_max_iter, not a.no_batch64)
        if a.only_sweep:
            out["table1_sweep"] = table1_sweep(ctx, a.max_iter)
        if a.only_closed_loop:
            out["closed_loop"] = closed_loop_leg(ctx, a.closed_loop_hours, a.closed_loop_iters, bool(a.closed_loop_warm))
        print(json.dumps(out), flush=True)
        ctx.close()
        return 0
    inst = ds.barcelona_instance()
    nx, nu, ne = inst.sys["nx"], inst.sys["nu"], inst.sys["ne"]
    ctx = solver.Context(0)
    system, tree = solver.from_instance(ctx, inst, precond=2, power_iters=200)
    lam, S = tree.factor_info(with_scale=True)
    info = tree.info()
    # tune 1: the warm-up solve times every chunk-length pair on its first
    # blocks and the tree's plan keeps the fastest
    opts = dict(tol=1e-3, max_iter=a.max_iter, check_every=10, precision=64, want_x=False, want_y=False, tune=1)
    if a.chunk64:
        opts.update(tune=0, chunk64=tuple(int(v) for v in a.chunk64.split(",")))
    print(f"[bench] plain FP64: M={inst.M} chains={info['n_chains']} levels={info['n_levels']} lambda={lam:.4e}",
          file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        tree.solve(inst.p, inst.q, **opts)
    torch.cuda.synchronize()
    lat, iters, conv = [], [], []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s0 = time.perf_counter()
        r = tree.solve(inst.p, inst.q, **opts)
        lat.append(time.perf_counter() - s0)
        iters.append(r["iterations"])
        conv.append(r["status"] == 0)
        print(f"[bench] step {len(iters)}: {r['iterations']} it in {lat[-1]:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = sum(iters) / elapsed
    print(f"[bench] plain FP64: {a.steps} solves, {iters[0]} iterations each, {elapsed:.3f} s, "
          f"{value:.1f} it/s, status {r['status']} r_p {r['r_primal']:.3e}", file=sys.stderr, flush=True)
    ob = tree.objective()

    # same steps again with per-kernel HIP events for the roofline
    ctx.reset_stats()
    ctx.profiling(True)
    for k in range(a.steps):
        tree.solve(inst.p, inst.q, **opts)
        print(f"[bench] profiled step {k + 1}", file=sys.stderr, flush=True)
    stats = ctx.kernel_stats()
    ctx.profiling(False)
    dom = max(stats, key=lambda k: stats[k]["total_ms"])
    avg_ms = stats[dom]["total_ms"] / stats[dom]["launches"]
    # one launch covers every node of the tree once
    if dom.startswith("iter"):
        chunk = f"{r['chunk64'][0]},{r['chunk64'][1]}"
        traffic = measured_traffic(f"{dom} chunks {chunk}")
    else:
        chunk = str(r["chunk64"][0 if dom.startswith("backward") else 1])
        traffic = measured_traffic(f"{dom} chunk {chunk}")
    roofline = roofline_entry(dom, avg_ms, inst.M, nx, nu, ne, 8, traffic)
    roofline["chunk"] = chunk
    kernels = {k: {"launches": v["launches"], "avg_us": round(1e3 * v["total_ms"] / v["launches"], 2),
                   "share": round(v["total_ms"] / sum(x["total_ms"] for x in stats.values()), 3)}
               for k, v in stats.items()}

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "APG iterations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(1e3 * elapsed / a.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Barcelona-shaped plain method, FP64: nx=63 nu=114 nd=88 ne=17, N=24, "
                               "branching [7,7,7] (343 scenarios, 7260 nodes), tol 1e-3, cold start",
                   "nodes": inst.M, "tol": 1e-3, "check_every": 10,
                   "precond": "single-branch block diagonal to the power -1/4",
                   "chunks_fp64": list(r["chunk64"])},
        "solves_per_s": round(sum(conv) / elapsed, 3),
        "solves_reaching_tol": int(sum(conv)),
        "r_primal_at_exit": r["r_primal"],
        "iterations_per_solve": iters[0],
        "node_iterations_per_s": round(value * inst.M, 1),
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 3)},
        "objective_at_exit": {"cost": ob["cost"], "gap": ob["gap"],
                              "relative_gap": ob["gap"] / max(abs(ob["cost"]), 1e-12),
                              "dual_violation": ob["dual_violation"]},
        "roofline": roofline,
        "kernels": kernels,
    }

    if not a.no_batch:
        out["batched"] = batched_leg(ctx, a.batch_steps, a.batch_max_iter, not a.no_batch64)

    if not a.no_sweep:
        out["table1_sweep"] = table1_sweep(ctx, a.max_iter)

    if a.closed_loop_hours > 0:
        out["closed_loop"] = closed_loop_leg(ctx, a.closed_loop_hours, a.closed_loop_iters, bool(a.closed_loop_warm))

    if a.serve_window > 0:
        out["serving"] = serving_leg(ctx, a.serve_controllers, a.serve_rate, a.serve_window, a.serve_drain,
                                     a.serve_max_iter, a.serve_max_active, a.serve_warm)

    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, a.cpu_seconds, S, lam)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


def _rel_inf(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(float(np.max(np.abs(b))), 1e-12))


def batched_leg(ctx, steps: int, max_iter: int, with_fp64: bool) -> dict:
    """64 trees: the float32-bulk batch (timed), the roofline of its float32
    launch with every tree resident, then (with_fp64) the same trees solved
    one at a time by the plain float64 solver, with per-tree differences."""
    import torch

    import dwn_synth as ds

    insts = ds.batch_instances(64)
    system = ctx.system(insts[0].sys)
    trees = []
    t0 = time.perf_counter()
    for k, inst in enumerate(insts):
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=2, power_iters=100)
        trees.append(t)
        if k % 16 == 15:
            print(f"[bench] batch setup {k + 1}/{len(insts)}", file=sys.stderr, flush=True)
    setup_s = time.perf_counter() - t0
    nodes = sum(i.M for i in insts)
    # float32 solve steps on a float64 dual, 20 float64 polish iterations
    kw = dict(tol=1e-3, max_iter=max_iter, check_every=10, precision=32, polish_iters=20, dual64=True,
              want_x=False, want_y=False, tune=1)
    ps = [i.p for i in insts]
    qs = [i.q for i in insts]
    print(f"[bench] batch: {len(trees)} trees, {nodes} nodes, setup {setup_s:.1f} s", file=sys.stderr, flush=True)
    system.solve_batch(trees, ps, qs, **dict(kw, max_iter=200))  # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        code, res = system.solve_batch(trees, ps, qs, **kw)
        print(f"[bench] batch step {k + 1}: {time.perf_counter() - t0:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # objectives of the batch results (outside the timed region)
    obj32 = [t.objective() for t in trees]
    tree_iters = sum(r["iterations"] for r in res) * steps
    node_iters = sum(r["iterations"] * i.M for r, i in zip(res, insts)) * steps
    reached = sum(1 for r in res if r["status"] == 0)
    nx, nu, ne = insts[0].sys["nx"], insts[0].sys["nu"], insts[0].sys["ne"]
    out = {"trees": len(insts), "nodes": nodes,
           "fp32_bulk": {"solves_per_s": round(reached * steps / dt, 3),
                         "solves_per_s_note": "trees meeting the stop test per second of batch wall time",
                         "tree_iterations_per_s": round(tree_iters / dt, 1),
                         "node_iterations_per_s": round(node_iters / dt, 1),
                         "ms_per_batch": round(1e3 * dt / steps, 2),
                         "trees_reaching_tol": reached,
                         "iterations_max": max(r["iterations"] for r in res),
                         "iterations_median": float(np.median([r["iterations"] for r in res])),
                         "fp32_iterations_median": float(np.median([r["fp32_iterations"] for r in res])),
                         "status_worst": int(code),
                         "chunks_fp32": list(res[0]["chunk32"]), "chunks_fp64": list(res[0]["chunk64"]),
                         "dtype": "f32 solve steps on an f64 dual (extrapolation, prox, update in f64), "
                                  "20 f64 polish"},
           "max_iter": max_iter, "setup_s": round(setup_s, 2)}
    # roofline of the float32 launch with all 64 trees resident (fixed
    # iteration count, no stop test)
    ctx.reset_stats()
    ctx.profiling(True)
    _, rr = system.solve_batch(trees, ps, qs, tol=0.0, max_iter=60, check_every=10, precision=32, polish_iters=0,
                               dual64=True, want_x=False, want_y=False, tune=1)
    stats = ctx.kernel_stats()
    ctx.profiling(False)
    if "iter_mix" in stats:
        avg = stats["iter_mix"]["total_ms"] / stats["iter_mix"]["launches"]
        chunk = f"{rr[0]['chunk32'][0]},{rr[0]['chunk32'][1]}"
        out["fp32_bulk"]["roofline"] = roofline_entry("iter_mix", avg, nodes, nx, nu, ne, 4,
                                                      measured_traffic(f"iter_mix chunks {chunk}"), dual_elem=8)
        out["fp32_bulk"]["roofline"]["chunk"] = chunk
    if with_fp64:
        res64, t64 = [], 0.0
        kw64 = dict(tol=1e-3, max_iter=max_iter, check_every=10, precision=64, want_x=False, want_y=False, tune=1)
        trees[0].solve(ps[0], qs[0], **dict(kw64, max_iter=200))  # warm-up
        torch.cuda.synchronize()
        du0, dcost, gaps64 = [], [], []
        for k, t in enumerate(trees):
            s0 = time.perf_counter()
            r64 = t.solve(ps[k], qs[k], **kw64)
            torch.cuda.synchronize()
            t64 += time.perf_counter() - s0
            res64.append(r64)
            o64 = t.objective()
            du0.append(_rel_inf(res[k]["u0"], r64["u0"]))
            dcost.append(abs(obj32[k]["cost"] - o64["cost"]) / max(abs(o64["cost"]), 1e-12))
            gaps64.append(o64["gap"] / max(abs(o64["cost"]), 1e-12))
        reached64 = sum(1 for r in res64 if r["status"] == 0)
        out["fp64_plain_per_tree"] = {
            "solves_per_s": round(reached64 / t64, 3), "seconds": round(t64, 2), "trees_reaching_tol": reached64,
            "iterations_median": float(np.median([r["iterations"] for r in res64])),
            "tree_iterations_per_s": round(sum(r["iterations"] for r in res64) / t64, 1),
            "dtype": "f64", "note": "the same 64 trees, one smpc_solve each, tuned chunks"}
        out["fp32_over_fp64_solves_per_s"] = round(out["fp32_bulk"]["solves_per_s"] / max(reached64 / t64, 1e-12), 3)
        out["per_tree_vs_fp64"] = {
            "u0_rel_diff": {"median": float(np.median(du0)), "max": float(np.max(du0))},
            "cost_rel_diff": {"median": float(np.median(dcost)), "max": float(np.max(dcost))},
            "note": "batch result (float32 solve steps on a float64 dual + float64 polish) against the plain float64 "
                    "solve of the same tree; both stop at tol 1e-3, so the difference is bounded by the tolerance, "
                    "not float32"}
    rg32 = [o["gap"] / max(abs(o["cost"]), 1e-12) for o in obj32]
    out["fp32_bulk"]["relative_gap"] = {"median": float(np.median(rg32)), "max": float(np.max(rg32))}
    if with_fp64:
        out["fp64_plain_per_tree"]["relative_gap"] = {"median": float(np.median(gaps64)),
                                                      "max": float(np.max(gaps64))}
    system.close()
    ctx.systems.remove(system)
    return out


def table1_sweep(ctx, max_iter: int) -> list:
    """Runtime against scenario count: each Table 1 controller (Sec. V-B, N =
    24) on the Barcelona-shaped system, solved to tol 1e-3 in plain float64
    and with float32 solve steps on a float64 dual (tuned chunks, one
    untimed warm-up solve each)."""
    import torch

    import dwn_synth as ds

    rows = []
    sysd = None
    system = None
    for name in ds.TABLE1:
        inst = ds.table1_instance(name)
        if system is None:
            sysd = inst.sys
            system = ctx.system(sysd)
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=2, power_iters=200)
        row = {"controller": name, "scenarios": int(inst.tree["scenarios"]), "nodes": inst.M}
        for prec, kw in ((64, {}), (32, dict(polish_iters=20, dual64=True))):
            opts = dict(tol=1e-3, max_iter=max_iter, check_every=10, precision=prec, want_x=False, want_y=False,
                        tune=1, **kw)
            t.solve(inst.p, inst.q, **opts)  # warm-up and chunk tuning
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            r = t.solve(inst.p, inst.q, **opts)
            torch.cuda.synchronize()
            dt = time.perf_counter() - s0
            row[f"fp{prec}"] = {"seconds": round(dt, 4), "iterations": r["iterations"],
                                "us_per_iteration": round(1e6 * dt / max(r["iterations"], 1), 2),
                                "status": r["status"]}
        rows.append(row)
        print(f"[bench] table1 {name}: M={inst.M} fp64 {row['fp64']['seconds']} s fp32 {row['fp32']['seconds']} s",
              file=sys.stderr, flush=True)
        t.close()
        system.trees.remove(t)
    system.close()
    ctx.systems.remove(system)
    return rows


def closed_loop_leg(ctx, hours: int, iters: int, warm: bool,
                    names=("CE-MPC", "SMPC1", "SMPC2", "SMPC3", "SMPC4", "SMPC5", "SMPC6")) -> list:
    """Closed loop of Alg. 2 for ``hours`` steps per controller of the KPI
    table of Sec. V-B on the Barcelona-shaped system: every controller sees
    the same demand profile and the same realised demands
    (``dwn_synth.closed_loop_demands``).  Each step runs the device cost
    update, a fixed budget of ``iters`` float64 APG iterations (the
    termination rule of Sec. IV: a fixed count set by the sampling time,
    quality checked afterwards by the duality gap and ``||Hz - t||_inf``) and
    the plant step; cold starts as Alg. 2 states, or warm starts from the
    shifted dual.  The KPIs of Sec. V-B summarise the run."""
    import dwn_synth as ds
    from paper_1604_01074_amd import closed_loop

    rows = []
    for name in names:
        inst = ds.table1_instance(name)
        system = ctx.system(inst.sys)
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=2)
        steps = ds.closed_loop_demands(inst.sys, inst.tree, hours)
        t0 = time.perf_counter()
        r = closed_loop.run(t, inst.p, inst.q, steps, warm=warm, tol=0.0, max_iter=iters, precision=64, gap=True,
                            tune=1)
        wall = time.perf_counter() - t0
        rel_gap = np.abs(np.asarray(r["gap"])) / np.maximum(1.0, np.abs(np.asarray(r["cost"])))
        rows.append({"controller": name, "scenarios": int(inst.tree["scenarios"]), "nodes": inst.M, "hours": hours,
                     "iterations_per_step": iters, "start": "warm" if warm else "cold",
                     "kpi": {k: round(v, 4) for k, v in r["kpi"].items()},
                     "relative_gap": {"median": float(np.median(rel_gap)), "max": float(rel_gap.max())},
                     "hz_t_max": {"median": float(np.median(r["hz_t_max"])), "max": float(np.max(r["hz_t_max"]))},
                     "ms_per_step_median": round(1e3 * float(np.median(r["seconds"])), 2),
                     "seconds": round(wall, 2)})
        print(f"[bench] closed loop {name} ({rows[-1]['start']}): kpi {rows[-1]['kpi']} relative gap median "
              f"{rows[-1]['relative_gap']['median']:.2e} |Hz-t| median {rows[-1]['hz_t_max']['median']:.3g} "
              f"{wall:.1f} s", file=sys.stderr, flush=True)
        del steps
        system.close()
        ctx.systems.remove(system)
    return rows


def serving_leg(ctx, n_ctrl: int, rate: float, window_s: float, drain_s: float, max_iter: int, max_active: int,
                warm: int, seed: int = 2024) -> dict:
    """Served closed loop: ``n_ctrl`` controllers (tree sizes as in the batch)
    issue MPC steps at Poisson times (total offered rate ``rate``) for
    ``window_s`` seconds; a controller's next step waits for its previous
    control (at most one request each in flight), its plant advances by
    ``x+ = A x + B u0 + Gd d0`` (d0: the realised root demand, levels clipped
    to the box).  After the window no new request is issued and the loop
    drains for at most ``drain_s`` seconds.  Latency = queue + run time
    measured by the library."""
    import dwn_synth as ds

    insts = ds.serving_controllers(n_ctrl, seed)
    sysd = insts[0].sys
    system = ctx.system(sysd)
    t0 = time.perf_counter()
    trees = []
    for k, inst in enumerate(insts):
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=2, power_iters=100)
        trees.append(t)
        if k % 64 == 63:
            print(f"[bench] serving setup {k + 1}/{len(insts)}", file=sys.stderr, flush=True)
    setup_s = time.perf_counter() - t0
    nodes = sum(i.M for i in insts)
    A, B, Gd = (np.asarray(sysd[k]) for k in ("A", "B", "Gd"))
    lo, hi = np.asarray(sysd["xmin"]), np.asarray(sysd["xmax"])
    rng = np.random.default_rng([seed, 1])
    x = [i.p.copy() for i in insts]
    q = [i.q.copy() for i in insts]
    step = [0] * n_ctrl
    last_d = [None] * n_ctrl
    busy = [None] * n_ctrl
    nxt = list(rng.exponential(n_ctrl / rate, n_ctrl))  # each controller: Poisson at rate / n_ctrl
    srv = system.server(tol=1e-3, max_iter=max_iter, check_every=10, precision=32, polish_iters=20, dual64=True,
                        max_active=max_active, tune=1)
    done, lat, cold_it, warm_it, reached, submitted, peak = [], [], [], [], 0, 0, 0
    start = time.perf_counter()
    last_print = 0
    try:
        while True:
            now = time.perf_counter() - start
            if now < window_s:
                for c in range(n_ctrl):
                    if busy[c] is None and nxt[c] <= now:
                        d, a2 = ds.step_demands(insts[c], step[c], rng)
                        nroot = int(np.sum(np.asarray(insts[c].tree["parent"]) == 0))
                        w = 1 if (warm and step[c] > 0) else 0
                        busy[c] = srv.submit(trees[c], x[c], q[c], d=d, alpha2=a2, warm=w,
                                             realized=int(rng.integers(max(nroot, 1))) if nroot else -1)
                        last_d[c] = d
                        submitted += 1
            outstanding = sum(1 for b in busy if b is not None)
            peak = max(peak, outstanding)
            if now >= window_s and (outstanding == 0 or now >= window_s + drain_s):
                break
            for c in range(n_ctrl):
                if busy[c] is None:
                    continue
                r = srv.poll(busy[c], wait_ms=0)
                if r is None:
                    continue
                busy[c] = None
                done.append(r)
                lat.append(r["queue_ms"] + r["run_ms"])
                (warm_it if (warm and step[c] > 0) else cold_it).append(r["iterations"])
                reached += int(r["status"] == 0)
                u0 = r["u0"]
                x[c] = np.clip(A @ x[c] + B @ u0 + Gd @ last_d[c][0], lo, hi)
                q[c] = u0
                step[c] += 1
                nxt[c] = max(nxt[c], time.perf_counter() - start) + rng.exponential(n_ctrl / rate)
            time.sleep(0.0002)
            if len(done) >= last_print + 50:
                last_print = len(done)
                print(f"[bench] serving {len(done)} done, {outstanding} outstanding, t={now:.1f} s",
                      file=sys.stderr, flush=True)
    finally:
        wall = time.perf_counter() - start
        for c in range(n_ctrl):  # past the drain limit: withdraw what is left
            if busy[c] is not None:
                srv.cancel(busy[c])
        srv.close()
    system.close()
    ctx.systems.remove(system)
    return {"controllers": n_ctrl, "nodes": nodes, "offered_rate_per_s": rate, "arrival_window_s": window_s,
            "submitted": submitted, "completed": len(done), "unfinished_at_cutoff": submitted - len(done),
            "max_active": max_active, "wall_s": round(wall, 2), "solves_per_s": round(len(done) / wall, 3),
            "reached_tol_per_s": round(reached / wall, 3), "reached_tol": reached,
            "peak_outstanding": peak,
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2) if lat else None,
                           "p99": round(float(np.percentile(lat, 99)), 2) if lat else None},
            "iterations_cold_median": float(np.median(cold_it)) if cold_it else None,
            "iterations_warm_median": float(np.median(warm_it)) if warm_it else None,
            "warm_start": bool(warm), "setup_s": round(setup_s, 2),
            "dtype": "f32 solve steps on an f64 dual, 20 f64 polish"}


if __name__ == "__main__":
    sys.exit(main())
