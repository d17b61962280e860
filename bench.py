#!/usr/bin/env python3
"""Benchmark of the APG solver for scenario-tree SMPC on one MI355X.

Default workload: the Barcelona-shaped plain method in float64 -- 63 tanks,
114 flows, 88 demands, 17 junctions, horizon N = 24, branching 7 at the first
three stages (343 scenarios, 7260 decision nodes), log-normal demands around a
24-periodic profile, cold start, tolerance 1e-3.  One step = one solve to
tolerance; `value` is APG iterations per second over the timed steps (inputs
resident in HBM; each solve uploads p and the root term, ~1.4 kB, and reads
back u0).

A second leg solves 64 trees of uneven size (horizons 12/18/24, 16..512
scenarios, ~260k nodes) in one batch with the float32 bulk + float64 finish
recipe (float32 until the stop test or a stall at float32's accuracy floor,
then float64) and reports its solves/s to tolerance and iterations/s beside
the float64 number.

The roofline's `traffic` comes from the rocprofv3 FETCH_SIZE / WRITE_SIZE
summary committed under profiles/; it is reported only while the kernel
source still has the hash recorded there (null otherwise).

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
PMC_SUMMARY = os.path.join(ROOT, "profiles", "apg_iteration_f64_barcelona7260_hbm_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1604_01074_amd", "csrc", "smpc_kernels.hip")


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
METRIC = "APG iters/s + solves/s to tol 1e-3 (FP32 batched vs FP64 plain); p50/p99 latency"


def node_bytes(kernel: str, nx: int, nu: int, elem: int, scaled: bool) -> int:
    """Compulsory bytes per node of one kernel launch (each input read once,
    each output written once)."""
    D = 2 * nx + nu
    sc = 3 if scaled else 0
    if kernel.startswith("backward"):
        # y^nu, y^{nu-1}, beta, pi, scale -> du
        return elem * (2 * D + nu + 1 + sc + nu)
    if kernel.startswith("forward"):
        # du, uhat, e, pi, scale, y^nu, y^{nu-1} -> y^{nu+1}
        return elem * (2 * nu + nx + 1 + sc + 2 * D + D)
    if kernel.startswith("iter"):
        # fused launch: the forward rollout of one iteration and the backward
        # sweep of the next
        return node_bytes("backward", nx, nu, elem, scaled) + node_bytes("forward", nx, nu, elem, scaled)
    return 0


def iteration_bytes(nx: int, nu: int, elem: int, scaled: bool) -> int:
    """Minimum bytes one APG iteration must move per node: the dual iterates
    y^nu, y^{nu-1} read and y^{nu+1} written once, the node data beta, uhat,
    e, pi (and the scaling) read once."""
    D = 2 * nx + nu
    return elem * (3 * D + 2 * nu + nx + 1 + (3 if scaled else 0))


def cpu_baseline(inst, seconds: float, precond_scale, lam) -> dict:
    import oracle as O

    try:
        from threadpoolctl import threadpool_info

        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    t0 = time.perf_counter()
    O.apg(P, lam, 2, F, scale=precond_scale)
    per = (time.perf_counter() - t0) / 2
    iters = max(2, int(seconds / max(per, 1e-6)))
    t0 = time.perf_counter()
    O.apg(P, lam, iters, F, scale=precond_scale)
    dt = time.perf_counter() - t0
    return {"value": iters / dt, "unit": "APG iterations/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{iters} FP64 iterations of the 7260-node Barcelona-shaped tree (no stop test)",
            "seconds": dt}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch-steps", type=int, default=1)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--max-iter", type=int, default=50000, help="iteration cap of the float64 solves")
    ap.add_argument("--batch-max-iter", type=int, default=30000, help="iteration cap of the batched solves")
    ap.add_argument("--only-batch", action="store_true", help="run only the batched FP32 leg (profiling aid)")
    ap.add_argument("--serve-requests", type=int, default=100, help="requests of the served closed loop (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=2.0, help="Poisson arrival rate of the served loop, req/s")
    ap.add_argument("--serve-controllers", type=int, default=256)
    ap.add_argument("--serve-max-iter", type=int, default=20000)
    ap.add_argument("--serve-max-active", type=int, default=64)
    ap.add_argument("--only-serve", action="store_true", help="run only the served closed loop")
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
    if a.only_serve:
        ctx = solver.Context(0)
        print(json.dumps({"serving": serving_leg(ctx, a.serve_controllers, a.serve_requests, a.serve_rate,
                                                  a.serve_max_iter, a.serve_max_active)}), flush=True)
        ctx.close()
        return 0
    if a.only_batch:
        ctx = solver.Context(0)
        print(json.dumps({"batched_fp32": batched_leg(ctx, a.batch_steps, a.batch_max_iter)}), flush=True)
        ctx.close()
        return 0
    inst = ds.barcelona_instance()
    nx, nu = inst.sys["nx"], inst.sys["nu"]
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
    # one launch of either kernel covers every node of the tree once
    nodes_per_launch = inst.M
    per_node = node_bytes(dom, nx, nu, 8, True)
    achieved = per_node * nodes_per_launch / (avg_ms * 1e-3) / 1e9
    if dom.startswith("iter"):
        chunk = f"{r['chunk64'][0]},{r['chunk64'][1]}"
        traffic = measured_traffic(f"{dom} chunks {chunk}")
    else:
        chunk = r["chunk64"][0 if dom.startswith("backward") else 1]
        traffic = measured_traffic(f"{dom} chunk {chunk}")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom, "chunk": chunk,
                "avg_launch_us": round(avg_ms * 1e3, 2), "bytes_per_launch": per_node * nodes_per_launch}
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
        "iteration_bytes_per_node": iteration_bytes(nx, nu, 8, True),
        "achieved_iteration_GBs": round(iteration_bytes(nx, nu, 8, True) * inst.M * value / 1e9, 1),
        "roofline": roofline,
        "kernels": kernels,
    }

    if not a.no_batch:
        out["batched_fp32"] = batched_leg(ctx, a.batch_steps, a.batch_max_iter)

    if a.serve_requests > 0:
        out["serving"] = serving_leg(ctx, a.serve_controllers, a.serve_requests, a.serve_rate, a.serve_max_iter,
                                     a.serve_max_active)

    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, a.cpu_seconds, S, lam)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


def serving_leg(ctx, n_ctrl: int, n_req: int, rate: float, max_iter: int, max_active: int,
                seed: int = 2024) -> dict:
    """Served closed loop: ``n_ctrl`` controllers (tree sizes as in the batch)
    issue MPC steps at Poisson times (total rate ``rate``); a controller's
    next step waits for its previous control, its plant advances by
    ``x+ = A x + B u0 + Gd d0`` (d0: the realised root demand, levels clipped
    to the box) and it starts warm from its shifted resident dual along a
    random realised root child.  Latency = queue + run time measured by the
    library; solves/s = completed requests over the loop's wall time."""
    import dwn_synth as ds

    insts = ds.serving_controllers(n_ctrl, seed)
    sysd = insts[0].sys
    system = ctx.system(sysd)
    t0 = time.perf_counter()
    trees = []
    for k, inst in enumerate(insts):
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=2, power_iters=50)
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
    srv = system.server(tol=1e-3, max_iter=max_iter, check_every=10, precision=32, polish_iters=20,
                        max_active=max_active)
    done, lat, cold_it, warm_it, reached, submitted = [], [], [], [], 0, 0
    start = time.perf_counter()
    try:
        while len(done) < n_req:
            now = time.perf_counter() - start
            for c in range(n_ctrl):
                if busy[c] is None and nxt[c] <= now and submitted < n_req:
                    d, a2 = ds.step_demands(insts[c], step[c], rng)
                    nroot = int(np.sum(np.asarray(insts[c].tree["parent"]) == 0))
                    warm = 1 if step[c] > 0 else 0
                    busy[c] = srv.submit(trees[c], x[c], q[c], d=d, alpha2=a2, warm=warm,
                                         realized=int(rng.integers(max(nroot, 1))) if nroot else -1)
                    last_d[c] = d
                    submitted += 1
            for c in range(n_ctrl):
                if busy[c] is None:
                    continue
                r = srv.poll(busy[c], wait_ms=0)
                if r is None:
                    continue
                busy[c] = None
                done.append(r)
                lat.append(r["queue_ms"] + r["run_ms"])
                (warm_it if step[c] > 0 else cold_it).append(r["iterations"])
                reached += int(r["status"] == 0)
                u0 = r["u0"]
                x[c] = np.clip(A @ x[c] + B @ u0 + Gd @ last_d[c][0], lo, hi)
                q[c] = u0
                step[c] += 1
                nxt[c] = max(nxt[c], time.perf_counter() - start) + rng.exponential(n_ctrl / rate)
            time.sleep(0.0002)
            if len(done) and len(done) % 100 == 0 and len(done) != getattr(serving_leg, "_last", -1):
                serving_leg._last = len(done)
                print(f"[bench] serving {len(done)}/{n_req} done", file=sys.stderr, flush=True)
    finally:
        srv.close()
    wall = time.perf_counter() - start
    system.close()
    ctx.systems.remove(system)
    return {"controllers": n_ctrl, "nodes": nodes, "requests": len(done), "arrival_rate_per_s": rate,
            "max_active": max_active, "wall_s": round(wall, 2), "solves_per_s": round(len(done) / wall, 2),
            "reached_tol": reached,
            "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2), "p99": round(float(np.percentile(lat, 99)), 2)},
            "iterations_cold_median": float(np.median(cold_it)) if cold_it else None,
            "iterations_warm_median": float(np.median(warm_it)) if warm_it else None,
            "setup_s": round(setup_s, 2), "dtype": "f32 bulk, f64 finish after a stall, 20 f64 polish"}


def batched_leg(ctx, steps: int, max_iter: int) -> dict:
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
    kw = dict(tol=1e-3, max_iter=max_iter, check_every=10, precision=32, polish_iters=20, stall_checks=100,
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
    tree_iters = sum(r["iterations"] for r in res) * steps
    node_iters = sum(r["iterations"] * i.M for r, i in zip(res, insts)) * steps
    reached = sum(1 for r in res if r["status"] == 0)
    nx, nu = insts[0].sys["nx"], insts[0].sys["nu"]
    out = {"trees": len(insts), "nodes": nodes, "solves_per_s": round(reached * steps / dt, 3),
           "solves_per_s_note": "trees meeting the stop test per second of batch wall time",
           "tree_iterations_per_s": round(tree_iters / dt, 1),
           "node_iterations_per_s": round(node_iters / dt, 1),
           "ms_per_batch": round(1e3 * dt / steps, 2),
           "achieved_iteration_GBs_fp32": round(iteration_bytes(nx, nu, 4, True) * node_iters / dt / 1e9, 1),
           "iterations_max": max(r["iterations"] for r in res),
           "trees_reaching_tol": int(sum(1 for r in res if r["status"] == 0)),
           "iterations_median": float(np.median([r["iterations"] for r in res])),
           "fp32_iterations_median": float(np.median([r["fp32_iterations"] for r in res])),
           "max_iter": max_iter, "status_worst": int(code), "setup_s": round(setup_s, 2),
           "chunks_fp32": list(res[0]["chunk32"]), "chunks_fp64": list(res[0]["chunk64"]),
           "dtype": "f32 bulk, f64 finish after a float32 stall (100 checks), 20 f64 polish"}
    system.close()
    ctx.systems.remove(system)
    return out


if __name__ == "__main__":
    sys.exit(main())
