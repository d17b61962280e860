"""Continuous-batching server: each request's result equals the direct
solve of the same tree and inputs bit for bit, alone or in the mix, cold or
warm-started from the shifted resident dual."""

import numpy as np
import pytest

import dwn_synth as ds

pytestmark = pytest.mark.gpu

KW = dict(tol=1e-3, max_iter=3000, check_every=10, precision=32, polish_iters=20)
SHAPES = [(6, (3, 2)), (8, (2, 2, 2)), (5, (4,)), (7, (3, 3)), (6, ())]


@pytest.fixture(scope="module")
def setup():
    from paper_1604_01074_amd import solver

    ctx = solver.Context(0)
    sysd = ds.barcelona_shaped_system(1)
    system = ctx.system(sysd)
    insts = [ds.barcelona_instance(N=N, branching=b, sys=sysd, demand_seed=10 + k) for k, (N, b) in enumerate(SHAPES)]
    trees = []
    for inst in insts:
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=1, power_iters=100)
        trees.append(t)
    yield system, insts, trees
    ctx.close()


def _same(a, b):
    assert a["status"] == b["status"]
    assert a["iterations"] == b["iterations"] and a["fp32_iterations"] == b["fp32_iterations"]
    assert np.array_equal(a["u0"], b["u0"])
    assert a["r_primal"] == b["r_primal"]


def test_server_results_equal_direct_solves(setup):
    system, insts, trees = setup
    ref = [t.solve(i.p, i.q, want_x=False, want_y=False, **KW) for t, i in zip(trees, insts)]
    srv = system.server(max_active=3, **KW)
    try:
        tickets = [srv.submit(t, i.p, i.q) for t, i in zip(trees, insts)]
        got = [srv.poll(tk) for tk in tickets]
    finally:
        srv.close()
    for a, b in zip(got, ref):
        _same(a, b)
        assert a["queue_ms"] >= 0.0 and a["run_ms"] > 0.0
    print("[serve] iterations", [g["iterations"] for g in got], flush=True)


def _steps(inst, k):
    rng = np.random.default_rng(100 + k)
    d = inst.d * np.exp(0.05 * rng.standard_normal(inst.d.shape))
    p = inst.p * (1.0 + 0.02 * rng.standard_normal(inst.p.shape))
    return d, p


def test_server_warm_sequences_equal_direct_calls(setup):
    system, insts, trees = setup
    chosen = [0, 1, 3]
    seq = {j: [_steps(insts[j], k) for k in range(3)] for j in chosen}
    ref = {}
    for j in chosen:
        t, inst = trees[j], insts[j]
        out = []
        for k, (d, p) in enumerate(seq[j]):
            t.set_data(d, inst.alpha2)
            if k == 0:
                out.append(t.solve(p, inst.q, want_x=False, want_y=False, **KW))
            else:
                t.shift_warm_start(1)
                out.append(t.solve(p, inst.q, want_x=False, want_y=False, resident=True, **KW))
        ref[j] = out
    srv = system.server(max_active=2, **KW)
    try:
        tickets = []
        for k in range(3):  # interleaved over the trees; each tree keeps its order
            for j in chosen:
                d, p = seq[j][k]
                tickets.append((j, k, srv.submit(trees[j], p, insts[j].q, d=d, alpha2=insts[j].alpha2,
                                                 warm=0 if k == 0 else 1, realized=1)))
        got = {(j, k): srv.poll(tk) for j, k, tk in tickets}
    finally:
        srv.close()
    for j in chosen:
        for k in range(3):
            _same(got[(j, k)], ref[j][k])
    warm_its = [got[(j, k)]["iterations"] for j in chosen for k in (1, 2)]
    cold_its = [got[(j, 0)]["iterations"] for j in chosen]
    print(f"[serve] cold {cold_its} warm {warm_its}", flush=True)


def test_server_errors(setup):
    from paper_1604_01074_amd import smpc, solver

    system, insts, trees = setup
    # trees are built before the server exists (afterwards they are used only
    # through it)
    fresh = system.tree(insts[4].tree)
    fresh.set_data(insts[4].d, insts[4].alpha2)
    fresh.factor(precond=1, power_iters=20)
    other = system.ctx.system(ds.tiny_tank_system(0))
    tiny = ds.tiny_instance()
    ot = other.tree(tiny.tree)
    srv = system.server(**KW)
    try:
        with pytest.raises(smpc.SmpcError) as e:
            srv.poll(12345, wait_ms=0)
        assert e.value.code == smpc.EINVAL
        with pytest.raises(smpc.SmpcError) as e:
            srv.submit(ot, tiny.p, tiny.q)  # a tree of another system
        assert e.value.code == smpc.EINVAL
        tk = srv.submit(fresh, insts[4].p, insts[4].q, warm=1, realized=0)  # nothing resident
        with pytest.raises(smpc.SmpcError) as e:
            srv.poll(tk)
        assert e.value.code == smpc.EINVAL
    finally:
        srv.close()


def test_server_cancel(setup):
    """A withdrawn request reports SMPC_ECANCELED, queued or running; the
    other requests are unaffected and equal their direct solves."""
    from paper_1604_01074_amd import smpc

    system, insts, trees = setup
    ref = trees[2].solve(insts[2].p, insts[2].q, want_x=False, want_y=False, **KW)
    srv = system.server(max_active=1, **KW)
    try:
        t0 = srv.submit(trees[0], insts[0].p, insts[0].q)    # runs first
        t1 = srv.submit(trees[1], insts[1].p, insts[1].q)    # queued behind it
        t2 = srv.submit(trees[2], insts[2].p, insts[2].q)
        srv.cancel(t1)
        srv.cancel(t0)
        r0, r1, r2 = srv.poll(t0), srv.poll(t1), srv.poll(t2)
    finally:
        srv.close()
    assert r1["status"] == smpc.ECANCELED
    # the first request was running (or had just finished) when canceled
    assert r0["status"] in (smpc.ECANCELED, smpc.OK, smpc.MAX_ITER)
    _same(r2, ref)


def test_server_waits_for_memory_then_admits(lib_free_ctx):
    """Back-pressure: with an HBM budget that holds the float32 buffers of
    one tree at a time, requests for three trees all complete -- each waits
    until the previous tree is idle and gives its float32 buffers up -- and
    each result equals the direct solve of the same tree bit for bit."""
    from paper_1604_01074_amd import solver

    sysd = ds.barcelona_shaped_system(1)
    shapes = [(6, (3, 2)), (8, (2, 2, 2)), (7, (3, 3))]
    insts = [ds.barcelona_instance(N=N, branching=b, sys=sysd, demand_seed=30 + k) for k, (N, b) in enumerate(shapes)]

    def build(ctx):
        system = ctx.system(sysd)
        trees = []
        for inst in insts:
            t = system.tree(inst.tree)
            t.set_data(inst.d, inst.alpha2)
            t.factor(precond=1, power_iters=100)
            trees.append(t)
        return system, trees

    # footprint without float32 buffers, and with each tree's; the probe's
    # solves are the references
    probe = solver.Context(0)
    system, trees = build(probe)
    base = probe.mem_used()
    used32, ref = [], []
    for t, inst in zip(trees, insts):
        before = probe.mem_used()
        ref.append(t.solve(inst.p, inst.q, want_x=False, want_y=False, **KW))
        used32.append(probe.mem_used() - before)
    probe.close()
    budget = base + max(used32) + min(used32) // 2  # one tree's float32 buffers at a time
    print(f"[serve-mem] base {base} float32 {used32} budget {budget}", flush=True)
    ctx = solver.Context(0, hbm_budget=budget)
    try:
        system, trees = build(ctx)
        srv = system.server(max_active=3, **KW)
        try:
            tickets = [srv.submit(t, i.p, i.q) for t, i in zip(trees, insts)]
            got = [srv.poll(tk) for tk in tickets]
        finally:
            srv.close()
        assert ctx.mem_used() <= budget
        for a, b in zip(got, ref):
            _same(a, b)
        # each later request waited for the one before it to finish
        for k in (1, 2):
            assert got[k]["queue_ms"] >= 0.5 * got[k - 1]["run_ms"], [(g["queue_ms"], g["run_ms"]) for g in got]
    finally:
        ctx.close()


@pytest.fixture
def lib_free_ctx():
    from paper_1604_01074_amd import solver  # noqa: F401  (fails loudly if not built)

    yield None
