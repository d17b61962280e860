"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances.  The library computes the solve step in input space with the
projector P = L (L'Wu L)^{-1} L' and sparse B, the oracle in the reduced
variables with Lambda, Phi, Psi (App. B); both are exact up to rounding, so the
float64 results agree to a small multiple of machine precision times the
magnitude of the data (relative 1e-10 below is ~1e5 ulp, the sum of a few
hundred rounded terms over up to 24 stages).  Float32 parity uses 1e-4
relative (the float32 target), float32-with-float64-polish parity the same.
"""

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_1604_01074_amd import smpc, solver  # fails loudly if not built

    return smpc, solver


@pytest.fixture(scope="module")
def ctx(lib):
    _, solver = lib
    c = solver.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


STEP_CASES = {
    "tiny": lambda: ds.tiny_instance(),
    "random-A-ne2": lambda: ds.random_small_instance(0, nx=4, nu=5, nd=3, ne=2, N=3, branching=(2, 2)),
    "ragged": lambda: ds.random_small_instance(1, nx=3, nu=6, nd=2, ne=2, N=5, branching=(3, 2), scenarios=5),
    "single-node": lambda: ds.random_small_instance(3, nx=3, nu=4, nd=2, ne=1, N=1, branching=()),
    "one-scenario": lambda: ds.random_small_instance(4, nx=3, nu=4, nd=2, ne=2, N=7, branching=()),
    "long-inner-chains": lambda: ds.random_small_instance(6, nx=3, nu=5, nd=2, ne=2, N=7, branching=(2, 1, 1, 3)),
    "barcelona-small": lambda: ds.barcelona_instance(N=6, branching=(3, 2)),
    "barcelona-7260": lambda: ds.barcelona_instance(),
}


@pytest.mark.parametrize("name", list(STEP_CASES))
@pytest.mark.parametrize("precision", [64, 32])
def test_solve_step_parity(ctx, name, precision):
    inst = STEP_CASES[name]()
    print(f"[solve-step] case={name} M={inst.M} precision={precision}", flush=True)
    sysh, tree = None, None
    from paper_1604_01074_amd import solver

    system, tree = solver.from_instance(ctx, inst, lambda_override=1.0)
    try:
        P = O.OracleProblem.from_instance(inst)
        F = O.factor_step(P)
        rng = np.random.default_rng(7)
        for trial in range(2):
            w = rng.standard_normal((inst.M, P.dual_dim)) * (10.0 if trial else 1.0)
            xo, uo = O.solve_step(P, F, w)
            xg, ug = tree.solve_step(inst.p, inst.q, w, precision=precision)
            tol = 1e-10 if precision == 64 else 1e-4
            scale = max(1.0, np.abs(xo).max(), np.abs(uo).max())
            assert np.abs(xg - xo).max() <= tol * scale, (name, np.abs(xg - xo).max() / scale)
            assert np.abs(ug - uo).max() <= tol * scale, (name, np.abs(ug - uo).max() / scale)
    finally:
        system.close()
        ctx.systems.remove(system)


def _dense_lambda(inst, scale=None):
    P = O.OracleProblem.from_instance(inst)
    K = O.dual_hessian_dense(P, None, scale)
    return 1.0 / np.linalg.eigvalsh(0.5 * (K + K.T))[-1]


def test_power_iteration_step_size(ctx, lib):
    _, solver = lib
    inst = ds.tiny_instance()
    system, tree = solver.from_instance(ctx, inst, power_iters=500)
    try:
        lam = tree.factor_info()
        lam_dense = _dense_lambda(inst)
        # library uses lambda = 1 / (1.02 L)
        assert abs(1.0 / (lam * 1.02) - 1.0 / lam_dense) <= 1e-7 / lam_dense
    finally:
        system.close()
        ctx.systems.remove(system)


def test_single_branch_preconditioner_matches_dense_diagonal(ctx, lib):
    """precond=1 on a one-scenario tree: s_{n,b}^-2 equals the block mean of
    the dense dual Hessian diagonal (pi = 1 on a single branch)."""
    _, solver = lib
    inst = ds.random_small_instance(21, nx=3, nu=5, nd=2, ne=2, N=5, branching=())
    system, tree = solver.from_instance(ctx, inst, precond=1, power_iters=300)
    try:
        lam, S = tree.factor_info(with_scale=True)
        P = O.OracleProblem.from_instance(inst)
        K = O.dual_hessian_dense(P)
        dg = np.diag(K).reshape(inst.M, P.dual_dim)
        nx = P.nx
        means = np.stack([dg[:, :nx].mean(1), dg[:, nx:2 * nx].mean(1), dg[:, 2 * nx:].mean(1)], 1)
        assert np.allclose(1.0 / S ** 2, means, rtol=1e-10)
        # the library's step is the power-iteration estimate of the scaled operator
        lam_dense = _dense_lambda(inst, S)
        assert abs(1.0 / (lam * 1.02) - 1.0 / lam_dense) <= 1e-6 / lam_dense
    finally:
        system.close()
        ctx.systems.remove(system)


def _apg_pair(ctx, inst, iters, precision=64, polish=0, tol=0.0, check_every=10, precond=0, y0=None,
              power_iters=300):
    from paper_1604_01074_amd import solver

    system, tree = solver.from_instance(ctx, inst, precond=precond, power_iters=power_iters)
    lam, S = tree.factor_info(with_scale=True)
    g = tree.solve(inst.p, inst.q, tol=tol, max_iter=iters, check_every=check_every, precision=precision,
                   polish_iters=polish, y0=y0)
    P = O.OracleProblem.from_instance(inst)
    r = O.apg(P, lam, iters, tol=tol, check_every=check_every, scale=None if precond == 0 else S, y0=y0)
    system.close()
    ctx.systems.remove(system)
    return g, r, P


def test_apg_fp64_tiny_500(ctx):
    """Plain method, tiny tank network, 500 float64 iterations: u0 within
    1e-10 relative of the oracle at equal (lambda, S, y0)."""
    inst = ds.tiny_instance()
    g, r, P = _apg_pair(ctx, inst, 500)
    assert g["iterations"] == 500 and g["status"] == 1
    assert np.max(np.abs(g["u0"] - r.u0)) <= 1e-10 * max(np.max(np.abs(r.u0)), 1e-12)
    assert _rel(g["u"], r.u) <= 1e-10 and _rel(g["x"], r.x) <= 1e-10
    assert _rel(g["y"], r.y) <= 1e-10
    assert abs(g["r_primal"] - r.r_primal) <= 1e-9 * max(1.0, r.r_primal)


@pytest.mark.parametrize("seed,branching,scen", [(0, (3, 2), 5), (5, (3, 2), 5), (7, (2, 1, 1, 3), None)])
def test_apg_fp64_general_system_scaled(ctx, seed, branching, scen):
    inst = ds.random_small_instance(seed, nx=4, nu=6, nd=3, ne=2, N=6, branching=branching, scenarios=scen)
    g, r, P = _apg_pair(ctx, inst, 300, precond=1)
    assert _rel(g["u"], r.u) <= 1e-9 and _rel(g["x"], r.x) <= 1e-9 and _rel(g["y"], r.y) <= 1e-9


def test_apg_fp32_polish_tiny(ctx):
    """Precision variant of the tiny case: float32 for 480 iterations, then 20
    float64 polish iterations, against the float64 oracle after 500.

    u0 meets the 1e-4 relative target.  The cost of the iterate does not:
    after 500 iterations the iterate is far from optimal (r_p ~ 0.2) and its
    cost is ill-conditioned in the dual, whose entries reach the soft-penalty
    weights (up to 500) and map to the primal with gain L ~ 5e3.  Rounding
    only the stored dual iterates to float32 in an otherwise float64 run of the
    oracle already moves the cost by 7e-4, so the bound checked here is 2e-3
    (that storage effect with margin), not 1e-4."""
    inst = ds.tiny_instance()
    g, r, P = _apg_pair(ctx, inst, 500, precision=32, polish=20)
    assert g["iterations"] == 500 and g["fp32_iterations"] == 480
    err_u0 = np.max(np.abs(g["u0"] - r.u0)) / np.max(np.abs(r.u0))
    c_g = O.primal_cost(P, g["x"], g["u"])
    c_o = O.primal_cost(P, r.x, r.u)
    print(f"[fp32+polish] u0 rel err {err_u0:.3e}  cost rel err {abs(c_g - c_o) / abs(c_o):.3e}", flush=True)
    assert err_u0 <= 1e-4
    assert abs(c_g - c_o) <= 2e-3 * abs(c_o)


def test_fp32_stall_continues_in_fp64(ctx):
    """With a short stall window the float32 phase stops early (no new
    minimum of r_p for stall_checks checks), the tree continues in float64 and
    meets the stop test; with stall detection off the float32 phase runs its
    whole budget instead."""
    inst = ds.tiny_instance()
    s = ctx.system(inst.sys)
    try:
        t = s.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=0, power_iters=100)
        kw = dict(tol=2e-5, max_iter=20000, check_every=10, precision=32, polish_iters=20)
        r = t.solve(inst.p, inst.q, stall_checks=5, **kw)
        print(f"[stall] fp32 {r['fp32_iterations']} total {r['iterations']} r_p {r['r_primal']:.3e}", flush=True)
        assert r["status"] == 0
        assert 0 < r["fp32_iterations"] < r["iterations"] - 20
        assert r["r_primal"] <= 2e-5 * (1 + r["hz_t_max"])
        r64 = t.solve(inst.p, inst.q, tol=2e-5, max_iter=20000, check_every=10, precision=64)
        assert r64["status"] == 0
        # two iterates that both pass the stop test: close, not equal
        assert np.max(np.abs(r["u0"] - r64["u0"])) <= 1e-2 * max(1.0, np.max(np.abs(r64["u0"])))
        off = t.solve(inst.p, inst.q, stall_checks=-1, **dict(kw, tol=1e-9, max_iter=3000))
        assert off["status"] == 1 and off["fp32_iterations"] == 2980 and off["iterations"] == 3000
    finally:
        s.close()
        ctx.systems.remove(s)


def test_apg_tolerance_stop_matches_oracle(ctx):
    inst = ds.tiny_instance()
    g, r, P = _apg_pair(ctx, inst, 5000, tol=1e-3, check_every=10)
    assert g["status"] == 0 and r.converged
    assert g["iterations"] == r.iterations and g["iterations"] % 10 == 0
    assert g["r_primal"] <= 1e-3 * (1 + g["hz_t_max"])
    assert _rel(g["u"], r.u) <= 1e-10


def test_apg_warm_start(ctx):
    inst = ds.random_small_instance(2, nx=3, nu=5, nd=2, ne=1, N=4, branching=(2, 2))
    P = O.OracleProblem.from_instance(inst)
    y0 = np.random.default_rng(0).standard_normal((inst.M, P.dual_dim)) * 0.1
    g, r, _ = _apg_pair(ctx, inst, 120, y0=y0)
    assert _rel(g["y"], r.y) <= 1e-10 and _rel(g["u"], r.u) <= 1e-10


def test_apg_barcelona_full_size_fixed_iterations(ctx):
    """Barcelona-shaped tree at full size (7260 nodes, 343 scenarios, N = 24),
    40 float64 iterations, compared element by element with the oracle."""
    inst = ds.barcelona_instance()
    print(f"[barcelona] M={inst.M}", flush=True)
    g, r, P = _apg_pair(ctx, inst, 40, power_iters=100, precond=1)
    assert _rel(g["u"], r.u) <= 1e-9 and _rel(g["x"], r.x) <= 1e-9
    assert _rel(g["y"], r.y) <= 1e-9


def test_batch_equals_alone_bitwise(ctx, lib):
    _, solver = lib
    insts = ds.batch_instances(4, first_seed=100)
    system = ctx.system(insts[0].sys)
    trees = []
    for inst in insts:
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=1, power_iters=100)
        trees.append(t)
    try:
        for precision, polish in ((64, 0), (32, 10)):
            kw = dict(tol=1e-3, max_iter=400, check_every=10, precision=precision, polish_iters=polish)
            alone = [t.solve(i.p, i.q, **kw) for t, i in zip(trees, insts)]
            code, batch = system.solve_batch(trees, [i.p for i in insts], [i.q for i in insts], **kw)
            for a, b in zip(alone, batch):
                assert a["iterations"] == b["iterations"]
                assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["x"], b["x"])
                assert np.array_equal(a["y"], b["y"])
            # repeated solve is bitwise identical (deterministic reductions)
            again = trees[0].solve(insts[0].p, insts[0].q, **kw)
            assert np.array_equal(again["y"], alone[0]["y"])
    finally:
        system.close()
        ctx.systems.remove(system)


def test_full_batch_sampled_trees(ctx, lib):
    """The batched workload at full size (64 trees, 259 942 nodes) in the
    configuration the benchmark times (precond 2, tuned chunk pairs): sampled
    trees give the bits of their own solves in float64 and in float32 with a
    float64 polish, and the smallest and the largest match the oracle in
    float64."""
    _, solver = lib
    insts = ds.batch_instances(64)
    sizes = [i.M for i in insts]
    print(f"[batch64] nodes={sum(sizes)} smallest={min(sizes)} largest={max(sizes)}", flush=True)
    system = ctx.system(insts[0].sys)
    trees = []
    for inst in insts:
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=2, power_iters=100)
        trees.append(t)
    small, large = int(np.argmin(sizes)), int(np.argmax(sizes))
    sample = sorted({0, small, large, len(insts) - 1})
    ps, qs = [i.p for i in insts], [i.q for i in insts]
    try:
        for precision, polish, iters in ((64, 0, 40), (32, 20, 60)):
            kw = dict(tol=0.0, max_iter=iters, check_every=10, precision=precision, polish_iters=polish)
            print(f"[batch64] precision={precision} iterations={iters} sample={sample}", flush=True)
            _, batch = system.solve_batch(trees, ps, qs, tune=1, **kw)
            for k in sample:
                alone = trees[k].solve(ps[k], qs[k], **kw)
                assert alone["iterations"] == batch[k]["iterations"]
                for key in ("u", "x", "y"):
                    assert np.array_equal(alone[key], batch[k][key]), (k, key)
            if precision == 64:
                for k in (small, large):
                    print(f"[batch64] oracle tree={k} M={sizes[k]}", flush=True)
                    lam, S = trees[k].factor_info(with_scale=True)
                    r = O.apg(O.OracleProblem.from_instance(insts[k]), lam, iters, tol=0.0, check_every=10,
                              scale=S)
                    assert _rel(batch[k]["u"], r.u) <= 1e-9 and _rel(batch[k]["x"], r.x) <= 1e-9
                    assert _rel(batch[k]["y"], r.y) <= 1e-9
    finally:
        system.close()
        ctx.systems.remove(system)


def test_torch_stream_interop(ctx, lib):
    """The library runs on a torch side stream (one HIP runtime in the
    process) and gives the same bits as on its own stream."""
    import torch

    _, solver = lib
    inst = ds.tiny_instance()
    side = torch.cuda.Stream()
    c2 = solver.Context(0, stream=side.cuda_stream)
    try:
        _, t2 = solver.from_instance(c2, inst, lambda_override=1e-4)
        r2 = t2.solve(inst.p, inst.q, tol=0.0, max_iter=50)
    finally:
        c2.close()
    system, t1 = solver.from_instance(ctx, inst, lambda_override=1e-4)
    try:
        r1 = t1.solve(inst.p, inst.q, tol=0.0, max_iter=50)
    finally:
        system.close()
        ctx.systems.remove(system)
    assert np.array_equal(r1["y"], r2["y"]) and np.array_equal(r1["u"], r2["u"])


def test_graph_replay_equals_eager_launches(ctx, lib):
    """Solves replay captured iteration blocks (hipGraph); with profiling on
    the same iterations are launched one by one.  Both give the same bits,
    over many replays with host synchronisation between them."""
    _, solver = lib
    inst = ds.barcelona_instance(N=8, branching=(3, 2))
    system, tree = solver.from_instance(ctx, inst, precond=1, power_iters=50)
    try:
        for precision, polish in ((64, 0), (32, 5)):
            kw = dict(tol=0.0, max_iter=120, check_every=10, precision=precision, polish_iters=polish)
            g1 = tree.solve(inst.p, inst.q, **kw)
            ctx.profiling(True)
            e1 = tree.solve(inst.p, inst.q, **kw)
            ctx.profiling(False)
            g2 = tree.solve(inst.p, inst.q, **kw)
            for k in ("y", "u", "x"):
                assert np.array_equal(g1[k], e1[k]) and np.array_equal(g1[k], g2[k])
    finally:
        system.close()
        ctx.systems.remove(system)


def test_power_iteration_converged_on_a_barcelona_tree(ctx, lib):
    """The step size comes from a converged estimate: with the scaling the
    benchmark uses (precond 2) and a short minimum of 50 steps, the
    library's L lies within 0.1 % below the oracle's power iteration run for
    3 000 steps on the same scaled operator (the Rayleigh quotient approaches
    L from below, and the 2 % margin of the step covers what is left)."""
    _, solver = lib
    inst = ds.barcelona_instance(N=8, branching=(3, 2))
    system, tree = solver.from_instance(ctx, inst, precond=2, power_iters=50)
    try:
        lam, S = tree.factor_info(with_scale=True)
        L = 1.0 / (1.02 * lam)
        P = O.OracleProblem.from_instance(inst)
        L_ref = O.dual_lmax_power(P, 3000, scale=S)
        print(f"[power] library {L:.8e} oracle-3000 {L_ref:.8e}", flush=True)
        assert L <= L_ref * (1.0 + 1e-9)
        assert L >= L_ref * (1.0 - 1e-3)
    finally:
        system.close()
        ctx.systems.remove(system)
