"""The fused APG iteration (one launch: the forward rollout of iteration nu
and the backward sweep of iteration nu + 1) against the two-launch
iteration: the same arithmetic in the same order, so the bits agree.  The
inner nodes' dual entries cross workgroups inside the fused launch; a stale
read there would show up as a difference."""

import numpy as np
import pytest

import dwn_synth as ds

pytestmark = pytest.mark.gpu

CASES = {
    "barcelona-small": lambda: ds.barcelona_instance(N=12, branching=(3, 2)),
    "deep-branching": lambda: ds.random_small_instance(6, nx=3, nu=5, nd=2, ne=2, N=12, branching=(2, 1, 2, 1, 3)),
    "wide": lambda: ds.random_small_instance(8, nx=70, nu=80, nd=3, ne=2, N=10, branching=(2, 1, 3)),
    "single-node": lambda: ds.random_small_instance(3, nx=3, nu=4, nd=2, ne=1, N=1, branching=()),
}


@pytest.fixture(scope="module")
def lib():
    from paper_1604_01074_amd import smpc, solver

    return smpc, solver


@pytest.fixture(scope="module")
def ctx(lib):
    _, solver = lib
    c = solver.Context(0)
    yield c
    c.close()


def _same(a, b):
    assert a["iterations"] == b["iterations"] and a["status"] == b["status"]
    assert a["fp32_iterations"] == b["fp32_iterations"]
    for k in ("u0", "x", "u", "y"):
        if k in a:
            assert np.array_equal(a[k], b[k]), k
    assert a["r_primal"] == b["r_primal"]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision,polish", [(64, 0), (32, 20)])
def test_fused_equals_two_launches(ctx, lib, name, precision, polish):
    S, solver = lib
    inst = CASES[name]()
    print(f"[fused] case={name} M={inst.M} precision={precision}", flush=True)
    system, tree = solver.from_instance(ctx, inst, precond=2, power_iters=60)
    try:
        for kw in (dict(tol=0.0, max_iter=97, check_every=10), dict(tol=1e-3, max_iter=2000, check_every=10)):
            kw.update(precision=precision, polish_iters=polish)
            two = tree.solve(inst.p, inst.q, unfused=True, **kw)
            one = tree.solve(inst.p, inst.q, **kw)
            _same(one, two)
            # a chunk pair other than the default, and a tuned solve
            other = {"chunk64" if precision == 64 else "chunk32": tuple(
                S.smpc_chunk_lengths(precision, w)[-1] for w in (0, 1))}
            _same(tree.solve(inst.p, inst.q, **other, **kw), two)
            _same(tree.solve(inst.p, inst.q, tune=1, **kw), two)
    finally:
        system.close()
        ctx.systems.remove(system)


def test_fused_batch_and_stall_continuation(ctx, lib):
    S, solver = lib
    insts = ds.batch_instances(4, first_seed=100)
    system = ctx.system(insts[0].sys)
    trees = []
    for inst in insts:
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=2, power_iters=60)
        trees.append(t)
    try:
        ps, qs = [i.p for i in insts], [i.q for i in insts]
        # a stall window short enough that some trees continue in float64
        kw = dict(tol=1e-3, max_iter=1500, check_every=10, precision=32, polish_iters=20, stall_checks=5)
        _, two = system.solve_batch(trees, ps, qs, unfused=True, **kw)
        _, one = system.solve_batch(trees, ps, qs, **kw)
        for a, b in zip(one, two):
            _same(a, b)
        alone = [t.solve(i.p, i.q, **kw) for t, i in zip(trees, insts)]
        for a, b in zip(one, alone):
            _same(a, b)
    finally:
        system.close()
        ctx.systems.remove(system)
