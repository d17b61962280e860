"""Chunk lengths and the chunk-length autotuner.

A chunk length only decides how many nodes a kernel stages between two
barriers; the per-node recursions, the matrix-core product of a node's row
and the per-thread maxima keep their order.  So every built length must give
the same bits, and a tuned solve (whose first blocks run every pair in turn)
must give the bits of an untuned one."""

import itertools

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O

pytestmark = pytest.mark.gpu

CASES = {
    # chains of 36 and 39 nodes: several chunks of every length plus a ragged tail
    "long-chains": lambda: ds.random_small_instance(6, nx=3, nu=5, nd=2, ne=2, N=40, branching=(2, 1, 1, 3)),
    # nx > 64 and nu > 64: the two-row state and 128-wide input kernels
    "wide": lambda: ds.random_small_instance(8, nx=70, nu=80, nd=3, ne=2, N=20, branching=(2, 1, 3)),
    # the network's dimensions (nu > 64, identity A, sparse B)
    "barcelona-small": lambda: ds.barcelona_instance(N=12, branching=(3, 2)),
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


def _pairs(S, precision):
    return list(itertools.product(S.smpc_chunk_lengths(precision, 0), S.smpc_chunk_lengths(precision, 1)))


def _same(a, b):
    assert a["iterations"] == b["iterations"] and a["status"] == b["status"]
    for k in ("u0", "x", "u", "y"):
        assert np.array_equal(a[k], b[k]), k
    assert a["r_primal"] == b["r_primal"]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [64, 32])
def test_every_chunk_pair_gives_the_same_bits(ctx, lib, name, precision):
    S, solver = lib
    inst = CASES[name]()
    print(f"[chunks] case={name} M={inst.M} precision={precision}", flush=True)
    system, tree = solver.from_instance(ctx, inst, precond=1, power_iters=60)
    try:
        key = "chunk32" if precision == 32 else "chunk64"
        kw = dict(tol=0.0, max_iter=60, check_every=10, precision=precision, polish_iters=0)
        pairs = _pairs(S, precision)
        ref = tree.solve(inst.p, inst.q, **kw)
        assert ref[key] == pairs[0]  # the default pair
        for pair in pairs:
            print(f"[chunks]   pair={pair}", flush=True)
            got = tree.solve(inst.p, inst.q, **{key: pair}, **kw)
            assert got[key] == pair
            _same(got, ref)
        if precision == 64:
            # and the shared result is the oracle's
            lam, sc = tree.factor_info(with_scale=True)
            P = O.OracleProblem.from_instance(inst)
            r = O.apg(P, lam, 60, tol=0.0, check_every=10, scale=sc)
            scale = max(1.0, float(np.abs(r.y).max()))
            assert np.abs(ref["y"] - r.y).max() <= 1e-9 * scale
    finally:
        system.close()
        ctx.systems.remove(system)


def test_tuned_solve_equals_untuned_and_keeps_its_choice(ctx, lib):
    S, solver = lib
    inst = CASES["barcelona-small"]()
    system, tree = solver.from_instance(ctx, inst, precond=1, power_iters=60)
    try:
        # long enough for every pair to be timed in both precisions
        for precision in (64, 32):
            key = "chunk32" if precision == 32 else "chunk64"
            kw = dict(tol=0.0, max_iter=300, check_every=10, precision=precision, polish_iters=0)
            plain = tree.solve(inst.p, inst.q, **kw)
            tuned = tree.solve(inst.p, inst.q, tune=1, **kw)
            _same(tuned, plain)
            assert tuned[key] in _pairs(S, precision)
            again = tree.solve(inst.p, inst.q, tune=1, **kw)
            assert again[key] == tuned[key]  # kept by the plan, not re-timed
            _same(again, plain)
            # tune 0 goes back to the default pair
            assert tree.solve(inst.p, inst.q, **kw)[key] == _pairs(S, precision)[0]
        # a solve too short to time every pair: same bits, a listed pair
        short = dict(tol=0.0, max_iter=30, check_every=10, precision=32, polish_iters=10)
        a = tree.solve(inst.p, inst.q, **short)
        b = tree.solve(inst.p, inst.q, tune=1, **short)
        _same(a, b)
        assert b["chunk32"] in _pairs(S, 32) and b["chunk64"] in _pairs(S, 64)
    finally:
        system.close()
        ctx.systems.remove(system)


def test_tuned_batch_equals_untuned_and_server_takes_the_system_choice(ctx, lib):
    S, solver = lib
    insts = ds.batch_instances(4, first_seed=100)
    system = ctx.system(insts[0].sys)
    trees = []
    for inst in insts:
        t = system.tree(inst.tree)
        t.set_data(inst.d, inst.alpha2)
        t.factor(precond=1, power_iters=60)
        trees.append(t)
    try:
        kw = dict(tol=1e-3, max_iter=600, check_every=10, precision=32, polish_iters=20)
        ps, qs = [i.p for i in insts], [i.q for i in insts]
        _, plain = system.solve_batch(trees, ps, qs, **kw)
        _, tuned = system.solve_batch(trees, ps, qs, tune=1, **kw)
        for a, b in zip(plain, tuned):
            _same(a, b)
        choice = tuned[0]["chunk32"]
        assert all(r["chunk32"] == choice for r in tuned)
        # a server with tune 1 launches with the system's tuned float32 pair
        srv = system.server(max_active=4, tune=1, **kw)
        try:
            tickets = [srv.submit(t, i.p, i.q) for t, i in zip(trees, insts)]
            got = [srv.poll(tk) for tk in tickets]
        finally:
            srv.close()
        for g, a in zip(got, plain):
            assert g["chunk32"] == choice
            assert g["iterations"] == a["iterations"] and np.array_equal(g["u0"], a["u0"])
    finally:
        system.close()
        ctx.systems.remove(system)


def test_chunk_option_errors(ctx, lib):
    S, solver = lib
    inst = ds.tiny_instance()
    system, tree = solver.from_instance(ctx, inst, lambda_override=1.0)
    try:
        for bad in (dict(chunk32=(24, 8)), dict(chunk32=(16, 16)), dict(chunk64=(16, 16)), dict(tune=2)):
            with pytest.raises(S.SmpcError) as ei:
                tree.solve(inst.p, inst.q, tol=0.0, max_iter=10, **bad)
            assert ei.value.code == S.EINVAL
        # a half-given pair takes the default for the other kernel
        r = tree.solve(inst.p, inst.q, tol=0.0, max_iter=10, chunk64=(32, 0))
        assert r["chunk64"] == (32, S.smpc_chunk_lengths(64, 1)[0])
    finally:
        system.close()
        ctx.systems.remove(system)
