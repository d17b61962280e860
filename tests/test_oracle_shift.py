"""Pins of the receding-horizon warm start of the oracle (``shift_map``,
``shift_dual``): the reading of the shift is stated in the oracle; these tests
check the implementation against constructions written independently of it."""

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O


def _problem(N, branching, seed=0):
    inst = ds.random_small_instance(seed, nx=3, nu=4, nd=2, ne=1, N=N, branching=branching)
    return O.OracleProblem.from_instance(inst)


def test_one_scenario_shift_drops_the_first_stage():
    P = _problem(6, ())
    D = P.dual_dim
    y = np.arange(P.M * D, dtype=float).reshape(P.M, D)
    expect = np.vstack([y[1:], y[-1:]])  # stage j <- stage j + 1, last duplicated
    assert np.array_equal(O.shift_dual(P, y, 0), expect)


@pytest.mark.parametrize("realized", [0, 1, 2])
def test_uniform_tree_images_by_construction(realized):
    # branching 3 at stage 0 and 2 at stage 1, N = 4: stage sizes 1, 3, 6, 6
    # with node ids 0 | 1..3 | 4..9 | 10..15, children numbered consecutively
    P = _problem(4, (3, 2))
    assert list(np.bincount(P.stage)) == [1, 3, 6, 6]
    img = O.shift_map(P, realized)
    expect = np.empty(16, dtype=int)
    expect[0] = 1 + realized                      # new root = realised child
    for k in range(3):                            # new stage 1, child k of the root
        expect[1 + k] = 4 + 2 * realized + min(k, 1)   # old stage-2 child (2 per node)
    for a in range(3):                            # new stage 2: children of new node 1 + a
        for k in range(2):
            old_parent = expect[1 + a]            # an old stage-2 node, one child each
            expect[4 + 2 * a + k] = 10 + (old_parent - 4)
    for n in range(10, 16):                       # new stage 3: below the old last stage
        expect[n] = expect[4 + (n - 10)]
    assert np.array_equal(img, expect)


def test_probability_weighted_invariant():
    P = _problem(5, (2, 3), seed=3)
    nx, nu = P.nx, P.nu
    rng = np.random.default_rng(0)
    a, b, c = rng.normal(size=(P.N, nx)), rng.normal(size=(P.N, nx)), rng.normal(size=(P.N, nu))
    pi, s = P.prob, P.stage
    y = np.hstack([pi[:, None] * a[s], b[s], pi[:, None] * c[s]])
    out = O.shift_dual(P, y, 1)
    s_img = np.minimum(s + 1, P.N - 1)  # image stage: one later, the last one repeated
    expect = np.hstack([pi[:, None] * a[s_img], b[s_img], pi[:, None] * c[s_img]])
    assert np.allclose(out, expect, rtol=1e-14, atol=1e-14)


def test_unweighted_safety_block_is_not_rescaled():
    P = _problem(4, (2, 2))
    P.weight_safety_by_prob = 0
    y = np.ones((P.M, P.dual_dim))
    out = O.shift_dual(P, y, 0)
    assert np.all(out[:, :2 * P.nx] == 1.0)
    img = O.shift_map(P, 0)
    assert np.allclose(out[:, 2 * P.nx:], (P.prob / P.prob[img])[:, None])


def test_realized_child_out_of_range():
    P = _problem(4, (2, 2))
    with pytest.raises(ValueError):
        O.shift_map(P, 2)


def test_shift_is_a_closer_start_when_the_data_repeat():
    """The receding-horizon case the shift is built for: the next problem is
    the realised subtree one stage later with the same node data (the last
    stage repeated), started from the state and input the first solve
    applied.  Warm-started from the shifted dual the APG meets the tolerance
    in far fewer iterations than from zero."""
    inst = ds.tiny_instance(N=8, branching=(2, 2))
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    lam = 1.0 / (1.02 * O.dual_lmax_power(P, 300, F))
    r0 = O.apg(P, lam, 50000, F, tol=1e-3)
    assert r0.converged
    img = O.shift_map(P, 0)
    Q = O.OracleProblem.from_parts(inst.sys, inst.tree, P.d[img], P.alpha2, r0.x[0], r0.u0)
    FQ = O.factor_step(Q)
    cold = O.apg(Q, lam, 50000, FQ, tol=1e-3)
    warm = O.apg(Q, lam, 50000, FQ, tol=1e-3, y0=O.shift_dual(P, r0.y, 0))
    assert cold.converged and warm.converged
    assert warm.iterations < 0.5 * cold.iterations, (warm.iterations, cold.iterations)
