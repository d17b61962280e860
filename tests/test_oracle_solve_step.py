"""Pins of the oracle's solve step (Alg. 1, App. B) against dense KKT solves."""

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O
from tests.kkt_reference import node_kkt_solve, scenario_kkt_solve


CASES = [
    ("random-A-ne2", lambda: ds.random_small_instance(0, nx=4, nu=5, nd=3, ne=2, N=3, branching=(2, 2))),
    ("random-A-ne1-ragged", lambda: ds.random_small_instance(1, nx=3, nu=4, nd=2, ne=1, N=4, branching=(3, 2), scenarios=4)),
    ("random-A-ne0", lambda: ds.random_small_instance(2, nx=4, nu=3, nd=2, ne=0, N=3, branching=(2, 3))),
    ("tiny-tank", lambda: ds.tiny_instance()),
    ("single-node", lambda: ds.random_small_instance(3, nx=3, nu=4, nd=2, ne=1, N=1, branching=())),
    ("one-scenario", lambda: ds.random_small_instance(4, nx=3, nu=4, nd=2, ne=2, N=5, branching=())),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_solve_step_matches_dense_kkt(case):
    inst = case[1]()
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    rng = np.random.default_rng(11)
    for _ in range(3):
        w = rng.standard_normal((P.M, P.dual_dim)) * 3.0
        x, u = O.solve_step(P, F, w)
        xk, uk = node_kkt_solve(inst, w)
        scale = max(1.0, np.abs(xk).max(), np.abs(uk).max())
        assert np.abs(x - xk).max() <= 1e-12 * scale
        assert np.abs(u - uk).max() <= 1e-12 * scale
        # dynamics and coupling hold exactly at every node
        for n in range(P.M):
            a = P.parent[n]
            xa = P.p if a < 0 else x[a]
            assert np.abs(x[n] - P.A @ xa - P.B @ u[n] - P.Gd @ P.d[n]).max() <= 1e-12 * scale
            if P.ne:
                assert np.abs(P.E @ u[n] + P.Ed @ P.d[n]).max() <= 1e-12 * scale


@pytest.mark.parametrize("case", CASES[:3], ids=[c[0] for c in CASES[:3]])
def test_solve_step_matches_scenario_form(case):
    """Same minimiser from the scenario formulation with explicit
    non-anticipativity (one copy per root-to-leaf path)."""
    inst = case[1]()
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    w = np.random.default_rng(5).standard_normal((P.M, P.dual_dim))
    x, u = O.solve_step(P, F, w)
    xs, us, spread = scenario_kkt_solve(inst, w)
    scale = max(1.0, np.abs(xs).max(), np.abs(us).max())
    assert spread <= 1e-12 * scale
    assert np.abs(x - xs).max() <= 1e-11 * scale
    assert np.abs(u - us).max() <= 1e-11 * scale


def test_solve_step_invariant_to_null_space_basis():
    """Any full-rank basis of ker E gives the same (x, u) (App. A leaves L free)."""
    inst = ds.random_small_instance(7, nx=3, nu=6, nd=3, ne=2, N=3, branching=(2, 2))
    P = O.OracleProblem.from_instance(inst)
    L = O.null_space_basis(P.E, P.nu)
    T = np.random.default_rng(1).standard_normal((L.shape[1], L.shape[1])) + 2 * np.eye(L.shape[1])
    F1 = O.factor_step(P)
    F2 = O.factor_step(P, O.cost_update(P, L @ T))
    w = np.random.default_rng(2).standard_normal((P.M, P.dual_dim))
    x1, u1 = O.solve_step(P, F1, w)
    x2, u2 = O.solve_step(P, F2, w)
    assert np.abs(x1 - x2).max() < 1e-10 * max(1, np.abs(x1).max())
    assert np.abs(u1 - u2).max() < 1e-10 * max(1, np.abs(u1).max())


def test_identical_siblings_get_identical_solutions():
    inst = ds.random_small_instance(8, nx=3, nu=4, nd=2, ne=1, N=3, branching=(3, 1))
    # give the three stage-1 siblings (and their children) identical data
    sib = np.flatnonzero(inst.tree["stage"] == 1)
    inst.d[sib] = inst.d[sib[0]]
    kids = np.flatnonzero(inst.tree["stage"] == 2)
    inst.d[kids] = inst.d[kids[0]]
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    w = np.random.default_rng(3).standard_normal((P.M, P.dual_dim))
    w[sib] = w[sib[0]]
    w[kids] = w[kids[0]]
    x, u = O.solve_step(P, F, w)
    for group in (sib, kids):
        assert np.abs(x[group] - x[group[0]]).max() < 1e-12
        assert np.abs(u[group] - u[group[0]]).max() < 1e-12


def test_solve_step_linear_part_is_linear():
    inst = ds.random_small_instance(9, N=3, branching=(2, 2))
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    rng = np.random.default_rng(4)
    w1, w2 = rng.standard_normal((2, P.M, P.dual_dim))
    xa, ua = O.solve_step(P, F, 2.0 * w1 - 3.0 * w2, affine=False)
    x1, u1 = O.solve_step(P, F, w1, affine=False)
    x2, u2 = O.solve_step(P, F, w2, affine=False)
    assert np.allclose(xa, 2 * x1 - 3 * x2, atol=1e-10)
    assert np.allclose(ua, 2 * u1 - 3 * u2, atol=1e-10)
    # affine part = solve step at w = 0
    x0, u0 = O.solve_step(P, F, np.zeros_like(w1))
    xf, uf = O.solve_step(P, F, w1)
    assert np.allclose(xf, x0 + x1, atol=1e-10)
    assert np.allclose(uf, u0 + u1, atol=1e-10)
