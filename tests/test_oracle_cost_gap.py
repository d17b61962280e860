"""Pins of the oracle's objective functions: the primal cost of eq. Sc-MPC,
the dual objective of eq. optim:prob and the a-posteriori duality gap of
Sec. IV-E.

Each pin is independent of the function it checks: a hand-computed worked
example, the objective value of an SLSQP solve of the epigraph form written
separately in ``tests/kkt_reference.py``, the inequality that defines a
convex conjugate (Fenchel-Young) against primal points from the dense KKT
reference, and weak/strong duality."""

import math

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O
from tests.kkt_reference import node_kkt_solve, slsqp_solve


def _three_node_problem():
    """Root + two children (probabilities 1, 0.25, 0.75), nx = 2, nu = 1."""
    sys = {
        "nx": 2, "nu": 1, "nd": 1, "ne": 0,
        "A": np.eye(2), "B": np.array([[1.0], [0.0]]), "Gd": np.array([[-1.0], [0.0]]),
        "E": np.zeros((0, 1)), "Ed": np.zeros((0, 1)),
        "umin": np.array([-10.0]), "umax": np.array([10.0]),
        "xmin": np.array([0.0, 0.0]), "xmax": np.array([3.0, 3.0]), "xs": np.array([1.0, 1.0]),
        "W_alpha": 2.0, "alpha1": np.array([1.5]), "Wu": np.array([[4.0]]),
        "W_x": 10.0, "gamma_d": 7.0, "weight_safety_by_prob": 1,
    }
    tree = {"N": 2, "M": 3, "stage": [0, 1, 1], "parent": [-1, 0, 0], "prob": [1.0, 0.25, 0.75]}
    return O.OracleProblem.from_parts(sys, tree, np.zeros((3, 1)), np.array([[0.0], [1.0]]),
                                      np.zeros(2), np.array([1.0]))


def test_primal_cost_worked_example():
    """eq. Sc-MPC at a hand-chosen point, summed by hand:

    * economic: stage-0 price 2 * 1.5 = 3, stage-1 price 2 * 2.5 = 5;
      1 * 3 * 2 + 0.25 * 5 * 3 + 0.75 * 5 * 0 = 9.75
    * smoothing (Wu = 4, q = 1): 1 * 4 * 1^2 + 0.25 * 4 * 1^2 + 0.75 * 4 * 2^2 = 17
    * safety (W_x = 10 weighted by pi, xs = (1, 1)): x0 = (0, 2) is 1 below,
      x1 = (-2, -3) is (3, 4) below -> 10 * 1 * 1 + 10 * 0.25 * 5 = 22.5
    * soft box (gamma_d = 7, [0, 3]^2): only x1 is outside, by (2, 3) -> 7 sqrt(13)
    """
    P = _three_node_problem()
    x = np.array([[0.0, 2.0], [-2.0, -3.0], [1.5, 1.0]])
    u = np.array([[2.0], [3.0], [0.0]])
    expected = 9.75 + 17.0 + 22.5 + 7.0 * math.sqrt(13.0)
    assert abs(O.primal_cost(P, x, u) - expected) <= 1e-12 * expected
    assert abs(O.stage_cost(P, u) - 26.75) <= 1e-12 * 26.75
    assert abs(O.soft_cost(P, x, x) - (22.5 + 7.0 * math.sqrt(13.0))) <= 1e-12 * 50


@pytest.fixture(scope="module")
def tiny_opt():
    """The tiny instance solved by SLSQP (epigraph form) and by 20 000 FP64
    APG iterations."""
    inst = ds.tiny_instance()
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    S = np.repeat(np.sqrt(P.prob)[:, None], 3, 1)
    K = O.dual_hessian_dense(P, F, S)
    lam = 1.0 / np.linalg.eigvalsh(0.5 * (K + K.T))[-1]
    r = O.apg(P, lam, 20000, F, scale=S)
    xq, uq, res = slsqp_solve(inst)
    return inst, P, F, r, xq, uq, res


def test_primal_cost_equals_slsqp_objective(tiny_opt):
    """At the SLSQP optimum the epigraph variables equal the distances, so
    its objective value (computed from the slacks) is the primal cost.
    (SLSQP at ftol 1e-14 ends with its line-search status 8 on this
    instance; its equality constraints and epigraph slacks hold to about
    1e-8, which bounds the agreement: 1e-7 relative.  A dropped probability
    on a cost term or a wrong weight moves the cost by far more.)"""
    inst, P, F, r, xq, uq, res = tiny_opt
    assert abs(O.primal_cost(P, xq, uq) - res.fun) <= 1e-7 * abs(res.fun)


def test_dual_objective_is_a_conjugate(tiny_opt):
    """f*(-H'y) = sup_z <-H'y, z> - f(z): the value from the solve step is at
    least -(<y, Hz> + f(z)) for every dynamically feasible z (points from the
    dense KKT reference at random duals), with equality at z = z(y)."""
    inst, P, F, r, xq, uq, res = tiny_opt
    rng = np.random.default_rng(3)
    for trial in range(4):
        y = rng.standard_normal((P.M, P.dual_dim)) * (1.0 + 10.0 * trial)
        xy, uy = node_kkt_solve(inst, y)
        sval, _ = O.support_g(P, y)
        fconj = O.dual_objective(P, F, y)[0] - sval
        assert abs(fconj + O.stage_cost(P, uy) + np.sum(y * O.smpc_oracle.hz(xy, uy))) <= 1e-9 * max(1.0, abs(fconj))
        for _ in range(5):
            xz, uz = node_kkt_solve(inst, rng.standard_normal((P.M, P.dual_dim)) * 20.0)
            lower = -(O.stage_cost(P, uz) + np.sum(y * O.smpc_oracle.hz(xz, uz)))
            assert fconj >= lower - 1e-9 * max(1.0, abs(lower))


def test_support_function_by_sampling():
    """g*(y) >= <y, t> - g(t) for sampled t (Fenchel-Young), on one node of
    the tiny instance, with y in the domain of g*."""
    inst = ds.tiny_instance()
    P = O.OracleProblem.from_instance(inst)
    rng = np.random.default_rng(5)
    nx = P.nx
    for _ in range(20):
        y = np.zeros((P.M, P.dual_dim))
        ys = -np.abs(rng.standard_normal((P.M, nx)))
        ys *= (P.safety_weight() * rng.uniform(0, 1, P.M) / np.linalg.norm(ys, axis=1))[:, None]
        yz = rng.standard_normal((P.M, nx))
        yz *= (P.box_weight() * rng.uniform(0, 1, P.M) / np.linalg.norm(yz, axis=1))[:, None]
        y[:, :nx], y[:, nx:2 * nx], y[:, 2 * nx:] = ys, yz, rng.standard_normal((P.M, P.nu)) * 3
        val, viol = O.support_g(P, y)
        assert viol <= 0.0
        for _ in range(20):
            t = rng.uniform(-5, 15, (P.M, P.dual_dim))
            t[:, 2 * nx:] = rng.uniform(P.umin, P.umax, (P.M, P.nu))  # in the input box
            g = O.soft_cost(P, t[:, :nx], t[:, nx:2 * nx])
            assert val >= np.sum(y * t) - g - 1e-9 * max(1.0, abs(val))


def test_strong_duality_and_gap_at_the_optimum(tiny_opt):
    """D(y) at the long-run dual equals minus the optimal cost (SLSQP), and
    the gap of the APG's last (z, t, y) vanishes."""
    inst, P, F, r, xq, uq, res = tiny_opt
    D, viol = O.dual_objective(P, F, r.y)
    assert viol <= 1e-9 * max(P.W_x, P.gamma_d)
    assert abs(D + res.fun) <= 1e-6 * abs(res.fun)
    gap = O.duality_gap(P, F, r.x, r.u, r.t, r.y)
    assert abs(gap) <= 1e-6 * abs(res.fun)


def test_weak_duality_gap_nonnegative(tiny_opt):
    """For the feasible primal pair (z, t = Hz) of the SLSQP optimum and any
    dual y in dom g*, the gap is >= 0.  For an APG iterate, H z^nu != t^nu,
    so the gap may have either sign, and like the residual it does not fall
    monotonically; over a few thousand iterations it falls by orders of
    magnitude."""
    inst, P, F, r, xq, uq, res = tiny_opt
    nx = P.nx
    rng = np.random.default_rng(11)
    tq = O.smpc_oracle.hz(xq, uq)
    for _ in range(10):
        y = r.y + rng.standard_normal(r.y.shape) * rng.uniform(0.01, 5.0)
        # move y into dom g*: sigma~ <= 0 and both balls
        y[:, :nx] = np.minimum(y[:, :nx], 0.0)
        for b, c in ((0, P.safety_weight()), (1, P.box_weight())):
            blk = y[:, b * nx:(b + 1) * nx]
            nr = np.linalg.norm(blk, axis=1)
            blk *= np.minimum(1.0, c / np.maximum(nr, 1e-300))[:, None]
        assert O.support_g(P, y)[1] <= 1e-12
        assert O.duality_gap(P, F, xq, uq, tq, y) >= -1e-8 * abs(res.fun)
    lam = 1.0 / (1.02 * O.dual_lmax_power(P, 500, F))
    gaps = []
    for k in (50, 400, 6400):
        rk = O.apg(P, lam, k, F)
        gaps.append(O.duality_gap(P, F, rk.x, rk.u, rk.t, rk.y))
    assert abs(gaps[2]) < 1e-2 * abs(gaps[1]) and abs(gaps[1]) < 0.5 * abs(gaps[0])
