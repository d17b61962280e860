"""Pins of the oracle's closed-loop pieces (Sec. II eq. model, Sec. V-B
KPIs): a hand-summed two-step example and the plant step written out."""

import numpy as np

import dwn_synth as ds
import oracle as O


def test_kpis_hand_summed_example():
    alpha1 = np.array([1.0, 2.0])
    alpha2 = np.array([[0.5, 0.0], [0.0, 1.0]])
    u = np.array([[1.0, -2.0], [3.0, 0.0]])
    x = np.array([[1.0, 3.0], [2.5, 0.5]])
    xs = np.array([2.0, 2.0])
    k = O.closed_loop_kpis(alpha1, alpha2, xs, x, u, np.zeros(2))
    # E: ((1.5, 2).(1, 2) + (1, 3).(3, 0)) / 2; the |u| matters (u has a -2)
    assert abs(k["E"] - 4.25) <= 1e-15
    # dU: (|(1, -2) - 0|^2 + |(3, 0) - (1, -2)|^2) / 2 = (5 + 8) / 2
    assert abs(k["dU"] - 6.5) <= 1e-15
    # S: [xs - x1]_+ = (1, 0), [xs - x2]_+ = (0, 1.5)
    assert abs(k["S"] - 2.5) <= 1e-15
    # R: |xs|_1 / mean |x_k|_1 = 4 / ((4 + 3) / 2), in percent
    assert abs(k["R"] - 400.0 / 3.5) <= 1e-12


def test_kpis_invariants():
    rng = np.random.default_rng(3)
    Hs, nx, nu = 7, 4, 3
    a1, a2 = rng.uniform(0.5, 2, nu), rng.uniform(0, 1, (Hs, nu))
    u, x = rng.normal(size=(Hs, nu)), rng.uniform(1, 5, (Hs, nx))
    xs = np.full(nx, 0.5)
    k = O.closed_loop_kpis(a1, a2, xs, x, u, u[0])
    assert k["S"] == 0.0                                   # never below the safety level
    assert k["dU"] >= 0.0 and k["E"] > 0.0
    k2 = O.closed_loop_kpis(a1, a2, xs, 2.0 * x, u, u[0])  # double the volumes
    assert abs(k2["R"] - k["R"] / 2.0) <= 1e-12 * k["R"]
    k3 = O.closed_loop_kpis(a1, a2, xs, x, -u, -u[0])     # E uses |u|; dU is even
    assert abs(k3["E"] - k["E"]) <= 1e-12 * k["E"] and abs(k3["dU"] - k["dU"]) <= 1e-12 * k["dU"]


def test_plant_step_is_the_flow_model():
    inst = ds.random_small_instance(4, nx=3, nu=4, nd=2, ne=1, N=3, branching=(2,))
    P = O.OracleProblem.from_instance(inst)
    x, u, d = np.array([1.0, 2.0, 3.0]), np.array([0.5, -1.0, 2.0, 0.0]), np.array([0.3, 0.7])
    expect = np.array([sum(P.A[i, j] * x[j] for j in range(3)) + sum(P.B[i, j] * u[j] for j in range(4))
                       + sum(P.Gd[i, j] * d[j] for j in range(2)) for i in range(3)])
    assert np.allclose(O.plant_step(P, x, u, d), expect, rtol=1e-14, atol=1e-14)
