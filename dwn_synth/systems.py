"""Synthetic flow-based water-network models (paper Sec. II, eq. model and
eq. demand-control) with boxes and cost weights (Sec. III-A, III-D).

A system is a plain dict of float64 numpy arrays and scalars:

``nx, nu, nd, ne``            dimensions (``ne`` may be 0)
``A (nx,nx), B (nx,nu), Gd (nx,nd)``   dynamics ``x+ = A x + B u + Gd d``
``E (ne,nu), Ed (ne,nd)``     coupling ``E u + Ed d = 0``
``umin, umax`` (nu)           hard input box
``xmin, xmax`` (nx)           soft state box (distance penalty ``gamma_d``)
``xs`` (nx)                   safety level (distance penalty ``W_x``)
``W_alpha, alpha1 (nu), Wu (nu,nu), W_x, gamma_d``  cost weights
``weight_safety_by_prob``     1: the safety cost of node n is ``W_x * pi_n``

Nothing here computes anything the solver computes.
"""

from __future__ import annotations

import numpy as np


def tiny_tank_system(seed: int = 0) -> dict:
    """Four tanks, three flows, two demands, no junctions.

    ``A = I``; each column of ``B`` has a +1 at one tank and, with probability
    1/2, a -1 at another tank; the two demands drain two distinct tanks
    (``Gd = -selector``).  Boxes ``0 <= x <= 10`` (soft), ``0 <= u <= 5``
    (hard); safety level 2 with weight 100, soft-box weight 500; linear cost
    ``alpha1 ~ U[0.5, 2]``, smoothing weight ``Wu = 0.1 I``.
    """
    rng = np.random.default_rng(seed)
    nx, nu, nd = 4, 3, 2
    B = np.zeros((nx, nu))
    for j in range(nu):
        tanks = rng.permutation(nx)
        B[tanks[0], j] = 1.0
        if rng.random() < 0.5:
            B[tanks[1], j] = -1.0
    Gd = np.zeros((nx, nd))
    dt = rng.permutation(nx)[:nd]
    for k in range(nd):
        Gd[dt[k], k] = -1.0
    return {
        "nx": nx, "nu": nu, "nd": nd, "ne": 0,
        "A": np.eye(nx), "B": B, "Gd": Gd,
        "E": np.zeros((0, nu)), "Ed": np.zeros((0, nd)),
        "umin": np.zeros(nu), "umax": np.full(nu, 5.0),
        "xmin": np.zeros(nx), "xmax": np.full(nx, 10.0),
        "xs": np.full(nx, 2.0),
        "W_alpha": 1.0, "alpha1": rng.uniform(0.5, 2.0, nu),
        "Wu": 0.1 * np.eye(nu), "W_x": 100.0, "gamma_d": 500.0,
        "weight_safety_by_prob": 1,
    }


BARCELONA_DIMS = {"nx": 63, "nu": 114, "nd": 88, "ne": 17}
N_PUMPS = 38


def barcelona_shaped_system(seed: int = 1) -> dict:
    """A random supplied flow network with the Barcelona DWN dimensions (Sec. V).

    63 tanks, 114 flows, 88 demands, 17 junctions, ``A = I``.  Every flow
    carries water from an origin (a source such as a treatment plant or well, a
    tank, or a junction) to a destination (a tank or a junction):
    ``B[dest_tank, j] = +1``, ``B[orig_tank, j] = -1``, and a junction row of
    ``E`` has +1 for its inflow and -1 for its outflows, so ``E u + Ed d = 0``
    with ``Ed = -[I 0]`` is the junction mass balance (first 17 demands are
    junction consumption).  Supply structure: 14 sources feed 14 hub tanks
    directly and 6 sources feed 6 junctions whose 12 outflows feed 12 more hub
    tanks; 11 junctions take water from a hub tank and feed 22 tanks; each of
    the remaining 15 tanks gets a transfer from a hub tank; the remaining 34
    flows are random tank-to-tank transfers.  Tank and flow labels are then
    shuffled.  The other 71 demands drain tanks (``Gd = -selector``, every tank
    drained at least once).
    Tanks ``x in [0, 20 + U(0,30)]`` (soft), safety level ``0.3 x_max``;
    flows ``u in [0, u_max]``, ``u_max ~ U[10, 20]`` for sources and
    ``U[4, 12]`` otherwise.  ``alpha1 ~ U[0.5, 2]``; 38 flows are pumps whose
    time-varying cost weight is stored as ``pump_cols``/``pump_weight``.
    Weights keep the paper's ratios (``W_u = 5 I, W_x = 500, gamma_d = 2500``).
    """
    rng = np.random.default_rng(seed)
    nx, nu, nd, ne = 63, 114, 88, 17
    flows = []  # (origin, destination): ("src",), ("tank", k), ("junc", r)
    hubs = list(range(26))
    for k in range(14):
        flows.append((("src",), ("tank", k)))
    for r in range(6):
        flows.append((("src",), ("junc", r)))
        flows.append((("junc", r), ("tank", 14 + 2 * r)))
        flows.append((("junc", r), ("tank", 15 + 2 * r)))
    for r in range(6, ne):
        flows.append((("tank", int(rng.choice(hubs))), ("junc", r)))
        flows.append((("junc", r), ("tank", 26 + 2 * (r - 6))))
        flows.append((("junc", r), ("tank", 27 + 2 * (r - 6))))
    for k in range(48, nx):
        flows.append((("tank", int(rng.choice(hubs))), ("tank", k)))
    while len(flows) < nu:
        a, b = rng.choice(nx, size=2, replace=False)
        flows.append((("tank", int(a)), ("tank", int(b))))
    tank_label = rng.permutation(nx)
    order = rng.permutation(nu)
    flows = [flows[k] for k in order]
    B = np.zeros((nx, nu))
    E = np.zeros((ne, nu))
    is_src = np.zeros(nu, dtype=bool)
    for j, (orig, dest) in enumerate(flows):
        if dest[0] == "tank":
            B[tank_label[dest[1]], j] = 1.0
        else:
            E[dest[1], j] = 1.0
        if orig[0] == "src":
            is_src[j] = True
        elif orig[0] == "tank":
            B[tank_label[orig[1]], j] = -1.0
        else:
            E[orig[1], j] = -1.0
    assert np.linalg.matrix_rank(E) == ne
    Ed = np.zeros((ne, nd))
    Ed[:, :ne] = -np.eye(ne)
    Gd = np.zeros((nx, nd))
    tank_cols = np.arange(ne, nd)  # 71 tank demands
    tanks = np.concatenate([rng.permutation(nx), rng.integers(0, nx, size=len(tank_cols) - nx)])
    Gd[tanks, tank_cols] = -1.0
    xmax = 20.0 + rng.uniform(0.0, 30.0, nx)
    umax = np.where(is_src, rng.uniform(10.0, 20.0, nu), rng.uniform(4.0, 12.0, nu))
    pump_cols = np.sort(rng.choice(nu, size=N_PUMPS, replace=False))
    pump_weight = rng.uniform(0.0, 1.0, N_PUMPS)
    return {
        "nx": nx, "nu": nu, "nd": nd, "ne": ne,
        "A": np.eye(nx), "B": B, "Gd": Gd, "E": E, "Ed": Ed,
        "umin": np.zeros(nu), "umax": umax,
        "xmin": np.zeros(nx), "xmax": xmax, "xs": 0.3 * xmax,
        "W_alpha": 1.0, "alpha1": rng.uniform(0.5, 2.0, nu),
        "Wu": 5.0 * np.eye(nu), "W_x": 500.0, "gamma_d": 2500.0,
        "weight_safety_by_prob": 1,
        "pump_cols": pump_cols, "pump_weight": pump_weight, "source_cols": np.flatnonzero(is_src),
    }


def random_dense_system(seed: int, nx: int = 4, nu: int = 5, nd: int = 3, ne: int = 2) -> dict:
    """Small dense system with a general ``A`` and a non-diagonal SPD ``Wu``.

    Used to exercise the method beyond the water-network special structure
    (``A != I``, dense ``B``, ``ne >= 1`` couplings).
    """
    rng = np.random.default_rng(seed)
    A = np.eye(nx) + 0.3 * rng.standard_normal((nx, nx))
    B = rng.standard_normal((nx, nu))
    Gd = rng.standard_normal((nx, nd))
    E = rng.standard_normal((ne, nu)) if ne > 0 else np.zeros((0, nu))
    Ed = rng.standard_normal((ne, nd)) if ne > 0 else np.zeros((0, nd))
    G = rng.standard_normal((nu, nu))
    Wu = G @ G.T / nu + 0.5 * np.eye(nu)
    return {
        "nx": nx, "nu": nu, "nd": nd, "ne": ne,
        "A": A, "B": B, "Gd": Gd, "E": E, "Ed": Ed,
        "umin": -2.0 * np.ones(nu), "umax": 2.0 * np.ones(nu),
        "xmin": -1.0 * np.ones(nx), "xmax": 3.0 * np.ones(nx),
        "xs": 0.5 * np.ones(nx),
        "W_alpha": 1.0, "alpha1": rng.uniform(-1.0, 1.0, nu),
        "Wu": Wu, "W_x": 3.0, "gamma_d": 7.0,
        "weight_safety_by_prob": 1,
    }
