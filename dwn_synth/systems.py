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
    """A random flow network with the Barcelona DWN dimensions (Sec. V).

    63 tanks, 114 flows, 88 demands, 17 junctions, ``A = I``.  Every flow
    carries water from an origin (a source such as a treatment plant or well, a
    tank, or a junction) to a destination (a tank or a junction):
    ``B[dest_tank, j] = +1``, ``B[orig_tank, j] = -1``, and a junction row of
    ``E`` has +1 for its inflows and -1 for its outflows, so
    ``E u + Ed d = 0`` with ``Ed = -[I 0]`` is the junction mass balance
    (first 17 demands).  The flows are: 17 x 3 junction flows (one inflow, from
    a source for 6 junctions and from a tank for 11, and two outflows to
    tanks), 14 sources feeding tanks directly and 49 tank-to-tank transfers;
    every tank receives at least one inflow.  The other 71 demands drain tanks
    (``Gd = -selector``, every tank drained at least once).
    Tanks ``x in [0, 20 + U(0,30)]`` (soft), safety level ``0.3 x_max``;
    flows ``u in [0, u_max]``, ``u_max ~ U[4, 12]`` for sources and
    ``U[2, 10]`` otherwise.  ``alpha1 ~ U[0.5, 2]``; 38 flows are pumps whose
    time-varying cost weight is stored as ``pump_cols``/``pump_weight``.
    Weights keep the paper's ratios (``W_u = 5 I, W_x = 500, gamma_d = 2500``).
    """
    rng = np.random.default_rng(seed)
    nx, nu, nd, ne = 63, 114, 88, 17
    # (origin kind, destination kind): kinds are "src", "tank", "junc"
    flows = []
    for r in range(ne):
        flows.append(("src" if r < 6 else "tank", ("junc", r)))
        flows.append((("junc", r), "tank"))
        flows.append((("junc", r), "tank"))
    flows += [("src", "tank")] * 14
    flows += [("tank", "tank")] * (nu - len(flows))
    assert len(flows) == nu
    order = rng.permutation(nu)
    flows = [flows[k] for k in order]
    n_dest_tank = sum(1 for f in flows if f[1] == "tank")
    dest_tanks = np.concatenate([rng.permutation(nx), rng.integers(0, nx, size=n_dest_tank - nx)])
    rng.shuffle(dest_tanks)
    B = np.zeros((nx, nu))
    E = np.zeros((ne, nu))
    is_src = np.zeros(nu, dtype=bool)
    k = 0
    for j, (orig, dest) in enumerate(flows):
        if dest == "tank":
            dt = int(dest_tanks[k])
            k += 1
            B[dt, j] = 1.0
        else:
            dt = -1
            E[dest[1], j] = 1.0
        if orig == "src":
            is_src[j] = True
        elif orig == "tank":
            ot = int(rng.integers(0, nx))
            while ot == dt:
                ot = int(rng.integers(0, nx))
            B[ot, j] = -1.0
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
    umax = np.where(is_src, rng.uniform(4.0, 12.0, nu), rng.uniform(2.0, 10.0, nu))
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
