"""Complete problem instances: system + scenario tree + node demands + initial
conditions (paper eq. demand:tree, eq. Sc-MPC).

Workload recipes (all seeded, all synthetic):

* ``tiny_instance``: 4 tanks / 3 flows / 2 demands, ``N = 4``, branching
  [2, 2] (4 scenarios, 11 nodes), demands ``N(1.0, 0.1^2)`` per node and
  component, ``p = 5``, ``q = 1``.
* ``barcelona_instance``: Barcelona-shaped system (63/114/88/17), ``N = 24``,
  branching [7, 7, 7] (343 scenarios, 7260 nodes), log-normal demands around
  a 24-periodic profile with 10 % spread (junction consumption within the
  junction's inflow capacity), hourly pumping tariff, ``p = 0.6 x_max``,
  ``q = 0.3 u_max``.
* ``batch_instances``: 64 trees (seeds 100..163) on the Barcelona-shaped
  system, horizons in {12, 18, 24}, scenario counts in {16, 64, 125, 343, 512}.
* ``random_small_instance``: small dense systems with general ``A`` and
  couplings, for exact-arithmetic checks.
* ``serving_controllers``: 256 controllers on the shared Barcelona-shaped
  system, tree sizes drawn as for the batch (seed 2024), for the served
  closed loop; ``step_demands`` draws a controller's demands for a later
  hour (shifted profile, fresh per-node noise).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .systems import barcelona_shaped_system, random_dense_system, tiny_tank_system
from .trees import table1_tree, uniform_tree


@dataclass
class Instance:
    """One scenario-tree MPC problem.  ``d`` is ``(M, nd)``, ``alpha2`` is
    ``(N, nu)``, ``p`` the measured state, ``q`` the previous input."""

    name: str
    sys: dict
    tree: dict
    d: np.ndarray
    alpha2: np.ndarray
    p: np.ndarray
    q: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.tree["M"])

    @property
    def N(self) -> int:
        return int(self.tree["N"])


def tiny_instance(seed: int = 0, N: int = 4, branching=(2, 2)) -> Instance:
    sys = tiny_tank_system(seed)
    tree = uniform_tree(N, list(branching))
    rng = np.random.default_rng([seed, 1])
    d = rng.normal(1.0, 0.1, size=(tree["M"], sys["nd"]))
    alpha2 = np.zeros((N, sys["nu"]))
    return Instance("tiny", sys, tree, d, alpha2, np.full(sys["nx"], 5.0), np.ones(sys["nu"]))


def tariff(hour: int) -> float:
    """Two-level electricity tariff: peak 1.0 for hours 8..21, off-peak 0.4."""
    return 1.0 if 8 <= (hour % 24) < 22 else 0.4


def pumping_cost(sys: dict, N: int, start_hour: int = 0) -> np.ndarray:
    """Time-varying pumping cost ``alpha_2`` (N, nu): tariff x pump weight."""
    a2 = np.zeros((N, sys["nu"]))
    for j in range(N):
        a2[j, sys["pump_cols"]] = tariff(start_hour + j) * sys["pump_weight"]
    return a2


def barcelona_demands(sys: dict, tree: dict, rng: np.random.Generator, start_hour: int = 0):
    """Node demands for a Barcelona-shaped system.

    Every demand follows ``dhat_k(j) = b_k (1 + 0.3 sin(2 pi (j + phi_k) / 24))``
    with ``phi_k ~ U[0, 24)``, perturbed per node by the log-normal factor
    ``exp(0.1 eps - 0.005)``, ``eps ~ N(0, 1)``.  Tank demands use
    ``b_k ~ U[0.5, 2]``.  Junction demands (consumption at the junction, first
    ``ne`` entries) use ``b_k`` = 0.25 x the capacity of the junction's inflow,
    so with the profile and noise they stay below half of it: the point
    "inflow = junction demand, outflows = 0" satisfies ``E u + Ed d = 0`` inside
    the input box at every node.
    Returns ``(d, u_f)`` with ``u_f`` that feasible point per node.
    """
    M, ne, nd, nu = tree["M"], sys["ne"], sys["nd"], sys["nu"]
    E = sys["E"]
    base = np.empty(nd)
    base[ne:] = rng.uniform(0.5, 2.0, nd - ne)
    inflow = np.array([int(np.flatnonzero(E[r] > 0)[0]) for r in range(ne)], dtype=np.int64)
    base[:ne] = 0.25 * sys["umax"][inflow]
    phi = rng.uniform(0.0, 24.0, nd)
    hours = (start_hour + tree["stage"]).astype(np.float64)
    dhat = base[None, :] * (1.0 + 0.3 * np.sin(2.0 * np.pi * (hours[:, None] + phi[None, :]) / 24.0))
    eps = rng.standard_normal((M, nd))
    d = dhat * np.exp(0.1 * eps - 0.005)
    uf = np.zeros((M, nu))
    uf[:, inflow] = d[:, :ne]
    return d, uf


def barcelona_instance(seed: int = 1, N: int = 24, branching=(7, 7, 7), sys: dict | None = None,
                       demand_seed: int | None = None) -> Instance:
    if sys is None:
        sys = barcelona_shaped_system(seed)
    tree = uniform_tree(N, list(branching))
    rng = np.random.default_rng([seed if demand_seed is None else demand_seed, 2])
    d, uf = barcelona_demands(sys, tree, rng)
    alpha2 = pumping_cost(sys, N)
    p = 0.6 * sys["xmax"]
    q = 0.3 * sys["umax"]
    return Instance(f"barcelona-N{N}-b{'x'.join(map(str, branching))}", sys, tree, d, alpha2, p, q,
                    extra={"uf": uf})


BATCH_SHAPES = {16: [4, 4], 64: [4, 4, 4], 125: [5, 5, 5], 343: [7, 7, 7], 512: [8, 8, 8]}
BATCH_HORIZONS = (12, 18, 24)


def closed_loop_demands(sys: dict, tree: dict, hours: int, seed: int = 77):
    """Demands and pumping costs of ``hours`` closed-loop steps (Alg. 2) of a
    controller on a Barcelona-shaped system.

    One fixed 24-periodic profile per demand, ``b_k (1 + 0.3 sin(2 pi (h +
    phi_k) / 24))`` (``b_k``, ``phi_k`` as in ``barcelona_demands``), drawn
    from ``seed`` alone, so every controller sees the same profile and the
    same realised demands ``actual[h] = profile(h) exp(0.1 eps_h - 0.005)``.
    At step ``h`` the tree's root carries ``actual[h]`` (known when u_0 is
    decided) and a node at stage j the forecast ``profile(h + j)
    exp(0.1 eps - 0.005)`` with fresh per-node noise.  Returns a list of
    ``(d, alpha2)``; ``d[0]`` of step h is the demand the plant sees."""
    M, ne, nd = tree["M"], sys["ne"], sys["nd"]
    E = sys["E"]
    prof_rng = np.random.default_rng([seed, 1])
    base = np.empty(nd)
    base[ne:] = prof_rng.uniform(0.5, 2.0, nd - ne)
    inflow = np.array([int(np.flatnonzero(E[r] > 0)[0]) for r in range(ne)], dtype=np.int64)
    base[:ne] = 0.25 * sys["umax"][inflow]
    phi = prof_rng.uniform(0.0, 24.0, nd)

    def profile(hours_arr):
        return base[None, :] * (1.0 + 0.3 * np.sin(2.0 * np.pi * (hours_arr[:, None] + phi[None, :]) / 24.0))

    act_rng = np.random.default_rng([seed, 2])
    actual = profile(np.arange(hours, dtype=np.float64)) * np.exp(0.1 * act_rng.standard_normal((hours, nd)) - 0.005)
    out = []
    for h in range(hours):
        rng = np.random.default_rng([seed, 3, h])
        d = profile((h + tree["stage"]).astype(np.float64)) * np.exp(0.1 * rng.standard_normal((M, nd)) - 0.005)
        d[0] = actual[h]
        out.append((d, pumping_cost(sys, int(tree["N"]), start_hour=h)))
    return out


def table1_instance(name: str, seed: int = 1, sys: dict | None = None) -> Instance:
    """A Table 1 controller (Sec. V-B: its branching and scenario count, N =
    24) on the Barcelona-shaped system, with demands, pumping cost and initial
    state drawn as in ``barcelona_instance``."""
    if sys is None:
        sys = barcelona_shaped_system(seed)
    tree = table1_tree(name)
    rng = np.random.default_rng([seed, 2])
    d, uf = barcelona_demands(sys, tree, rng)
    return Instance(f"table1-{name}", sys, tree, d, pumping_cost(sys, int(tree["N"])), 0.6 * sys["xmax"],
                    0.3 * sys["umax"], extra={"uf": uf})


def batch_instances(n_trees: int = 64, first_seed: int = 100, system_seed: int = 1) -> list[Instance]:
    """``n_trees`` independent trees on one shared Barcelona-shaped system.

    Tree ``i`` uses seed ``first_seed + i`` to draw its horizon (uniform in
    {12, 18, 24}), its scenario count (uniform in {16, 64, 125, 343, 512},
    full branching over the first 2-3 stages), its demands and its initial
    tank levels ``p = x_max * U(0.4, 0.8)``.
    """
    sys = barcelona_shaped_system(system_seed)
    out = []
    for i in range(n_trees):
        seed = first_seed + i
        rng = np.random.default_rng(seed)
        N = int(rng.choice(BATCH_HORIZONS))
        scen = int(rng.choice(sorted(BATCH_SHAPES)))
        branching = BATCH_SHAPES[scen]
        tree = uniform_tree(N, branching)
        d, uf = barcelona_demands(sys, tree, rng)
        alpha2 = pumping_cost(sys, N)
        p = sys["xmax"] * rng.uniform(0.4, 0.8, sys["nx"])
        q = 0.3 * sys["umax"]
        out.append(Instance(f"batch{seed}-N{N}-s{scen}", sys, tree, d, alpha2, p, q, extra={"uf": uf}))
    return out


def random_small_instance(seed: int, nx: int = 4, nu: int = 5, nd: int = 3, ne: int = 2,
                          N: int = 3, branching=(2, 2), scenarios: int | None = None) -> Instance:
    """Dense random system (general ``A``, ``ne`` couplings) on a small tree."""
    sys = random_dense_system(seed, nx, nu, nd, ne)
    tree = uniform_tree(N, list(branching), scenarios=scenarios)
    rng = np.random.default_rng([seed, 3])
    d = rng.standard_normal((tree["M"], nd))
    alpha2 = 0.5 * rng.standard_normal((N, nu))
    p = rng.uniform(0.0, 2.0, nx)
    q = rng.uniform(-1.0, 1.0, nu)
    return Instance(f"random{seed}", sys, tree, d, alpha2, p, q)


def serving_controllers(n: int = 256, seed: int = 2024, system_seed: int = 1) -> list[Instance]:
    """``n`` controllers for the served closed loop: controller ``i`` draws its
    horizon, scenario count and initial levels like a batch tree, from
    ``default_rng([seed, i])``, on the shared Barcelona-shaped system."""
    sys = barcelona_shaped_system(system_seed)
    out = []
    for i in range(n):
        rng = np.random.default_rng([seed, i])
        N = int(rng.choice(BATCH_HORIZONS))
        scen = int(rng.choice(sorted(BATCH_SHAPES)))
        tree = uniform_tree(N, BATCH_SHAPES[scen])
        d, uf = barcelona_demands(sys, tree, rng)
        p = sys["xmax"] * rng.uniform(0.4, 0.8, sys["nx"])
        q = 0.3 * sys["umax"]
        out.append(Instance(f"ctrl{i}-N{N}-s{scen}", sys, tree, d, pumping_cost(sys, N), p, q,
                            extra={"uf": uf, "seed": [seed, i]}))
    return out


def step_demands(inst: Instance, step: int, rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """Demands and pumping cost of ``inst``'s tree for the MPC step ``step``
    hours later: the same per-demand profiles shifted by ``step`` hours, with
    fresh node noise."""
    sys, tree = inst.sys, inst.tree
    d, _ = barcelona_demands(sys, tree, rng, start_hour=step)
    return d, pumping_cost(sys, int(tree["N"]), start_hour=step)
