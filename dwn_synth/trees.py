"""Scenario-tree shapes (paper Sec. III-C; Table 1 controller shapes).

Node convention used throughout: the nodes are the *decision nodes* of the
tree.  A node at stage ``j`` (``0 <= j <= N-1``) carries the demand ``d_j``,
the input ``u_j`` decided once ``d_j`` is revealed, and the state ``x_{j+1}``
that results.  Stage 0 holds the root only.  With this convention a tree with
``mu(j)`` nodes at stage ``j`` has ``sum_j mu(j) * (n_x + n_u)`` primal and
``sum_j mu(j) * (2 n_x + n_u)`` dual variables, which is how Table 1 counts
them.

Nodes are returned stage-sorted (BFS order): every parent index is smaller than
its children's, and the children of a node are consecutive.
"""

from __future__ import annotations

import numpy as np

# Table 1 (Sec. V-B): controller name -> (maximum branching factors b_j of the
# first stages, number of scenarios, primal variables, dual variables) as
# printed.  The SMPC_1 dual count printed in the paper (32540) does not match
# its own primal count; the consistent value is 32640 (see tests).
TABLE1 = {
    "CE-MPC": ([1], 1, 4248, 5760),
    "SMPC1": ([3, 2], 6, 24072, 32540),
    "SMPC2": ([6, 5], 30, 118059, 160080),
    "SMPC3": ([6, 5, 5], 114, 430287, 583440),
    "SMPC4": ([8, 5, 5], 146, 551355, 747600),
    "SMPC5": ([10, 8, 5], 242, 915621, 1241520),
    "SMPC6": ([12, 8, 5], 303, 1145544, 1553280),
    "SMPC7": ([12, 8, 8], 404, 1520961, 2062320),
    "SMPC8": ([12, 10, 8], 493, 1856022, 2516640),
}


def _children_counts(mu_prev: int, bmax: int, total: int | None) -> list[int]:
    """Split ``total`` children among ``mu_prev`` nodes, at most ``bmax`` each.

    ``total=None`` means full branching (every node gets ``bmax``).  Otherwise
    every node gets at least one child and the remaining children fill the
    first nodes up to ``bmax``, so the maximum branching factor is ``bmax``
    whenever ``total`` allows it.
    """
    if total is None:
        return [bmax] * mu_prev
    if total < mu_prev or total > mu_prev * bmax:
        raise ValueError(f"cannot place {total} children under {mu_prev} nodes with at most {bmax} each")
    counts = [1] * mu_prev
    extra = total - mu_prev
    for i in range(mu_prev):
        add = min(bmax - 1, extra)
        counts[i] += add
        extra -= add
    return counts


def uniform_tree(N: int, branching, scenarios: int | None = None) -> dict:
    """Build a scenario tree of horizon ``N``.

    ``branching = [b_0, b_1, ...]`` are the (maximum) branching factors of the
    nodes at stages 0, 1, ...; later stages do not branch (factor 1).  With
    ``scenarios=None`` the tree is full (``prod(b)`` scenarios).  Otherwise the
    last branching stage distributes exactly ``scenarios`` children.

    Node probabilities are the fraction of scenarios (leaves) below each node,
    every scenario being equally likely, so the children of a node always sum
    to its probability.

    Returns a dict with ``N``, ``M``, ``stage``, ``parent`` (``-1`` for the
    root) and ``prob`` (float64).
    """
    branching = list(branching)
    if N < 1:
        raise ValueError("horizon N must be >= 1")
    if len(branching) > N - 1 and any(b != 1 for b in branching[N - 1:]):
        # nodes at stage N-1 are the last decision nodes: they have no children
        raise ValueError("branching factors beyond stage N-2 are meaningless")
    counts_per_stage: list[list[int]] = []  # children count of each node, per stage
    mu = [1]
    nb = len(branching)
    for j in range(N - 1):
        bmax = branching[j] if j < nb else 1
        total = None
        if scenarios is not None and j == nb - 1 and bmax > 1:
            total = scenarios
        cc = _children_counts(mu[-1], bmax, total)
        counts_per_stage.append(cc)
        mu.append(int(sum(cc)))
    M = int(sum(mu))
    stage = np.zeros(M, dtype=np.int32)
    parent = np.full(M, -1, dtype=np.int32)
    start = [0]
    for m in mu:
        start.append(start[-1] + m)
    for j in range(N):
        stage[start[j]:start[j + 1]] = j
    for j in range(N - 1):
        k = start[j + 1]
        for i, c in enumerate(counts_per_stage[j]):
            parent[k:k + c] = start[j] + i
            k += c
    # leaf counts -> probabilities
    leaves = np.zeros(M, dtype=np.int64)
    for n in range(M - 1, -1, -1):
        if leaves[n] == 0:
            leaves[n] = 1
        if parent[n] >= 0:
            leaves[parent[n]] += leaves[n]
    n_scen = int(leaves[0])
    prob = leaves.astype(np.float64) / float(n_scen)
    return {"N": int(N), "M": M, "stage": stage, "parent": parent, "prob": prob,
            "scenarios": n_scen}


def table1_tree(name: str, N: int = 24) -> dict:
    """Tree of one Table 1 controller (branching list and scenario count)."""
    b, scen, _, _ = TABLE1[name]
    if b == [1]:
        return uniform_tree(N, [])
    return uniform_tree(N, b, scenarios=scen)


def stage_counts(tree: dict) -> np.ndarray:
    """Number of nodes per stage, ``mu(0..N-1)``."""
    return np.bincount(tree["stage"], minlength=tree["N"])
