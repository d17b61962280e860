"""Independent references used to pin the oracle (test helpers, no solver code
shared with the oracle or the library).

* ``node_kkt_solve``: the minimiser of ``<z, H'w> + f(z)`` written as one
  dense equality-constrained QP over all node variables ``(x_n, u_n)`` and
  solved through its KKT system with ``numpy.linalg.solve``.
* ``scenario_kkt_solve``: the same minimiser written per scenario (one copy of
  every variable per root-to-leaf path, scenario-probability weights, the dual
  terms of node n split in proportion ``pi_s / pi_n``) with explicit
  non-anticipativity equalities.
* ``slsqp_solve``: the full soft-constrained problem (eq. Sc-MPC) in epigraph
  form, solved by ``scipy.optimize.minimize(method="SLSQP")``.
"""

from __future__ import annotations

import numpy as np


def _as(inst):
    s, t = inst.sys, inst.tree
    return s, t, np.asarray(t["stage"]), np.asarray(t["parent"]), np.asarray(t["prob"], dtype=float)


def node_kkt_solve(inst, w: np.ndarray):
    """Dense KKT solve of argmin_z <z, H'w> + f(z) (f of eq. fz)."""
    s, t, stage, parent, prob = _as(inst)
    nx, nu, ne = s["nx"], s["nu"], s["ne"]
    M = t["M"]
    A, B, Gd, E, Ed, Wu = (np.asarray(s[k], dtype=float) for k in ("A", "B", "Gd", "E", "Ed", "Wu"))
    E = E.reshape(ne, nu)
    Ed = Ed.reshape(ne, s["nd"])
    nz = M * (nx + nu)
    xo = lambda n: n * nx                 # offset of x_n
    uo = lambda n: M * nx + n * nu        # offset of u_n
    Hq = np.zeros((nz, nz))
    c = np.zeros(nz)
    for n in range(M):
        pi = prob[n]
        a = parent[n]
        # pi (u_n - u_a)' Wu (u_n - u_a): Hessian 2 pi [Wu -Wu; -Wu Wu]
        Hq[uo(n):uo(n) + nu, uo(n):uo(n) + nu] += 2 * pi * Wu
        if a >= 0:
            Hq[uo(a):uo(a) + nu, uo(a):uo(a) + nu] += 2 * pi * Wu
            Hq[uo(n):uo(n) + nu, uo(a):uo(a) + nu] -= 2 * pi * Wu
            Hq[uo(a):uo(a) + nu, uo(n):uo(n) + nu] -= 2 * pi * Wu
        else:
            c[uo(n):uo(n) + nu] += -2 * pi * Wu @ inst.q
        c[uo(n):uo(n) + nu] += pi * s["W_alpha"] * (s["alpha1"] + inst.alpha2[stage[n]])
        c[uo(n):uo(n) + nu] += w[n, 2 * nx:]
        c[xo(n):xo(n) + nx] += w[n, :nx] + w[n, nx:2 * nx]
    rows = []
    rhs = []
    for n in range(M):
        a = parent[n]
        R = np.zeros((nx, nz))
        R[:, xo(n):xo(n) + nx] = np.eye(nx)
        R[:, uo(n):uo(n) + nu] = -B
        b = Gd @ inst.d[n]
        if a >= 0:
            R[:, xo(a):xo(a) + nx] = -A
        else:
            b = b + A @ inst.p
        rows.append(R)
        rhs.append(b)
        if ne > 0:
            R2 = np.zeros((ne, nz))
            R2[:, uo(n):uo(n) + nu] = E
            rows.append(R2)
            rhs.append(-Ed @ inst.d[n])
    C = np.vstack(rows)
    b = np.concatenate(rhs)
    m = C.shape[0]
    K = np.block([[Hq, C.T], [C, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-c, b]))
    z = sol[:nz]
    x = z[:M * nx].reshape(M, nx)
    u = z[M * nx:].reshape(M, nu)
    return x, u


def scenario_paths(tree) -> list[list[int]]:
    parent = np.asarray(tree["parent"])
    M = tree["M"]
    has_child = np.zeros(M, dtype=bool)
    has_child[parent[parent >= 0]] = True
    paths = []
    for leaf in np.flatnonzero(~has_child):
        path = [int(leaf)]
        while parent[path[-1]] >= 0:
            path.append(int(parent[path[-1]]))
        paths.append(path[::-1])
    return paths


def scenario_kkt_solve(inst, w: np.ndarray):
    """Scenario-form KKT: per-scenario copies + non-anticipativity."""
    s, t, stage, parent, prob = _as(inst)
    nx, nu, ne = s["nx"], s["nu"], s["ne"]
    A, B, Gd, E, Ed, Wu = (np.asarray(s[k], dtype=float) for k in ("A", "B", "Gd", "E", "Ed", "Wu"))
    E = E.reshape(ne, nu)
    Ed = Ed.reshape(ne, s["nd"])
    paths = scenario_paths(t)
    S = len(paths)
    N = t["N"]
    assert all(len(pth) == N for pth in paths)
    nvar_s = N * (nx + nu)
    nz = S * nvar_s
    xo = lambda sc, j: sc * nvar_s + j * nx
    uo = lambda sc, j: sc * nvar_s + N * nx + j * nu
    pis = np.array([prob[pth[-1]] for pth in paths])
    Hq = np.zeros((nz, nz))
    c = np.zeros(nz)
    for sc, pth in enumerate(paths):
        ps = pis[sc]
        for j, n in enumerate(pth):
            Hq[uo(sc, j):uo(sc, j) + nu, uo(sc, j):uo(sc, j) + nu] += 2 * ps * Wu
            if j > 0:
                Hq[uo(sc, j - 1):uo(sc, j - 1) + nu, uo(sc, j - 1):uo(sc, j - 1) + nu] += 2 * ps * Wu
                Hq[uo(sc, j):uo(sc, j) + nu, uo(sc, j - 1):uo(sc, j - 1) + nu] -= 2 * ps * Wu
                Hq[uo(sc, j - 1):uo(sc, j - 1) + nu, uo(sc, j):uo(sc, j) + nu] -= 2 * ps * Wu
            else:
                c[uo(sc, j):uo(sc, j) + nu] += -2 * ps * Wu @ inst.q
            c[uo(sc, j):uo(sc, j) + nu] += ps * s["W_alpha"] * (s["alpha1"] + inst.alpha2[j])
            share = ps / prob[n]
            c[uo(sc, j):uo(sc, j) + nu] += share * w[n, 2 * nx:]
            c[xo(sc, j):xo(sc, j) + nx] += share * (w[n, :nx] + w[n, nx:2 * nx])
    rows, rhs = [], []
    first_owner = {}
    for sc, pth in enumerate(paths):
        for j, n in enumerate(pth):
            R = np.zeros((nx, nz))
            R[:, xo(sc, j):xo(sc, j) + nx] = np.eye(nx)
            R[:, uo(sc, j):uo(sc, j) + nu] = -B
            b = Gd @ inst.d[n]
            if j > 0:
                R[:, xo(sc, j - 1):xo(sc, j - 1) + nx] = -A
            else:
                b = b + A @ inst.p
            rows.append(R)
            rhs.append(b)
            if n not in first_owner:
                first_owner[n] = sc
                if ne > 0:
                    R2 = np.zeros((ne, nz))
                    R2[:, uo(sc, j):uo(sc, j) + nu] = E
                    rows.append(R2)
                    rhs.append(-Ed @ inst.d[n])
            else:
                s0 = first_owner[n]
                R3 = np.zeros((nu, nz))
                R3[:, uo(sc, j):uo(sc, j) + nu] = np.eye(nu)
                R3[:, uo(s0, j):uo(s0, j) + nu] = -np.eye(nu)
                rows.append(R3)
                rhs.append(np.zeros(nu))
    C = np.vstack(rows)
    b = np.concatenate(rhs)
    m = C.shape[0]
    K = np.block([[Hq, C.T], [C, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-c, b]))
    z = sol[:nz]
    M = t["M"]
    x = np.full((M, nx), np.nan)
    u = np.full((M, nu), np.nan)
    xs_all = {}
    for sc, pth in enumerate(paths):
        for j, n in enumerate(pth):
            xv = z[xo(sc, j):xo(sc, j) + nx]
            uv = z[uo(sc, j):uo(sc, j) + nu]
            xs_all.setdefault(n, []).append((xv, uv))
    spread = 0.0
    for n, lst in xs_all.items():
        x[n] = lst[0][0]
        u[n] = lst[0][1]
        for xv, uv in lst[1:]:
            spread = max(spread, np.max(np.abs(xv - x[n])), np.max(np.abs(uv - u[n])))
    return x, u, spread


def slsqp_solve(inst, maxiter: int = 2000):
    """Full soft-constrained problem in epigraph form, solved by SLSQP.

    Variables ``(x_n, u_n, r^S_n, r^d_n, s^S_n, s^d_n)``:
    ``r^S >= xs - x, r^S >= 0`` (componentwise excess below the safety level),
    ``r^d >= x - xmax, r^d >= xmin - x, r^d >= 0``, ``s >= 0`` and
    ``s^2 >= ||r||^2`` so that ``s`` is the Euclidean distance at the optimum.
    Objective: the expected stage cost plus ``cS_n s^S_n + cd_n s^d_n``.
    """
    from scipy.optimize import minimize

    s, t, stage, parent, prob = _as(inst)
    nx, nu, ne = s["nx"], s["nu"], s["ne"]
    M = t["M"]
    A, B, Gd, E, Ed, Wu = (np.asarray(s[k], dtype=float) for k in ("A", "B", "Gd", "E", "Ed", "Wu"))
    E = E.reshape(ne, nu)
    Ed = Ed.reshape(ne, s["nd"])
    cS = s["W_x"] * prob if s.get("weight_safety_by_prob", 1) else np.full(M, s["W_x"])
    cd = np.full(M, s["gamma_d"])
    per = nx + nu + 2 * nx + 2
    ox = lambda n: n * per
    ou = lambda n: n * per + nx
    orS = lambda n: n * per + nx + nu
    ord_ = lambda n: n * per + 2 * nx + nu
    osS = lambda n: n * per + 3 * nx + nu
    osd = lambda n: n * per + 3 * nx + nu + 1
    nz = M * per

    def obj(z):
        f = 0.0
        g = np.zeros(nz)
        for n in range(M):
            u = z[ou(n):ou(n) + nu]
            a = parent[n]
            ua = inst.q if a < 0 else z[ou(a):ou(a) + nu]
            du = u - ua
            lin = prob[n] * s["W_alpha"] * (s["alpha1"] + inst.alpha2[stage[n]])
            f += lin @ u + prob[n] * du @ Wu @ du
            g[ou(n):ou(n) + nu] += lin + 2 * prob[n] * Wu @ du
            if a >= 0:
                g[ou(a):ou(a) + nu] -= 2 * prob[n] * Wu @ du
            f += cS[n] * z[osS(n)] + cd[n] * z[osd(n)]
            g[osS(n)] += cS[n]
            g[osd(n)] += cd[n]
        return f, g

    eqs = []
    for n in range(M):
        a = parent[n]

        def dyn(z, n=n, a=a):
            xa = inst.p if a < 0 else z[ox(a):ox(a) + nx]
            return z[ox(n):ox(n) + nx] - A @ xa - B @ z[ou(n):ou(n) + nu] - Gd @ inst.d[n]

        eqs.append({"type": "eq", "fun": dyn})
        if ne > 0:
            eqs.append({"type": "eq", "fun": lambda z, n=n: E @ z[ou(n):ou(n) + nu] + Ed @ inst.d[n]})
    ineqs = []
    for n in range(M):
        def ineq(z, n=n):
            x = z[ox(n):ox(n) + nx]
            rS = z[orS(n):orS(n) + nx]
            rd = z[ord_(n):ord_(n) + nx]
            sS, sd = z[osS(n)], z[osd(n)]
            return np.concatenate([rS - (np.asarray(s["xs"]) - x), rS,
                                   rd - (x - np.asarray(s["xmax"])), rd - (np.asarray(s["xmin"]) - x), rd,
                                   [sS, sd, sS * sS - rS @ rS, sd * sd - rd @ rd]])
        ineqs.append({"type": "ineq", "fun": ineq})
    bounds = []
    for n in range(M):
        bounds += [(None, None)] * nx
        bounds += list(zip(np.asarray(s["umin"]), np.asarray(s["umax"])))
        bounds += [(0, None)] * (2 * nx + 2)
    z0 = np.zeros(nz)
    for n in range(M):
        z0[ou(n):ou(n) + nu] = np.clip(inst.q, s["umin"], s["umax"])
        z0[osS(n)] = z0[osd(n)] = 1.0
        z0[orS(n):orS(n) + nx] = 0.5
        z0[ord_(n):ord_(n) + nx] = 0.5
    res = minimize(lambda z: obj(z), z0, jac=True, method="SLSQP", constraints=eqs + ineqs,
                   bounds=bounds, options={"maxiter": maxiter, "ftol": 1e-14})
    z = res.x
    x = np.array([z[ox(n):ox(n) + nx] for n in range(M)])
    u = np.array([z[ou(n):ou(n) + nu] for n in range(M)])
    return x, u, res
