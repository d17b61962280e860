"""Closed loop of Alg. 2 over the C ABI.

Per step: the tree's new demands and pumping costs go to the device, where
the cost update of App. A runs (``smpc_tree_set_data``); the tree is solved
(``smpc_solve``, cold or warm from its shifted resident dual); ``u0`` is
applied to the plant with the realised root demand (``smpc_plant_step``) and
becomes the next previous input.  ``smpc_closed_loop_kpi`` evaluates the run
(Sec. V-B).  Marshalling only: every computation is a library call.
"""

from __future__ import annotations

import time

import numpy as np

from . import smpc as S


def run(tree, x0, q0, steps, *, warm: bool = False, realized=None, keep_y: bool = False, **solve_kw) -> dict:
    """Simulate ``len(steps)`` closed-loop steps of ``tree`` (a
    :class:`solver.Tree`, factored once: the step size does not depend on the
    data).  ``steps[k] = (d, alpha2)`` are the tree's node demands (M, nd) and
    pumping costs (N, nu) at step k; the realised demand is the root's
    ``d[0]``.  ``realized(k)`` picks the root child the warm start of step
    k + 1 follows (default 0).  Returns the applied inputs ``u`` (Hs, nu),
    the states ``x`` (Hs, nx) they lead to, per-step iterations, status,
    primal residual ``||Hz - t||_inf`` and wall time (with ``gap=True`` in
    ``solve_kw`` also each step's cost and duality gap, the a-posteriori
    check of Sec. IV-E), and the KPIs (with ``keep_y`` also each step's
    final dual ``y``)."""
    sysh = tree.system.h
    x = np.asarray(x0, dtype=np.float64).copy()
    q = np.asarray(q0, dtype=np.float64).copy()
    us, xs, its, st, secs, ys = [], [], [], [], [], []
    res, costs, gaps = [], [], []
    for k, (d, a2) in enumerate(steps):
        t0 = time.perf_counter()
        tree.set_data(d, a2)
        use_warm = warm and k > 0
        if use_warm:
            tree.shift_warm_start(0 if realized is None else int(realized(k - 1)))
        r = tree.solve(x, q, want_x=False, want_y=keep_y, resident=use_warm, **solve_kw)
        if keep_y:
            ys.append(r["y"])
        u0 = r["u0"]
        x = S.smpc_plant_step(sysh, x, u0, np.asarray(d)[0])
        secs.append(time.perf_counter() - t0)
        us.append(u0)
        xs.append(x.copy())
        its.append(r["iterations"])
        st.append(r["status"])
        res.append(r["hz_t_max"])
        if solve_kw.get("gap"):
            costs.append(r["cost"])
            gaps.append(r["gap"])
        q = u0
    u_arr, x_arr = np.array(us), np.array(xs)
    a2_arr = np.array([np.asarray(a2)[0] for _, a2 in steps])
    kpi = S.smpc_closed_loop_kpi(sysh, u_arr, x_arr, a2_arr, np.asarray(q0, dtype=np.float64))
    out = {"u": u_arr, "x": x_arr, "iterations": its, "status": st, "hz_t_max": res, "seconds": secs, "kpi": kpi}
    if gaps:
        out["cost"], out["gap"] = costs, gaps
    if keep_y:
        out["y"] = ys
    return out
