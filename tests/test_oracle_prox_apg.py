"""Pins of the oracle's prox (App. C), theta recursion, step size (Sec. IV-D)
and of the APG iteration itself (eq. apg-iteration)."""

import math

import numpy as np
import pytest
from scipy.optimize import minimize

import dwn_synth as ds
import oracle as O
from tests.kkt_reference import node_kkt_solve, slsqp_solve


# ---------------------------------------------------------------- prox

def _brute_prox(s, dist, tau):
    obj = lambda t: tau * dist(t) + 0.5 * np.sum((t - s) ** 2)
    best = None
    for x0 in (s, s + 0.1, s - 0.1):
        r = minimize(obj, x0, method="Nelder-Mead",
                     options={"xatol": 1e-11, "fatol": 1e-14, "maxiter": 40000, "maxfev": 40000})
        if best is None or r.fun < best.fun:
            best = r
    return best.x


@pytest.mark.parametrize("seed", range(6))
def test_prox_distance_brute_force_and_optimality(seed):
    rng = np.random.default_rng(seed)
    n = 3
    lo = rng.uniform(-1, 0, n)
    hi = lo + rng.uniform(0.5, 2, n)
    proj_box = lambda a: np.clip(a, lo, hi)
    xs = rng.uniform(-0.5, 0.5, n)
    proj_half = lambda a: np.maximum(a, xs)
    for proj in (proj_box, proj_half):
        for scale in (0.2, 1.0, 3.0):
            s = rng.standard_normal(n) * 2 * scale
            tau = rng.uniform(0.05, 1.5)
            t = O.prox_dist(s[None, :], lambda a: proj(a), tau)[0]
            dist = lambda v: np.linalg.norm(v - proj(v))
            tb = _brute_prox(s, dist, tau)
            assert np.abs(t - tb).max() < 1e-5
            # exact optimality: (s - t) / tau is a subgradient of dist at t
            g = (s - t) / tau
            dt = dist(t)
            if dt > 1e-12:
                assert np.allclose(g, (t - proj(t)) / dt, atol=1e-12)
            else:
                assert np.linalg.norm(g) <= 1 + 1e-12
                # normal cone of C at t: g . (c - t) <= 0 for points c of C
                for _ in range(20):
                    c = proj(rng.standard_normal(n) * 3)
                    assert g @ (c - t) <= 1e-10


def test_prox_g_blocks_and_scaling():
    inst = ds.tiny_instance()
    P = O.OracleProblem.from_instance(inst)
    rng = np.random.default_rng(0)
    v = rng.standard_normal((P.M, P.dual_dim)) * 5
    gamma = 0.01
    t = O.prox_g(P, v, gamma)
    nx = P.nx
    assert np.allclose(t[:, 2 * nx:], np.clip(v[:, 2 * nx:], P.umin, P.umax))
    for n in range(P.M):
        ts = O.prox_dist(v[n:n + 1, :nx], lambda a: np.maximum(a, P.xs), gamma * P.W_x * P.prob[n])
        tz = O.prox_dist(v[n:n + 1, nx:2 * nx], lambda a: np.clip(a, P.xmin, P.xmax), gamma * P.gamma_d)
        assert np.allclose(t[n, :nx], ts[0]) and np.allclose(t[n, nx:2 * nx], tz[0])
    # scaled prox of g(S^-1 .): brute force on one node, one block
    S = rng.uniform(0.3, 2.0, (P.M, 3))
    ts = O.prox_g(P, v, gamma, S)
    n = 3
    s1 = S[n, 0]
    dist = lambda a: np.linalg.norm(a - np.maximum(a, P.xs))
    obj = lambda tt: gamma * P.W_x * P.prob[n] * dist(tt / s1) + 0.5 * np.sum((tt - v[n, :nx]) ** 2)
    r = minimize(obj, v[n, :nx], method="Nelder-Mead", options={"xatol": 1e-11, "fatol": 1e-14, "maxiter": 40000})
    assert np.abs(ts[n, :nx] - r.x).max() < 1e-5


# ---------------------------------------------------------------- theta

def test_theta_recursion():
    th = O.theta_sequence(2000)
    assert th[0] == 1.0
    assert abs(th[1] - (math.sqrt(5) - 1) / 2) < 1e-15
    k = np.arange(1999)
    inv = (1 - th[1:]) / th[1:] ** 2
    assert np.allclose(inv, 1 / th[:-1] ** 2, rtol=1e-12)
    # theta_k ~ 2 / (k + 2)
    assert np.all(th[1:] <= 2.0 / (k + 2) + 1e-15)
    assert np.all(th[1:] >= 1.0 / (k + 2))


# ---------------------------------------------------------------- step size

def test_dual_hessian_closed_form_single_node():
    """One node, no coupling: z_lin(w) solves min (u'Wu u) + w'Hz with
    x = B u, so the dual Hessian is G Wu^{-1} G' / 2, G = [B; B; I]."""
    inst = ds.random_small_instance(5, nx=3, nu=4, nd=2, ne=0, N=1, branching=())
    P = O.OracleProblem.from_instance(inst)
    K = O.dual_hessian_dense(P)
    G = np.vstack([P.B, P.B, np.eye(P.nu)])
    Kc = G @ np.linalg.solve(P.Wu, G.T) / 2.0
    assert np.allclose(K, Kc, atol=1e-12 * np.abs(Kc).max())


@pytest.mark.parametrize("scaled", [False, True])
def test_dual_lmax_dense_vs_power(scaled):
    inst = ds.random_small_instance(6, N=3, branching=(2, 2))
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    S = np.repeat(np.sqrt(P.prob)[:, None], 3, 1) if scaled else None
    K = O.dual_hessian_dense(P, F, S)
    assert np.abs(K - K.T).max() <= 1e-10 * np.abs(K).max()
    ev = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert ev[0] >= -1e-9 * ev[-1]
    lp = O.dual_lmax_power(P, 2000, F, S)
    assert abs(lp - ev[-1]) <= 1e-8 * ev[-1]


# ---------------------------------------------------------------- APG

def _lam(P, F, S=None):
    K = O.dual_hessian_dense(P, F, S)
    return 1.0 / np.linalg.eigvalsh(0.5 * (K + K.T))[-1]


def test_apg_zero_dual_special_case():
    """No soft penalties and an inactive input box: g is the indicator of a
    box that never binds, so y* = 0 and the first iterate is already the
    unconstrained minimiser (dense KKT at w = 0)."""
    inst = ds.random_small_instance(10, N=3, branching=(2, 2))
    inst.sys["W_x"] = 0.0
    inst.sys["gamma_d"] = 0.0
    inst.sys["umin"] = -1e6 * np.ones(inst.sys["nu"])
    inst.sys["umax"] = 1e6 * np.ones(inst.sys["nu"])
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    r = O.apg(P, 1e-3, 5, F)
    xk, uk = node_kkt_solve(inst, np.zeros((P.M, P.dual_dim)))
    assert np.abs(r.y).max() == 0.0
    assert r.r_primal == 0.0
    assert np.abs(r.u - uk).max() < 1e-10 * max(1, np.abs(uk).max())
    assert np.abs(r.x - xk).max() < 1e-10 * max(1, np.abs(xk).max())


def _dual_objective(P, F, y):
    """D(y) = f*(-H'y) + g*(y) from the definitions of the conjugates:
    f*(-H'y) = -(<z(y), H'y> + f(z(y))) and g* = support functions of the
    sets (distance terms: support function on the ball of radius c)."""
    x, u = O.solve_step(P, F, y)
    nx = P.nx
    hy = np.sum(y * O.smpc_oracle.hz(x, u))
    fz = 0.0
    for n in range(P.M):
        a = P.parent[n]
        ua = P.q if a < 0 else u[a]
        du = u[n] - ua
        fz += P.prob[n] * (P.W_alpha * (P.alpha1 + P.alpha2[P.stage[n]]) @ u[n] + du @ P.Wu @ du)
    ys, yz, yp = y[:, :nx], y[:, nx:2 * nx], y[:, 2 * nx:]
    gs = np.sum(ys * P.xs)                                   # y_s <= 0 on dom
    gz = np.sum(np.maximum(yz * P.xmax, yz * P.xmin))
    gp = np.sum(np.maximum(yp * P.umax, yp * P.umin))
    infeas = max(np.max(ys), np.max(np.linalg.norm(ys, axis=1) - P.safety_weight()),
                 np.max(np.linalg.norm(yz, axis=1) - P.box_weight()))
    return -(hy + fz) + gs + gz + gp, infeas


@pytest.fixture(scope="module")
def tiny_long_run():
    inst = ds.tiny_instance()
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    S = np.repeat(np.sqrt(P.prob)[:, None], 3, 1)
    lam = _lam(P, F, S)
    r = O.apg(P, lam, 20000, F, scale=S)
    return inst, P, F, S, lam, r


def test_apg_kkt_certificate(tiny_long_run):
    """After 20k FP64 iterations the iterate satisfies the optimality system
    of eq. sc_prox: Hz = t, y in dg(t), z = z(y)."""
    inst, P, F, S, lam, r = tiny_long_run
    assert r.r_primal <= 2e-6
    zx, zu = O.solve_step(P, F, r.y)
    assert np.abs(zx - r.x).max() <= 1e-5 and np.abs(zu - r.u).max() <= 1e-5
    nx = P.nx
    ys, yz, yp = r.y[:, :nx], r.y[:, nx:2 * nx], r.y[:, 2 * nx:]
    ts, tz, tp = r.t[:, :nx], r.t[:, nx:2 * nx], r.t[:, 2 * nx:]
    # psi block: normal cone of the input box
    inner = (tp > P.umin + 1e-9) & (tp < P.umax - 1e-9)
    assert np.abs(yp[inner]).max(initial=0) <= 1e-9
    assert np.all(yp[np.isclose(tp, P.umin)] <= 1e-9)
    assert np.all(yp[np.isclose(tp, P.umax)] >= -1e-9)
    # distance blocks: y = c (t - P(t)) / ||t - P(t)|| outside, |y| <= c inside
    for yb, tb, proj, c in ((ys, ts, lambda a: np.maximum(a, P.xs), P.safety_weight()),
                            (yz, tz, lambda a: np.clip(a, P.xmin, P.xmax), P.box_weight())):
        for n in range(P.M):
            dvec = tb[n] - proj(tb[n:n + 1])[0]
            dn = np.linalg.norm(dvec)
            if dn > 1e-9:
                assert np.allclose(yb[n], c[n] * dvec / dn, atol=1e-7 * c[n])
            else:
                assert np.linalg.norm(yb[n]) <= c[n] * (1 + 1e-9)
    # independent check of the optimum: SLSQP on the epigraph form
    xq, uq, res = slsqp_solve(inst)
    cost_apg = O.primal_cost(P, r.x, r.u)
    cost_ref = O.primal_cost(P, xq, uq)
    assert abs(cost_apg - cost_ref) <= 1e-5 * abs(cost_ref)
    assert np.abs(r.u - uq).max() <= 2e-3


def test_apg_fista_bound(tiny_long_run):
    """Beck-Teboulle bound for this theta recursion:
    D(y^k) - D* <= 2 L ||y^0 - y*||^2 / (k + 1)^2."""
    inst, P, F, S, lam, _ = tiny_long_run
    # unscaled run so that the bound is in the plain dual norm
    lamu = _lam(P, F)
    ref = O.apg(P, lamu, 20000, F)
    dstar = min(_dual_objective(P, F, ref.y)[0], _dual_objective(P, F, ref.y_prev)[0])
    ystar = ref.y
    r = O.apg(P, lamu, 1500, F, record=True)
    L = 1.0 / lamu
    R2 = np.sum(ystar ** 2)
    for k, h in enumerate(r.history, start=1):
        if k % 25 and k > 30:
            continue
        dk, infeas = _dual_objective(P, F, h["y"])
        assert infeas <= 1e-9 * max(P.W_x, P.gamma_d)
        assert dk - dstar <= 2 * L * R2 / (k + 1) ** 2 * (1 + 1e-9) + 1e-9 * abs(dstar)


def test_apg_ergodic_residual_rate():
    """The ergodic primal iterate has an O(1/nu^2) primal residual: the
    product (nu+1)^2 ||H zbar - tbar||_inf stays bounded."""
    inst = ds.tiny_instance()
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    lam = _lam(P, F)
    vals = []
    for k in (100, 200, 400, 800, 1600):
        r = O.apg(P, lam, k, F, ergodic=True)
        rb = np.max(np.abs(O.smpc_oracle.hz(r.xbar, r.ubar) - r.tbar))
        vals.append((k + 1) ** 2 * rb)
    assert max(vals[1:]) <= 4.0 * vals[0]


def test_apg_matches_plain_fista_on_stacked_dual():
    """The APG equals FISTA written directly on the dual: gradient of
    f*(-H'y) is -H z(y), the prox of lambda g* follows from Moreau."""
    inst = ds.random_small_instance(12, N=3, branching=(2, 1))
    P = O.OracleProblem.from_instance(inst)
    F = O.factor_step(P)
    lam = _lam(P, F)
    r = O.apg(P, lam, 60, F)
    y = np.zeros((P.M, P.dual_dim))
    yp = y.copy()
    tk = 1.0
    tkm = 1.0
    for _ in range(60):
        w = y + ((tkm - 1) / tk) * (y - yp)
        x, u = O.solve_step(P, F, w)
        grad = -O.smpc_oracle.hz(x, u)
        v = w - lam * grad
        ynew = v - lam * O.prox_g(P, v / lam, 1.0 / lam)
        yp, y = y, ynew
        tkm, tk = tk, (1 + math.sqrt(1 + 4 * tk * tk)) / 2
    assert np.abs(y - r.y).max() <= 1e-9 * max(1, np.abs(y).max())
