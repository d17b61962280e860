"""Plain FP64 NumPy oracle of the APG solver for scenario-tree SMPC.

TEST INFRASTRUCTURE ONLY (see the package docstring): slow, obviously-correct
code that follows the paper's steps in its own order and notation.  Nothing in
the GPU library imports or calls it.

Notation (decision-node convention).  Nodes ``n = 0..M-1`` are stage-sorted;
node ``n`` at stage ``s(n)`` carries demand ``d_n``, input ``u_n`` and the
resulting state ``x_n`` (the paper's ``x_{s(n)+1}``), probability ``pi_n``
(the paper's ``p_j^i``) and parent ``a(n)`` (the paper's ``anc``).  The root's
parent quantities are ``x_{a(root)} = p``, ``u_{a(root)} = q`` and
``v_{a(root)} = 0`` (Alg. 1 initialisation; eq. Sc-MPC).

Problem (eq. Sc-MPC with the splitting of Sec. IV-A, eq. fz and eq. gzeta):

    f(z) = sum_n pi_n [ W_a (a1 + a2_{s(n)})' u_n + (u_n - u_a)' Wu (u_n - u_a) ]
           + indicator(E u_n + Ed d_n = 0) + indicator(x_n = A x_a + B u_n + Gd d_n)
    g(t) = sum_n [ cS_n dist(sigma_n | x >= xs) + cd_n dist(zeta_n | [xmin, xmax])
                   + indicator(psi_n in [umin, umax]) ]
    H z  = (x_n, x_n, u_n) per node

with ``cS_n = W_x pi_n`` (or ``W_x`` if ``weight_safety_by_prob`` is 0) and
``cd_n = gamma_d``.  The dual vector holds one block ``(sigma~_n, zeta~_n,
psi~_n)`` of size ``2 nx + nu`` per node.

Readings taken where the paper is ambiguous (each is also listed in the design
notes): decision-node indexing; ``xi_n = sigma~_n + zeta~_n`` (the ``H'w``
state part); ``Psi = Lambda L'`` (the printed ``Lambda L`` does not conform);
the prox of ``c dist_C`` with parameter ``1/lambda`` moves the point by
``min(1, tau/delta)`` towards its projection, ``tau = c/lambda``; ``beta`` as
re-derived from the expansion of the smoothing cost in App. A (the printed
factorisation multiplies every term by ``p``).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# ---------------------------------------------------------------------------
# problem container
# ---------------------------------------------------------------------------

@dataclass
class OracleProblem:
    """All inputs of one scenario-tree problem, as float64 numpy arrays."""

    nx: int
    nu: int
    nd: int
    ne: int
    A: np.ndarray
    B: np.ndarray
    Gd: np.ndarray
    E: np.ndarray
    Ed: np.ndarray
    umin: np.ndarray
    umax: np.ndarray
    xmin: np.ndarray
    xmax: np.ndarray
    xs: np.ndarray
    W_alpha: float
    alpha1: np.ndarray
    Wu: np.ndarray
    W_x: float
    gamma_d: float
    weight_safety_by_prob: int
    N: int
    stage: np.ndarray
    parent: np.ndarray
    prob: np.ndarray
    d: np.ndarray
    alpha2: np.ndarray
    p: np.ndarray
    q: np.ndarray

    @classmethod
    def from_parts(cls, sys: dict, tree: dict, d, alpha2, p, q) -> "OracleProblem":
        f = lambda a: np.array(a, dtype=np.float64, copy=True)
        return cls(
            nx=int(sys["nx"]), nu=int(sys["nu"]), nd=int(sys["nd"]), ne=int(sys["ne"]),
            A=f(sys["A"]), B=f(sys["B"]), Gd=f(sys["Gd"]),
            E=f(sys["E"]).reshape(int(sys["ne"]), int(sys["nu"])),
            Ed=f(sys["Ed"]).reshape(int(sys["ne"]), int(sys["nd"])),
            umin=f(sys["umin"]), umax=f(sys["umax"]), xmin=f(sys["xmin"]), xmax=f(sys["xmax"]),
            xs=f(sys["xs"]), W_alpha=float(sys["W_alpha"]), alpha1=f(sys["alpha1"]), Wu=f(sys["Wu"]),
            W_x=float(sys["W_x"]), gamma_d=float(sys["gamma_d"]),
            weight_safety_by_prob=int(sys.get("weight_safety_by_prob", 1)),
            N=int(tree["N"]), stage=np.array(tree["stage"], dtype=np.int64),
            parent=np.array(tree["parent"], dtype=np.int64), prob=f(tree["prob"]),
            d=f(d), alpha2=f(alpha2), p=f(p), q=f(q),
        )

    @classmethod
    def from_instance(cls, inst) -> "OracleProblem":
        return cls.from_parts(inst.sys, inst.tree, inst.d, inst.alpha2, inst.p, inst.q)

    @property
    def M(self) -> int:
        return int(self.stage.shape[0])

    @property
    def dual_dim(self) -> int:
        return 2 * self.nx + self.nu

    def children(self) -> list[list[int]]:
        ch: list[list[int]] = [[] for _ in range(self.M)]
        for n in range(self.M):
            if self.parent[n] >= 0:
                ch[int(self.parent[n])].append(n)
        return ch

    def stage_nodes(self) -> list[np.ndarray]:
        return [np.flatnonzero(self.stage == j) for j in range(self.N)]

    def safety_weight(self) -> np.ndarray:
        """Per-node weight ``cS_n`` of the safety distance."""
        if self.weight_safety_by_prob:
            return self.W_x * self.prob
        return np.full(self.M, self.W_x)

    def box_weight(self) -> np.ndarray:
        """Per-node weight ``cd_n`` of the soft state-box distance."""
        return np.full(self.M, self.gamma_d)


# ---------------------------------------------------------------------------
# App. A: elimination of the input-disturbance coupling (cost update)
# ---------------------------------------------------------------------------

def null_space_basis(E: np.ndarray, nu: int) -> np.ndarray:
    """Full-rank ``L`` (nu x nv) whose range is the kernel of ``E`` (App. A,
    eq. new:decision).  Orthonormal columns, taken from the SVD."""
    if E.shape[0] == 0:
        return np.eye(nu)
    _, s, vt = np.linalg.svd(E)
    tol = max(E.shape) * np.finfo(float).eps * (s[0] if s.size else 0.0)
    rank = int((s > tol).sum())
    return vt[rank:].T.copy()


@dataclass
class CostUpdate:
    """Output of App. A for one tree: ``L, uhat_n, e_n, Bbar, Rhat, Rbar,
    alphabar_j, beta_n``."""

    L: np.ndarray
    uhat: np.ndarray
    e: np.ndarray
    Bbar: np.ndarray
    Rhat: np.ndarray
    Rbar: np.ndarray
    alphabar: np.ndarray
    beta: np.ndarray


def cost_update(P: OracleProblem, L: np.ndarray | None = None) -> CostUpdate:
    """App. A.

    * ``u = L v + uhat(d)`` with ``E uhat + Ed d = 0``; ``uhat`` is the
      minimum-norm particular solution (pseudo-inverse of ``E``).
    * ``Bbar = B L``, ``e_n = B uhat_n + Gd d_n`` (eq. appendix:dist).
    * ``Rhat = Wu L``, ``Rbar = L' Rhat``, ``alphabar_j = W_a L'(a1 + a2_j)``.
    * ``beta_n`` is the coefficient of ``v_n`` left over when the smoothing
      cost ``pi_n (L dv_n + duhat_n)' Wu (L dv_n + duhat_n)`` and the linear
      cost are expanded and regrouped per node (eq. new:stage:cost):

        beta_n = pi_n alphabar_{s(n)}
                 + 2 Rhat' ( pibar_n uhat_n - pi_n uhat_{a(n)} - sum_c pi_c uhat_c ),
        pibar_n = pi_n + sum_c pi_c,     uhat_{a(root)} = q.
    """
    if L is None:
        L = null_space_basis(P.E, P.nu)
    M = P.M
    if P.ne > 0:
        uhat = -(np.linalg.pinv(P.E) @ (P.Ed @ P.d.T)).T
    else:
        uhat = np.zeros((M, P.nu))
    Bbar = P.B @ L
    e = uhat @ P.B.T + P.d @ P.Gd.T
    Rhat = P.Wu @ L
    Rbar = L.T @ Rhat
    alphabar = np.array([P.W_alpha * (L.T @ (P.alpha1 + P.alpha2[j])) for j in range(P.N)])
    ch = P.children()
    beta = np.zeros((M, L.shape[1]))
    for n in range(M):
        pi_n = P.prob[n]
        a = int(P.parent[n])
        u_par = P.q if a < 0 else uhat[a]
        pibar = pi_n + sum(P.prob[c] for c in ch[n])
        s_ch = np.zeros(P.nu)
        for c in ch[n]:
            s_ch += P.prob[c] * uhat[c]
        beta[n] = pi_n * alphabar[P.stage[n]] + 2.0 * Rhat.T @ (pibar * uhat[n] - pi_n * u_par - s_ch)
    return CostUpdate(L=L, uhat=uhat, e=e, Bbar=Bbar, Rhat=Rhat, Rbar=Rbar, alphabar=alphabar, beta=beta)


# ---------------------------------------------------------------------------
# App. B: factor step
# ---------------------------------------------------------------------------

@dataclass
class Factor:
    """Everything Alg. 1 needs: cost-update vectors plus ``Lambda, Phi, Psi``."""

    cu: CostUpdate
    Lambda: np.ndarray
    Phi: np.ndarray
    Psi: np.ndarray


def factor_step(P: OracleProblem, cu: CostUpdate | None = None) -> Factor:
    """App. B, eq. optimal matrices control: ``Lambda = -Rbar^{-1}`` through a
    Cholesky factorisation of ``Rbar``, ``Phi = Lambda Bbar'``, ``Psi = Lambda L'``."""
    if cu is None:
        cu = cost_update(P)
    C = np.linalg.cholesky(cu.Rbar)
    nv = cu.Rbar.shape[0]
    Rinv = np.linalg.solve(C.T, np.linalg.solve(C, np.eye(nv)))
    Lam = -Rinv
    return Factor(cu=cu, Lambda=Lam, Phi=Lam @ cu.Bbar.T, Psi=Lam @ cu.L.T)


# ---------------------------------------------------------------------------
# Alg. 1: solve step  z(w) = argmin <z, H'w> + f(z)
# ---------------------------------------------------------------------------

def solve_step(P: OracleProblem, F: Factor, w: np.ndarray, affine: bool = True):
    """Alg. 1 (with the dynamic-programming recursion of App. B).

    ``w`` is the dual point, ``(M, 2nx+nu)``.  Backward over stages
    ``N-1 .. 0``: for each node ``l`` with accumulated child terms
    ``q_l`` (state) and ``r_l`` (input),

        sigma_l = r_l + beta_l
        dv_l    = (Phi (xi_l + q_l) + Psi psi~_l + Lambda sigma_l) / (2 pi_l)
        r_{a(l)} += sigma_l + Bbar' (xi_l + q_l) + L' psi~_l
        q_{a(l)} += A' (xi_l + q_l)

    then forward over stages ``0 .. N-1``: ``v_l = v_{a(l)} + dv_l``,
    ``u_l = L v_l + uhat_l``, ``x_l = A x_{a(l)} + Bbar v_l + e_l``.

    With ``affine=False`` every term that does not depend on ``w`` is dropped
    (``beta, uhat, e, p`` set to zero): this is the linear part of the map,
    used for the dual Hessian.  Returns ``(x, u)``, each ``(M, n)``.
    """
    cu = F.cu
    nx, nu = P.nx, P.nu
    M = P.M
    nv = cu.L.shape[1]
    xi = w[:, :nx] + w[:, nx:2 * nx]
    psi = w[:, 2 * nx:]
    beta = cu.beta if affine else np.zeros_like(cu.beta)
    qacc = np.zeros((M, nx))
    racc = np.zeros((M, nv))
    dv = np.zeros((M, nv))
    stages = P.stage_nodes()
    for j in range(P.N - 1, -1, -1):
        idx = stages[j]
        qx = xi[idx] + qacc[idx]                      # xi_l + q_{j+1}^l
        sigma = racc[idx] + beta[idx]
        dv[idx] = (qx @ F.Phi.T + psi[idx] @ F.Psi.T + sigma @ F.Lambda.T) / (2.0 * P.prob[idx])[:, None]
        if j > 0:
            par = P.parent[idx]
            np.add.at(qacc, par, qx @ P.A)            # A' (xi + q)
            np.add.at(racc, par, sigma + qx @ cu.Bbar + psi[idx] @ cu.L)
    v = np.zeros((M, nv))
    x = np.zeros((M, nx))
    u = np.zeros((M, nu))
    uhat = cu.uhat if affine else np.zeros_like(cu.uhat)
    e = cu.e if affine else np.zeros_like(cu.e)
    p0 = P.p if affine else np.zeros(nx)
    for j in range(P.N):
        idx = stages[j]
        if j == 0:
            va = np.zeros((len(idx), nv))
            xa = np.tile(p0, (len(idx), 1))
        else:
            par = P.parent[idx]
            va = v[par]
            xa = x[par]
        v[idx] = va + dv[idx]
        u[idx] = v[idx] @ cu.L.T + uhat[idx]
        x[idx] = xa @ P.A.T + v[idx] @ cu.Bbar.T + e[idx]
    return x, u


# ---------------------------------------------------------------------------
# App. C: proximal operators
# ---------------------------------------------------------------------------

def prox_dist(s: np.ndarray, proj, tau) -> np.ndarray:
    """Prox of ``tau * dist(. | C)`` (Euclidean distance, row-wise).

    ``P = proj_C(s)``, ``delta = ||s - P||``: the result is ``P`` when
    ``delta <= tau`` and ``s + (tau / delta)(P - s)`` otherwise.  ``tau`` may
    be a scalar or one value per row.
    """
    s = np.atleast_2d(s)
    Pc = proj(s)
    delta = np.linalg.norm(s - Pc, axis=1)
    tau = np.broadcast_to(np.asarray(tau, dtype=np.float64), delta.shape)
    out = Pc.copy()
    far = delta > tau
    out[far] = s[far] + (tau[far] / delta[far])[:, None] * (Pc[far] - s[far])
    return out


def prox_g(P: OracleProblem, v: np.ndarray, gamma: float, scale: np.ndarray | None = None) -> np.ndarray:
    """``prox_{gamma g}(v)`` for the separable ``g`` of eq. gzeta (separable-sum
    rule, eq. separable-sum-property).

    With a per-(node, block) positive scaling ``s`` the function is
    ``g(S^{-1} t)`` and its prox is ``s * prox_{(gamma / s^2) g_b}(v_b / s)``.
    """
    nx = P.nx
    M = P.M
    if scale is None:
        scale = np.ones((M, 3))
    s1, s2, s3 = scale[:, 0:1], scale[:, 1:2], scale[:, 2:3]
    vs = v[:, :nx] / s1
    vz = v[:, nx:2 * nx] / s2
    vp = v[:, 2 * nx:] / s3
    ts = prox_dist(vs, lambda a: np.maximum(a, P.xs[None, :]), gamma * P.safety_weight() / scale[:, 0] ** 2)
    tz = prox_dist(vz, lambda a: np.clip(a, P.xmin[None, :], P.xmax[None, :]), gamma * P.box_weight() / scale[:, 1] ** 2)
    tp = np.clip(vp, P.umin[None, :], P.umax[None, :])
    return np.concatenate([s1 * ts, s2 * tz, s3 * tp], axis=1)


# ---------------------------------------------------------------------------
# eq. apg-iteration
# ---------------------------------------------------------------------------

def theta_next(theta: float) -> float:
    """eq. optim:theta:update."""
    return 0.5 * (math.sqrt(theta ** 4 + 4.0 * theta ** 2) - theta ** 2)


def theta_sequence(n: int) -> np.ndarray:
    """``theta_0 .. theta_{n-1}`` from ``theta_0 = 1``."""
    th = np.empty(n)
    t = 1.0
    for k in range(n):
        th[k] = t
        t = theta_next(t)
    return th


def hz(x: np.ndarray, u: np.ndarray) -> np.ndarray:
    """``H z`` of eq. optim:H:operator, per node ``(x, x, u)``."""
    return np.concatenate([x, x, u], axis=1)


@dataclass
class APGResult:
    x: np.ndarray
    u: np.ndarray
    y: np.ndarray            # y^{nu+1}, unscaled (S y')
    y_prev: np.ndarray       # y^{nu}, unscaled
    t: np.ndarray            # t^nu, unscaled
    iterations: int
    r_primal: float
    hz_t_max: float
    converged: bool
    theta: float
    theta_prev: float
    xbar: np.ndarray | None = None
    ubar: np.ndarray | None = None
    tbar: np.ndarray | None = None
    history: list | None = None

    @property
    def u0(self) -> np.ndarray:
        return self.u[0]


def apg(P: OracleProblem, lam: float, iters: int, F: Factor | None = None, *, tol: float = 0.0,
        check_every: int = 10, y0: np.ndarray | None = None, yprev0: np.ndarray | None = None,
        theta0: float = 1.0, theta_prev0: float = 1.0, scale: np.ndarray | None = None,
        ergodic: bool = False, record: bool = False) -> APGResult:
    """Accelerated dual proximal gradient, eq. apg-iteration, in FP64.

    Starting from ``y^0 = y^{-1} = y0`` (zero by default) and
    ``theta_0 = theta_{-1} = 1``, each iteration does

        w     = y + theta_nu (1/theta_{nu-1} - 1) (y - y_prev)
        z     = argmin <z, H'(S w)> + f(z)                 (Alg. 1)
        t     = prox_{(1/lambda) g~}(w / lambda + S H z)    (App. C)
        y_new = w + lambda (S H z - t)
        theta_{nu+1} from eq. optim:theta:update

    ``S`` is an optional diagonal scaling with one positive scalar per
    (node, block), ``scale`` of shape ``(M, 3)``; ``g~ = g(S^{-1} .)``.  The
    iterate that is reported is unscaled (``S y``).

    Stopping: at iterations with ``(nu + 1) % check_every == 0`` and at the
    last one, ``r_p = ||H z - t||_inf`` (unscaled) is compared with
    ``tol * (1 + max(||H z||_inf, ||t||_inf))``; ``tol = 0`` never stops early.
    Returns the last ``z^nu``, ``y^{nu+1}`` and the iteration count.
    """
    if F is None:
        F = factor_step(P)
    M, D = P.M, P.dual_dim
    nx = P.nx
    if scale is None:
        scale = np.ones((M, 3))
    svec = np.concatenate([np.repeat(scale[:, 0:1], nx, 1), np.repeat(scale[:, 1:2], nx, 1),
                           np.repeat(scale[:, 2:3], P.nu, 1)], axis=1)
    y = np.zeros((M, D)) if y0 is None else np.array(y0, dtype=np.float64) / svec
    y_prev = y.copy() if yprev0 is None else np.array(yprev0, dtype=np.float64) / svec
    theta, theta_prev = float(theta0), float(theta_prev0)
    xbar = ubar = tbar = None
    hist = [] if record else None
    x = u = t = None
    r_p = hzt = 0.0
    converged = False
    k = 0
    for k in range(iters):
        c = theta * (1.0 / theta_prev - 1.0)
        w = y + c * (y - y_prev)
        x, u = solve_step(P, F, svec * w)
        Hz = hz(x, u)
        SHz = svec * Hz
        t = prox_g(P, w / lam + SHz, 1.0 / lam, scale)
        y_new = w + lam * (SHz - t)
        t_un = t / svec
        if ergodic:
            if k == 0:
                xbar, ubar, tbar = x.copy(), u.copy(), t_un.copy()
            else:
                xbar = (1.0 - theta) * xbar + theta * x
                ubar = (1.0 - theta) * ubar + theta * u
                tbar = (1.0 - theta) * tbar + theta * t_un
        theta_prev, theta = theta, theta_next(theta)
        y_prev, y = y, y_new
        is_check = ((k + 1) % check_every == 0) or (k + 1 == iters)
        if record:
            hist.append({"r_p": float(np.max(np.abs(Hz - t_un))), "y": (svec * y).copy()})
        if is_check:
            r_p = float(np.max(np.abs(Hz - t_un)))
            hzt = float(max(np.max(np.abs(Hz)), np.max(np.abs(t_un))))
            if tol > 0.0 and r_p <= tol * (1.0 + hzt):
                converged = True
                break
    return APGResult(x=x, u=u, y=svec * y, y_prev=svec * y_prev, t=None if t is None else t / svec,
                     iterations=k + 1, r_primal=r_p, hz_t_max=hzt, converged=converged,
                     theta=theta, theta_prev=theta_prev, xbar=xbar, ubar=ubar, tbar=tbar, history=hist)


# ---------------------------------------------------------------------------
# objective and step size (Sec. IV-A, IV-D)
# ---------------------------------------------------------------------------

def stage_cost(P: OracleProblem, u: np.ndarray) -> float:
    """The smooth part of ``f`` (eq. fz): the expected economic cost plus the
    smoothing cost, ``sum_n pi_n [W_a (a1 + a2_{s(n)})' u_n + du_n' Wu du_n]``
    with ``du_n = u_n - u_{a(n)}`` and ``u_{a(root)} = q``.  (The indicators
    of the dynamics and of the coupling are zero on every point this is
    evaluated at.)"""
    cost = 0.0
    for n in range(P.M):
        a = int(P.parent[n])
        ua = P.q if a < 0 else u[a]
        du = u[n] - ua
        pi = P.prob[n]
        cost += pi * (P.W_alpha * (P.alpha1 + P.alpha2[P.stage[n]]) @ u[n] + du @ P.Wu @ du)
    return float(cost)


def soft_cost(P: OracleProblem, xs_part: np.ndarray, xz_part: np.ndarray) -> float:
    """The distance terms of ``g`` (eq. gzeta): ``sum_n cS_n dist(sigma_n |
    x >= xs) + cd_n dist(zeta_n | [xmin, xmax])`` (Euclidean distances)."""
    ds = np.linalg.norm(xs_part - np.maximum(xs_part, P.xs[None, :]), axis=1)
    db = np.linalg.norm(xz_part - np.clip(xz_part, P.xmin[None, :], P.xmax[None, :]), axis=1)
    return float(P.safety_weight() @ ds + P.box_weight() @ db)


def primal_cost(P: OracleProblem, x: np.ndarray, u: np.ndarray) -> float:
    """``E V + V_s`` of eq. Sc-MPC at ``(x, u)`` (box indicator not added)."""
    return stage_cost(P, u) + soft_cost(P, x, x)


def support_g(P: OracleProblem, y: np.ndarray) -> tuple[float, float]:
    """``g*(y)`` (App. C's sets, conjugates by definition): the conjugate of
    ``c dist(. | C)`` is the support function of ``C`` plus the indicator of
    the ball of radius ``c``; the conjugate of the indicator of the input box
    is its support function.  Returns ``(value, violation)``: the value of the
    support-function terms and the largest violation of the domain (the sign
    condition ``sigma~ <= 0`` of the half-space ``x >= xs`` and the two ball
    radii), which is ``<= 0`` exactly when ``y`` lies in ``dom g*``."""
    nx = P.nx
    ys, yz, yp = y[:, :nx], y[:, nx:2 * nx], y[:, 2 * nx:]
    val = float(np.sum(ys * P.xs) + np.sum(np.maximum(yz * P.xmax, yz * P.xmin))
                + np.sum(np.maximum(yp * P.umax, yp * P.umin)))
    viol = max(float(np.max(ys)),
               float(np.max(np.linalg.norm(ys, axis=1) - P.safety_weight())),
               float(np.max(np.linalg.norm(yz, axis=1) - P.box_weight())))
    return val, viol


def dual_objective(P: OracleProblem, F: Factor, y: np.ndarray) -> tuple[float, float]:
    """Dual objective of eq. optim:prob, ``D(y) = f*(-H'y) + g*(y)``, for an
    unscaled dual ``y``.  ``f*(-H'y) = -(f(z_y) + <y, H z_y>)`` with ``z_y``
    the minimiser of ``<z, H'y> + f(z)`` (Alg. 1, the conjugate subgradient
    theorem used in Sec. IV-A).  Returns ``(D(y), domain violation)`` as in
    ``support_g``; ``D(y) >= -V*`` for every ``y`` in the domain (weak
    duality) with equality at a dual optimum (strong duality, Sec. IV-A)."""
    x, u = solve_step(P, F, y)
    fconj = -(stage_cost(P, u) + float(np.sum(y * hz(x, u))))
    sval, viol = support_g(P, y)
    return fconj + sval, viol


def duality_gap(P: OracleProblem, F: Factor, x: np.ndarray, u: np.ndarray, t: np.ndarray,
                y: np.ndarray) -> float:
    """A-posteriori duality gap of Sec. IV-E for a primal pair ``(z, t)`` and
    a dual ``y`` (all unscaled): ``f(z) + g(t) + D(y)``.  ``t`` must satisfy
    the input box (the prox output always does); the soft terms of ``g`` are
    the distances of its state blocks.  For ``H z = t`` and ``y`` in the
    domain of ``g*`` this is ``>= 0`` (weak duality), and it tends to 0 with
    the APG's ``(z^nu, t^nu, y^{nu+1})``."""
    nx = P.nx
    return stage_cost(P, u) + soft_cost(P, t[:, :nx], t[:, nx:2 * nx]) + dual_objective(P, F, y)[0]


def _dual_hessian_apply(P: OracleProblem, F: Factor, w: np.ndarray, svec: np.ndarray) -> np.ndarray:
    x, u = solve_step(P, F, svec * w, affine=False)
    return -(svec * hz(x, u))


def dual_hessian_dense(P: OracleProblem, F: Factor | None = None, scale: np.ndarray | None = None) -> np.ndarray:
    """Dense matrix of ``w -> -S H z_lin(S w)``, the Hessian of the smooth dual
    term ``f*(-H' S y)`` (Sec. IV-A: its gradient is ``-S H z(y)``).  Only for
    tiny trees: one solve step per dual coordinate."""
    if F is None:
        F = factor_step(P)
    M, D = P.M, P.dual_dim
    if scale is None:
        scale = np.ones((M, 3))
    svec = np.concatenate([np.repeat(scale[:, 0:1], P.nx, 1), np.repeat(scale[:, 1:2], P.nx, 1),
                           np.repeat(scale[:, 2:3], P.nu, 1)], axis=1)
    n = M * D
    K = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        K[:, k] = _dual_hessian_apply(P, F, e.reshape(M, D), svec).ravel()
    return K


def dual_lmax_power(P: OracleProblem, iters: int = 300, F: Factor | None = None,
                    scale: np.ndarray | None = None, seed: int = 0) -> float:
    """Largest eigenvalue of the dual Hessian by power iteration (Sec. IV-D:
    ``lambda = 1 / L``); returns the Rayleigh quotient of the last iterate."""
    if F is None:
        F = factor_step(P)
    M, D = P.M, P.dual_dim
    if scale is None:
        scale = np.ones((M, 3))
    svec = np.concatenate([np.repeat(scale[:, 0:1], P.nx, 1), np.repeat(scale[:, 1:2], P.nx, 1),
                           np.repeat(scale[:, 2:3], P.nu, 1)], axis=1)
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, (M, D))
    w /= np.linalg.norm(w)
    lam = 0.0
    for _ in range(iters):
        g = _dual_hessian_apply(P, F, w, svec)
        lam = float(np.sum(w * g))
        nrm = np.linalg.norm(g)
        if nrm == 0.0:
            return 0.0
        w = g / nrm
    return lam


# ---------------------------------------------------------------------------
# Receding-horizon warm start (closed loop of Alg. 2)
#
# The paper starts every MPC step from y0 = 0; any dual point is a valid start
# for the APG, so a served controller may start from the previous step's dual
# moved one stage forward.  Reading used here (the paper does not define a
# shift): the new root takes the place of the realised stage-1 child of the old
# root; a new node at stage j + 1 takes the place of the child of its parent's
# image with the same child index (the last child when there are fewer); below
# the old last stage the image stays put (the last stage is duplicated).  Dual
# blocks whose cost is probability weighted (the safety distance when
# ``weight_safety_by_prob``, the input box of the probability-weighted input
# costs) are rescaled by pi_new / pi_old; the state-box block is kept.
# ---------------------------------------------------------------------------
def shift_map(P: OracleProblem, realized: int) -> np.ndarray:
    """Image ``m(n)`` in the previous tree of every node ``n`` of the next
    tree (the same tree structure one stage later)."""
    ch = P.children()
    if not 0 <= realized < len(ch[0]):
        raise ValueError("realized must index a child of the root")
    img = np.empty(P.M, dtype=np.int64)
    img[0] = ch[0][realized]
    for n in range(1, P.M):  # stage-sorted: the parent's image is known
        a = int(P.parent[n])
        k = ch[a].index(n)
        kids = ch[int(img[a])]
        img[n] = kids[min(k, len(kids) - 1)] if kids else img[a]
    return img


def shift_dual(P: OracleProblem, y: np.ndarray, realized: int) -> np.ndarray:
    """Shifted warm start ``y_new[n] = r_n y[m(n)]`` per block, ``r_n =
    pi[n] / pi[m(n)]`` for the probability-weighted blocks, 1 otherwise."""
    img = shift_map(P, realized)
    nx = P.nx
    ratio = P.prob / P.prob[img]
    out = y[img].copy()
    if P.weight_safety_by_prob:
        out[:, :nx] *= ratio[:, None]
    out[:, 2 * nx:] *= ratio[:, None]
    return out


# ---------------------------------------------------------------------------
# Closed loop (Alg. 2) and its performance indicators (Sec. V-B)
# ---------------------------------------------------------------------------
def plant_step(P: OracleProblem, x: np.ndarray, u: np.ndarray, d: np.ndarray) -> np.ndarray:
    """One step of the flow model (eq. model): ``x+ = A x + B u + Gd d``."""
    return P.A @ x + P.B @ u + P.Gd @ d


def closed_loop_kpis(alpha1: np.ndarray, alpha2: np.ndarray, xs: np.ndarray, x: np.ndarray, u: np.ndarray,
                     u_prev: np.ndarray) -> dict:
    """The four indicators of Sec. V-B over a simulation of ``Hs`` steps:
    ``alpha2`` (Hs, nu) the pumping cost of each applied step, ``u`` (Hs, nu)
    the applied inputs, ``x`` (Hs, nx) the states they lead to, ``u_prev``
    the input applied before the first step.

    * KPI_E  = (1/Hs) sum_k (alpha1 + alpha2_k)' |u_k|      (economic cost)
    * KPI_dU = (1/Hs) sum_k ||u_k - u_{k-1}||_2^2           (smoothness)
    * KPI_S  = sum_k ||[xs - x_k]_+||_1                     (water taken from the safety storage)
    * KPI_R  = ||xs||_1 / ((1/Hs) sum_k ||x_k||_1) * 100    (safety volume in % of the mean volume)
    """
    Hs = u.shape[0]
    e = sum(float((alpha1 + alpha2[k]) @ np.abs(u[k])) for k in range(Hs)) / Hs
    prev = np.vstack([u_prev[None, :], u[:-1]])
    du = sum(float(np.sum((u[k] - prev[k]) ** 2)) for k in range(Hs)) / Hs
    s = sum(float(np.sum(np.maximum(xs - x[k], 0.0))) for k in range(Hs))
    mean_vol = sum(float(np.sum(np.abs(x[k]))) for k in range(Hs)) / Hs
    r = float(np.sum(np.abs(xs))) / mean_vol * 100.0
    return {"E": e, "dU": du, "S": s, "R": r}
