"""Resident, shifted warm start (smpc_shift_warm_start + warm_start 1)
against the oracle's shift of the downloaded dual uploaded as y0."""

import numpy as np
import pytest

import dwn_synth as ds
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1604_01074_amd import solver

    c = solver.Context(0)
    yield c
    c.close()


def _tree(ctx, inst, precond=1):
    s = ctx.system(inst.sys)
    t = s.tree(inst.tree)
    t.set_data(inst.d, inst.alpha2)
    t.factor(precond=precond, power_iters=100)
    return s, t


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


@pytest.mark.parametrize("precision,realized,tol", [(64, 1, 1e-9), (64, 2, 1e-9), (32, 0, 1e-4)])
def test_resident_shift_matches_oracle_shift(ctx, precision, realized, tol):
    inst = ds.random_small_instance(2, nx=4, nu=5, nd=3, ne=2, N=5, branching=(3, 2), scenarios=6)
    s, t = _tree(ctx, inst)
    try:
        kw = dict(tol=0.0, check_every=10, precision=precision, polish_iters=0)
        first = t.solve(inst.p, inst.q, max_iter=300, **kw)
        P = O.OracleProblem.from_instance(inst)
        y0 = O.shift_dual(P, first["y"], realized)
        t.shift_warm_start(realized)
        a = t.solve(inst.p, inst.q, max_iter=60, resident=True, **kw)
        b = t.solve(inst.p, inst.q, max_iter=60, y0=y0, **kw)
        print(f"[shift] FP{precision} r={realized}: u {_rel(a['u'], b['u']):.2e} y {_rel(a['y'], b['y']):.2e}", flush=True)
        assert _rel(a["u"], b["u"]) <= tol and _rel(a["x"], b["x"]) <= tol and _rel(a["y"], b["y"]) <= tol
    finally:
        s.close()
        ctx.systems.remove(s)


def test_shift_errors(ctx):
    from paper_1604_01074_amd import smpc

    inst = ds.tiny_instance()
    s, t = _tree(ctx, inst, precond=0)
    try:
        with pytest.raises(smpc.SmpcError) as e:
            t.shift_warm_start(0)  # nothing resident yet
        assert e.value.code == smpc.EINVAL
        with pytest.raises(smpc.SmpcError) as e:
            t.solve(inst.p, inst.q, max_iter=10, resident=True)  # no shift prepared
        assert e.value.code == smpc.EINVAL
        t.solve(inst.p, inst.q, max_iter=10)
        with pytest.raises(smpc.SmpcError) as e:
            t.shift_warm_start(2)  # the root has two children
        assert e.value.code == smpc.EINVAL
        t.shift_warm_start(-1)  # resume unshifted
        r = t.solve(inst.p, inst.q, max_iter=10, resident=True)
        assert r["iterations"] == 10
        t.factor(precond=0, power_iters=10)  # overwrites the dual slots
        with pytest.raises(smpc.SmpcError) as e:
            t.shift_warm_start(0)
        assert e.value.code == smpc.EINVAL
    finally:
        s.close()
        ctx.systems.remove(s)


def test_resume_unshifted_equals_one_long_run(ctx):
    """Resuming from the resident dual (realized = -1) restarts the momentum
    (theta = 1) from y^{nu+1}: the same as a fresh solve from that dual."""
    inst = ds.tiny_instance()
    s, t = _tree(ctx, inst, precond=0)
    try:
        first = t.solve(inst.p, inst.q, max_iter=100)
        t.shift_warm_start(-1)
        a = t.solve(inst.p, inst.q, max_iter=50, resident=True)
        b = t.solve(inst.p, inst.q, max_iter=50, y0=first["y"])
        assert _rel(a["u"], b["u"]) <= 1e-12 and _rel(a["y"], b["y"]) <= 1e-12
    finally:
        s.close()
        ctx.systems.remove(s)
