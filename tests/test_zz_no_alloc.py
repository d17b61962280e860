"""The no-allocation objective entry point (smpc_tree_objective_noalloc)
against the allocating one (smpc_tree_objective): the same kernels on the
same iterates give the same bits; the call allocates no device memory; two
calls in a row on different trees, the second smaller, share the scratch."""

import pytest

import dwn_synth as ds

pytestmark = pytest.mark.gpu


def _solve(tree, inst):
    return tree.solve(inst.p, inst.q, tol=0.0, max_iter=200, check_every=10, precision=64, want_x=False,
                      want_y=False)


def test_noalloc_objective_matches_allocating_call():
    from paper_1604_01074_amd import smpc, solver

    ctx = solver.Context(0)
    try:
        cases = [(ds.barcelona_instance(N=8, branching=(3, 3)), 2), (ds.tiny_instance(), 0)]
        for inst, precond in cases:  # the second tree is the smaller one
            print(f"[no-alloc] M={inst.M}", flush=True)
            system, tree = solver.from_instance(ctx, inst, precond=precond, power_iters=100)
            _solve(tree, inst)
            used = ctx.mem_used()
            a = smpc.smpc_tree_objective_noalloc(tree.h)
            assert ctx.mem_used() == used
            assert smpc.smpc_tree_objective_noalloc(tree.h) == a  # cached for the same solve
            _solve(tree, inst)  # the same iterates again (the solve is deterministic)
            b = tree.objective()
            assert a == b, (a, b)
        # a tree solved only in a batch, with a given step size (no power
        # iteration), has no single-tree plan: refused
        inst = ds.tiny_instance(seed=1)
        t2 = system.tree(inst.tree)
        t2.set_data(inst.d, inst.alpha2)
        t2.factor(lambda_override=1e-3)
        system.solve_batch([t2], [inst.p], [inst.q], tol=0.0, max_iter=20, check_every=10, precision=64)
        with pytest.raises(smpc.SmpcError) as e:
            smpc.smpc_tree_objective_noalloc(t2.h)
        assert e.value.code == smpc.EINVAL
    finally:
        ctx.close()
