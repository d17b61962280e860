"""Small object layer over the C ABI: one context, one system, many trees.

Every method is a marshalling wrapper of one ``smpc_*`` call.
"""

from __future__ import annotations

import numpy as np

from . import smpc as S


class Context:
    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        if stream is None:
            try:
                import torch

                if torch.cuda.is_available():
                    stream = torch.cuda.current_stream(device).cuda_stream
            except Exception:  # torch absent: the library owns its stream
                stream = None
        self.h = S.smpc_ctx_create(device, stream, hbm_budget)
        self.systems: list[System] = []

    def system(self, sys: dict) -> "System":
        s = System(self, sys)
        self.systems.append(s)
        return s

    def mem_used(self) -> int:
        return S.smpc_ctx_mem_used(self.h)

    def profiling(self, on: bool) -> None:
        S.smpc_ctx_set_profiling(self.h, on)

    def kernel_stats(self) -> dict:
        return S.smpc_ctx_kernel_stats(self.h)

    def reset_stats(self) -> None:
        S.smpc_ctx_reset_stats(self.h)

    def close(self) -> None:
        for s in self.systems:
            s.close()
        self.systems = []
        if self.h is not None:
            S.smpc_ctx_destroy(self.h)
            self.h = None


class System:
    def __init__(self, ctx: Context, sys: dict):
        self.ctx = ctx
        self.desc = sys
        self.nx, self.nu = int(sys["nx"]), int(sys["nu"])
        self.h = S.smpc_sys_create(ctx.h, sys)
        self.trees: list[Tree] = []

    def tree(self, tree: dict) -> "Tree":
        t = Tree(self, tree)
        self.trees.append(t)
        return t

    def solve_batch(self, trees, ps, qs, **kw):
        return S.smpc_solve_batch([t.h for t in trees], ps, qs, dims_list=[t.dims for t in trees], **kw)

    def server(self, **kw) -> "Server":
        """Continuous-batching server over this system's trees (see
        smpc_server_create); close it before using the trees directly."""
        return Server(self, **kw)

    def close(self) -> None:
        for t in self.trees:
            t.close()
        self.trees = []
        if self.h is not None:
            S.smpc_sys_destroy(self.h)
            self.h = None


class Tree:
    def __init__(self, system: System, tree: dict):
        self.system = system
        self.N = int(tree["N"])
        self.M = int(np.asarray(tree["stage"]).shape[0])
        self.h = S.smpc_tree_create(system.h, self.N, tree["stage"], tree["parent"], tree["prob"])

    @property
    def dims(self):
        return (self.M, self.system.nx, self.system.nu)

    def set_data(self, d, alpha2=None) -> None:
        S.smpc_tree_set_data(self.h, d, alpha2)

    def get_data(self) -> dict:
        return S.smpc_tree_get_data(self.h, dims=self.dims)

    def objective(self) -> dict:
        return S.smpc_tree_objective(self.h)

    def factor(self, **kw) -> None:
        S.smpc_factor(self.h, **kw)

    def factor_info(self, with_scale: bool = False):
        return S.smpc_tree_get_factor(self.h, with_scale)

    def info(self) -> dict:
        return S.smpc_tree_info(self.h)

    def solve(self, p, q, **kw) -> dict:
        return S.smpc_solve(self.h, p, q, dims=self.dims, **kw)

    def shift_warm_start(self, realized: int) -> None:
        """Prepare the next solve (``resident=True``) from this tree's last
        dual, moved one stage forward along root child ``realized``."""
        S.smpc_shift_warm_start(self.h, realized)

    def solve_step(self, p, q, w, precision: int = 64):
        return S.smpc_solve_step(self.h, p, q, w, dims=self.dims, precision=precision)

    def close(self) -> None:
        if self.h is not None:
            S.smpc_tree_destroy(self.h)
            self.h = None


def from_instance(ctx: Context, inst, system: System | None = None, **factor_kw):
    """Create (system,) tree, upload data and factor for a ``dwn_synth`` instance."""
    if system is None:
        system = ctx.system(inst.sys)
    t = system.tree(inst.tree)
    t.set_data(inst.d, inst.alpha2)
    t.factor(**factor_kw)
    return system, t


class Server:
    def __init__(self, system: System, **kw):
        self.system = system
        self.h = S.smpc_server_create(system.h, **kw)

    def submit(self, tree: Tree, p, q, *, d=None, alpha2=None, warm: int = 0, realized: int = 0) -> int:
        return S.smpc_server_submit(self.h, tree.h, p, q, d=d, alpha2=alpha2, warm=warm, realized=realized)

    def poll(self, ticket: int, wait_ms: int = -1):
        return S.smpc_server_poll(self.h, ticket, self.system.nu, wait_ms)

    def cancel(self, ticket: int) -> None:
        S.smpc_server_cancel(self.h, ticket)

    def close(self) -> None:
        if self.h is not None:
            S.smpc_server_destroy(self.h)
            self.h = None
