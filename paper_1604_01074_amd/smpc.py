"""ctypes binding of ``libsmpc.so`` (declared in ``include/smpc.h``).

The functions keep the C names and only marshal arguments: numpy arrays in,
numpy arrays out, negative return codes raised as :class:`SmpcError`.  All
solver work happens in the library's HIP kernels and float64 host setup; there
is no Python or CPU fallback.  If the library is missing, importing this
module raises.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmpc.so")

OK, MAX_ITER, PENDING, STALLED = 0, 1, 2, 3
EINVAL, EDIM, ENOTSPD, ERANK, EPROB, ENOMEM, EDEVICE, ENOTFACTORED, EDIVERGED, ENAN, ECANCELED = range(-1, -12, -1)
STATUS_NAMES = {
    0: "SMPC_OK", 1: "SMPC_MAX_ITER", 2: "SMPC_PENDING", 3: "SMPC_STALLED", -1: "SMPC_EINVAL", -2: "SMPC_EDIM", -3: "SMPC_ENOTSPD",
    -4: "SMPC_ERANK", -5: "SMPC_EPROB", -6: "SMPC_ENOMEM", -7: "SMPC_EDEVICE",
    -8: "SMPC_ENOTFACTORED", -9: "SMPC_EDIVERGED", -10: "SMPC_ENAN", -11: "SMPC_ECANCELED",
}

EXPORTED = [
    "smpc_ctx_create", "smpc_ctx_destroy", "smpc_last_error", "smpc_ctx_mem_used",
    "smpc_sys_create", "smpc_sys_destroy",
    "smpc_tree_create", "smpc_tree_destroy", "smpc_tree_set_data", "smpc_tree_get_data", "smpc_tree_objective",
    "smpc_tree_objective_noalloc",
    "smpc_factor", "smpc_tree_get_factor", "smpc_tree_info",
    "smpc_solve", "smpc_solve_batch", "smpc_shift_warm_start", "smpc_solve_step",
    "smpc_ctx_set_profiling", "smpc_ctx_kernel_stats", "smpc_ctx_reset_stats",
    "smpc_server_create", "smpc_server_submit", "smpc_server_poll", "smpc_server_cancel", "smpc_server_destroy",
    "smpc_chunk_lengths", "smpc_plant_step", "smpc_closed_loop_kpi",
]


class SmpcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1604_01074_amd.build`")

# One HIP runtime per process.  PyTorch ships its own libamdhip64 (soname
# libamdhip64.so.7, loaded by torch under the file name libamdhip64.so) and its
# own HSA runtime.  Loading torch first makes libsmpc's libamdhip64.so.7
# dependency resolve to that same, already-loaded runtime, so torch streams
# are valid library streams and only one HSA runtime opens the GPU.  (With
# the other order the process would hold two runtimes and the one initialised
# second would see no device.)
try:
    import torch  # noqa: F401
except ImportError:  # no torch: the system ROCm runtime is used
    torch = None

_lib = C.CDLL(LIB_PATH)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


class SysDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("nu", C.c_int), ("nd", C.c_int), ("ne", C.c_int),
                ("A", _dp), ("B", _dp), ("Gd", _dp), ("E", _dp), ("Ed", _dp),
                ("umin", _dp), ("umax", _dp), ("xmin", _dp), ("xmax", _dp), ("xs", _dp),
                ("W_alpha", C.c_double), ("W_x", C.c_double), ("gamma_d", C.c_double),
                ("alpha1", _dp), ("Wu", _dp), ("weight_safety_by_prob", C.c_int)]


class FactorOpts(C.Structure):
    _fields_ = [("precond", C.c_int), ("power_iters", C.c_int), ("lambda_override", C.c_double),
                ("scale", _dp)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("check_every", C.c_int),
                ("precision", C.c_int), ("polish_iters", C.c_int), ("warm_start", C.c_int),
                ("y0", _dp), ("y_prev0", _dp), ("stall_checks", C.c_int), ("tune", C.c_int),
                ("chunk32", C.c_int * 2), ("chunk64", C.c_int * 2), ("unfused", C.c_int), ("gap", C.c_int),
                ("dual64", C.c_int)]


class Result(C.Structure):
    _fields_ = [("u0", _dp), ("x", _dp), ("u", _dp), ("y", _dp), ("iterations", C.c_int),
                ("fp32_iterations", C.c_int), ("r_primal", C.c_double), ("hz_t_max", C.c_double),
                ("status", C.c_int), ("queue_ms", C.c_double), ("run_ms", C.c_double),
                ("chunk32", C.c_int * 2), ("chunk64", C.c_int * 2), ("cost", C.c_double), ("gap", C.c_double)]


class Objective(C.Structure):
    _fields_ = [("cost", C.c_double), ("primal", C.c_double), ("dual", C.c_double), ("gap", C.c_double),
                ("dual_violation", C.c_double)]


class Kpi(C.Structure):
    _fields_ = [("E", C.c_double), ("dU", C.c_double), ("S", C.c_double), ("R", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("solve", SolveOpts), ("max_active", C.c_int)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int), ("total_ms", C.c_double)]


_sig = {
    "smpc_ctx_create": [C.c_int, _vp, C.c_size_t, C.POINTER(_vp)],
    "smpc_ctx_destroy": [_vp],
    "smpc_last_error": [C.c_char_p, C.c_size_t],
    "smpc_ctx_mem_used": [_vp, C.POINTER(C.c_size_t)],
    "smpc_sys_create": [_vp, C.POINTER(SysDesc), C.POINTER(_vp)],
    "smpc_sys_destroy": [_vp],
    "smpc_tree_create": [_vp, C.c_int, C.c_int, _ip, _ip, _dp, C.POINTER(_vp)],
    "smpc_tree_destroy": [_vp],
    "smpc_tree_set_data": [_vp, _dp, _dp],
    "smpc_tree_get_data": [_vp, _dp, _dp, _dp],
    "smpc_tree_objective": [_vp, C.POINTER(Objective)],
    "smpc_tree_objective_noalloc": [_vp, C.POINTER(Objective)],
    "smpc_factor": [_vp, C.POINTER(FactorOpts)],
    "smpc_tree_get_factor": [_vp, _dp, _dp],
    "smpc_tree_info": [_vp, _ip, _ip, _ip, _ip],
    "smpc_solve": [_vp, _dp, _dp, C.POINTER(SolveOpts), C.POINTER(Result)],
    "smpc_solve_batch": [C.POINTER(_vp), C.c_int, C.POINTER(_dp), C.POINTER(_dp), C.POINTER(SolveOpts),
                         C.POINTER(Result)],
    "smpc_shift_warm_start": [_vp, C.c_int],
    "smpc_solve_step": [_vp, _dp, _dp, _dp, C.c_int, _dp, _dp],
    "smpc_ctx_set_profiling": [_vp, C.c_int],
    "smpc_ctx_kernel_stats": [_vp, C.POINTER(KernelStat), C.c_int, _ip],
    "smpc_ctx_reset_stats": [_vp],
    "smpc_server_create": [_vp, C.POINTER(ServerOpts), C.POINTER(_vp)],
    "smpc_server_submit": [_vp, _vp, _dp, _dp, _dp, _dp, C.c_int, C.c_int, C.POINTER(C.c_uint64)],
    "smpc_server_poll": [_vp, C.c_uint64, C.POINTER(Result), C.c_int],
    "smpc_server_cancel": [_vp, C.c_uint64],
    "smpc_server_destroy": [_vp],
    "smpc_chunk_lengths": [C.c_int, C.c_int, _ip, C.c_int, _ip],
    "smpc_plant_step": [_vp, _dp, _dp, _dp, _dp],
    "smpc_closed_loop_kpi": [_vp, C.c_int, _dp, _dp, _dp, _dp, C.POINTER(Kpi)],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int


def last_error() -> str:
    buf = C.create_string_buffer(1024)
    _lib.smpc_last_error(buf, 1024)
    return buf.value.decode(errors="replace")


def _check(code: int) -> int:
    if code < 0:
        raise SmpcError(code, last_error())
    return code


def _check_solve(code: int) -> int:
    """A solve reports divergence as its result status, not as an exception."""
    if code < 0 and code != EDIVERGED:
        raise SmpcError(code, last_error())
    return code


def _f64(a, shape=None):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        arr = arr.reshape(shape)
    return arr


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


# ---------------------------------------------------------------- context

def smpc_ctx_create(device: int = 0, hip_stream: int | None = None, hbm_budget: int = 0):
    h = _vp()
    _check(_lib.smpc_ctx_create(int(device), hip_stream, int(hbm_budget), C.byref(h)))
    return h


def smpc_ctx_destroy(ctx) -> None:
    _check(_lib.smpc_ctx_destroy(ctx))


def smpc_ctx_mem_used(ctx) -> int:
    v = C.c_size_t()
    _check(_lib.smpc_ctx_mem_used(ctx, C.byref(v)))
    return int(v.value)


# ---------------------------------------------------------------- system

def smpc_sys_create(ctx, sys: dict):
    """``sys`` uses the keys of :mod:`dwn_synth.systems` (nx, nu, nd, ne, A, B,
    Gd, E, Ed, umin, umax, xmin, xmax, xs, W_alpha, alpha1, Wu, W_x, gamma_d,
    weight_safety_by_prob)."""
    nx, nu, nd, ne = (int(sys[k]) for k in ("nx", "nu", "nd", "ne"))
    keep = {k: _f64(sys[k]) for k in ("A", "B", "Gd", "umin", "umax", "xmin", "xmax", "xs", "alpha1", "Wu")}
    keep["E"] = _f64(sys["E"]) if ne else None
    keep["Ed"] = _f64(sys["Ed"]) if ne else None
    d = SysDesc(nx, nu, nd, ne, *(_ptr(keep[k]) for k in ("A", "B", "Gd", "E", "Ed", "umin", "umax", "xmin", "xmax", "xs")),
                float(sys["W_alpha"]), float(sys["W_x"]), float(sys["gamma_d"]), _ptr(keep["alpha1"]),
                _ptr(keep["Wu"]), int(sys.get("weight_safety_by_prob", 1)))
    h = _vp()
    _check(_lib.smpc_sys_create(ctx, C.byref(d), C.byref(h)))
    return h


def smpc_sys_destroy(s) -> None:
    _check(_lib.smpc_sys_destroy(s))


# ---------------------------------------------------------------- tree

def smpc_tree_create(s, N: int, stage, parent, prob):
    st = np.ascontiguousarray(stage, dtype=np.int32)
    pa = np.ascontiguousarray(parent, dtype=np.int32)
    pr = _f64(prob)
    M = int(st.shape[0])
    h = _vp()
    _check(_lib.smpc_tree_create(s, int(N), M, st.ctypes.data_as(_ip), pa.ctypes.data_as(_ip), _ptr(pr),
                                 C.byref(h)))
    return h


def smpc_tree_destroy(t) -> None:
    _check(_lib.smpc_tree_destroy(t))


def smpc_tree_set_data(t, d, alpha2=None) -> None:
    dd = _f64(d)
    a2 = None if alpha2 is None else _f64(alpha2)
    _check(_lib.smpc_tree_set_data(t, _ptr(dd), _ptr(a2)))


def smpc_tree_get_data(t, *, dims) -> dict:
    """uhat (M, nu), e (M, nx), beta (M, nu) as held on the device."""
    M, nx, nu = dims
    out = {"uhat": np.empty((M, nu)), "e": np.empty((M, nx)), "beta": np.empty((M, nu))}
    _check(_lib.smpc_tree_get_data(t, _ptr(out["uhat"]), _ptr(out["e"]), _ptr(out["beta"])))
    return out


def smpc_tree_objective(t) -> dict:
    """cost, primal, dual, gap, dual_violation at the tree's last solve."""
    o = Objective()
    _check(_lib.smpc_tree_objective(t, C.byref(o)))
    return {k: getattr(o, k) for k in ("cost", "primal", "dual", "gap", "dual_violation")}


def smpc_tree_objective_noalloc(t) -> dict:
    """smpc_tree_objective with the library's fixed device scratch (no
    device allocation)."""
    o = Objective()
    _check(_lib.smpc_tree_objective_noalloc(t, C.byref(o)))
    return {k: getattr(o, k) for k in ("cost", "primal", "dual", "gap", "dual_violation")}


def smpc_factor(t, precond: int = 0, power_iters: int = 0, lambda_override: float = 0.0, scale=None) -> None:
    sc = None if scale is None else _f64(scale)
    o = FactorOpts(int(precond), int(power_iters), float(lambda_override), _ptr(sc))
    _check(_lib.smpc_factor(t, C.byref(o)))


def smpc_tree_info(t) -> dict:
    v = [C.c_int32() for _ in range(4)]
    _check(_lib.smpc_tree_info(t, *(C.byref(x) for x in v)))
    return {"M": v[0].value, "N": v[1].value, "n_chains": v[2].value, "n_levels": v[3].value}


def smpc_tree_get_factor(t, with_scale: bool = False):
    lam = C.c_double()
    info = smpc_tree_info(t)
    sc = np.empty((info["M"], 3)) if with_scale else None
    _check(_lib.smpc_tree_get_factor(t, C.byref(lam), _ptr(sc)))
    return (lam.value, sc) if with_scale else lam.value


# ---------------------------------------------------------------- solve

def _pair(v):
    a = (C.c_int * 2)()
    if v is not None:
        a[0], a[1] = int(v[0]), int(v[1])
    return a


def _opts(tol, max_iter, check_every, precision, polish_iters, y0, y_prev0, stall_checks=0, resident=False,
          tune=0, chunk32=None, chunk64=None, unfused=False, gap=False, dual64=False):
    keep = [None if y0 is None else _f64(y0), None if y_prev0 is None else _f64(y_prev0)]
    if resident and y0 is not None:
        raise ValueError("a resident warm start and y0 exclude each other")
    warm = 1 if resident else (2 if y0 is not None else 0)
    o = SolveOpts(float(tol), int(max_iter), int(check_every), int(precision), int(polish_iters),
                  warm, _ptr(keep[0]), _ptr(keep[1]), int(stall_checks), int(tune), _pair(chunk32),
                  _pair(chunk64), int(bool(unfused)), int(bool(gap)), int(bool(dual64)))
    return o, keep


def _result(M, nx, nu, want_x, want_y):
    D = 2 * nx + nu
    out = {"u0": np.empty(nu)}
    if want_x:
        out["x"] = np.empty((M, nx))
        out["u"] = np.empty((M, nu))
    if want_y:
        out["y"] = np.empty((M, D))
    r = Result(_ptr(out["u0"]), _ptr(out.get("x")), _ptr(out.get("u")), _ptr(out.get("y")))
    return r, out


def _finish(r: Result, out: dict) -> dict:
    out.update(iterations=r.iterations, fp32_iterations=r.fp32_iterations, r_primal=r.r_primal,
               hz_t_max=r.hz_t_max, status=r.status, chunk32=tuple(r.chunk32), chunk64=tuple(r.chunk64),
               cost=r.cost, gap=r.gap)
    return out


def smpc_solve(t, p, q, *, dims, tol=1e-3, max_iter=1000, check_every=10, precision=64, polish_iters=0,
               y0=None, y_prev0=None, want_x=True, want_y=True, stall_checks=0, resident=False, tune=0,
               chunk32=None, chunk64=None, unfused=False, gap=False, dual64=False) -> dict:
    """``dims = (M, nx, nu)``.  Returns a dict with u0, x, u, y, iterations,
    fp32_iterations, r_primal, hz_t_max, status, chunk32, chunk64, cost, gap
    (the last two with ``gap=True``)."""
    M, nx, nu = dims
    o, keep = _opts(tol, max_iter, check_every, precision, polish_iters, y0, y_prev0, stall_checks, resident,
                    tune, chunk32, chunk64, unfused, gap, dual64)
    r, out = _result(M, nx, nu, want_x, want_y)
    pp, qq = _f64(p), _f64(q)
    _check_solve(_lib.smpc_solve(t, _ptr(pp), _ptr(qq), C.byref(o), C.byref(r)))
    return _finish(r, out)


def smpc_solve_batch(trees, ps, qs, *, dims_list, tol=1e-3, max_iter=1000, check_every=10, precision=64,
                     polish_iters=0, y0=None, y_prev0=None, want_x=True, want_y=True,
                     stall_checks=0, resident=False, tune=0, chunk32=None, chunk64=None,
                     unfused=False, gap=False, dual64=False) -> tuple[int, list]:
    n = len(trees)
    o, keep = _opts(tol, max_iter, check_every, precision, polish_iters, y0, y_prev0, stall_checks, resident,
                    tune, chunk32, chunk64, unfused, gap, dual64)
    res = (Result * n)()
    outs = []
    for k, (M, nx, nu) in enumerate(dims_list):
        r, out = _result(M, nx, nu, want_x, want_y)
        res[k] = r
        outs.append(out)
    pp = [_f64(p) for p in ps]
    qq = [_f64(q) for q in qs]
    parr = (_dp * n)(*[_ptr(a) for a in pp])
    qarr = (_dp * n)(*[_ptr(a) for a in qq])
    tarr = (_vp * n)(*[t.value if isinstance(t, _vp) else t for t in trees])
    code = _check_solve(_lib.smpc_solve_batch(tarr, n, parr, qarr, C.byref(o), res))
    return code, [_finish(res[k], outs[k]) for k in range(n)]


def smpc_shift_warm_start(t, realized: int) -> None:
    _check(_lib.smpc_shift_warm_start(t, int(realized)))


def smpc_solve_step(t, p, q, w, *, dims, precision=64):
    M, nx, nu = dims
    x = np.empty((M, nx))
    u = np.empty((M, nu))
    ww, pp, qq = _f64(w), _f64(p), _f64(q)
    _check(_lib.smpc_solve_step(t, _ptr(pp), _ptr(qq), _ptr(ww), int(precision), _ptr(x), _ptr(u)))
    return x, u


def smpc_chunk_lengths(precision: int, which: int) -> list:
    """Chunk lengths built for ``precision`` (32, 64) and kernel ``which``
    (0 backward, 1 forward), default first."""
    n = C.c_int32()
    _check(_lib.smpc_chunk_lengths(int(precision), int(which), None, 0, C.byref(n)))
    arr = (C.c_int32 * max(n.value, 1))()
    _check(_lib.smpc_chunk_lengths(int(precision), int(which), arr, n.value, C.byref(n)))
    return [arr[k] for k in range(n.value)]


# ---------------------------------------------------------------- closed loop

def smpc_plant_step(s, x, u, d):
    xx, uu = _f64(x), _f64(u)
    dd = None if d is None else _f64(d)
    out = np.empty_like(xx)
    _check(_lib.smpc_plant_step(s, _ptr(xx), _ptr(uu), _ptr(dd), _ptr(out)))
    return out


def smpc_closed_loop_kpi(s, u, x, alpha2, u_prev) -> dict:
    """KPIs of Sec. V-B: u (Hs, nu), x (Hs, nx), alpha2 (Hs, nu) or None."""
    uu, xx, pp = _f64(u), _f64(x), _f64(u_prev)
    aa = None if alpha2 is None else _f64(alpha2)
    k = Kpi()
    _check(_lib.smpc_closed_loop_kpi(s, int(uu.shape[0]), _ptr(uu), _ptr(xx), _ptr(aa), _ptr(pp), C.byref(k)))
    return {"E": k.E, "dU": k.dU, "S": k.S, "R": k.R}


# ---------------------------------------------------------------- profiling

def smpc_ctx_set_profiling(ctx, enable: bool) -> None:
    _check(_lib.smpc_ctx_set_profiling(ctx, int(bool(enable))))


def smpc_ctx_kernel_stats(ctx) -> dict:
    n = C.c_int32()
    _check(_lib.smpc_ctx_kernel_stats(ctx, None, 0, C.byref(n)))
    arr = (KernelStat * max(n.value, 1))()
    _check(_lib.smpc_ctx_kernel_stats(ctx, arr, n.value, C.byref(n)))
    return {arr[k].name.decode(): {"launches": arr[k].launches, "total_ms": arr[k].total_ms} for k in range(n.value)}


def smpc_ctx_reset_stats(ctx) -> None:
    _check(_lib.smpc_ctx_reset_stats(ctx))


# ---------------------------------------------------------------- serving

def smpc_server_create(sys_handle, *, tol=1e-3, max_iter=1000, check_every=10, precision=32, polish_iters=20,
                       stall_checks=0, max_active=0, tune=0, chunk32=None, chunk64=None, unfused=False,
                       dual64=False):
    o, _ = _opts(tol, max_iter, check_every, precision, polish_iters, None, None, stall_checks, False, tune,
                 chunk32, chunk64, unfused, False, dual64)
    so = ServerOpts(o, int(max_active))
    h = _vp()
    _check(_lib.smpc_server_create(sys_handle, C.byref(so), C.byref(h)))
    return h


def smpc_server_submit(srv, tree, p, q, *, d=None, alpha2=None, warm=0, realized=0) -> int:
    pp, qq = _f64(p), _f64(q)
    dd = None if d is None else _f64(d)
    aa = None if alpha2 is None else _f64(alpha2)
    tk = C.c_uint64()
    _check(_lib.smpc_server_submit(srv, tree, _ptr(dd), _ptr(aa), _ptr(pp), _ptr(qq), int(warm), int(realized),
                                   C.byref(tk)))
    return tk.value


def smpc_server_poll(srv, ticket: int, nu: int, wait_ms: int = -1):
    """None while the request runs, else a dict with u0, iterations,
    fp32_iterations, r_primal, hz_t_max, status, queue_ms, run_ms (only
    status and the times for a canceled request)."""
    u0 = np.empty(nu)
    r = Result(_ptr(u0), None, None, None)
    code = _lib.smpc_server_poll(srv, C.c_uint64(ticket), C.byref(r), int(wait_ms))
    if code == PENDING:
        return None
    if code < 0 and code not in (EDIVERGED, ECANCELED):
        raise SmpcError(code, last_error())
    if code == ECANCELED:
        return dict(status=code, queue_ms=r.queue_ms, run_ms=r.run_ms)
    return dict(u0=u0, iterations=r.iterations, fp32_iterations=r.fp32_iterations, r_primal=r.r_primal,
                hz_t_max=r.hz_t_max, status=r.status, queue_ms=r.queue_ms, run_ms=r.run_ms,
                chunk32=tuple(r.chunk32), chunk64=tuple(r.chunk64))


def smpc_server_cancel(srv, ticket: int) -> None:
    _check(_lib.smpc_server_cancel(srv, C.c_uint64(ticket)))


def smpc_server_destroy(srv) -> None:
    _check(_lib.smpc_server_destroy(srv))
