"""Python binding of the MI355X inexact-policy-iteration library.

The functions mirror the C ABI of include/mdp.h (same names) and only marshal
arguments: numpy arrays are passed as host pointers, torch tensors as host or
device pointers.  Every step of the computation runs in libmdp.so.
"""
import ctypes as C
import os

import numpy as np

from . import native
from .native import (MDP_FP64, MDP_MIXED_FP32, MDP_MIXED_FP16, MDP_INNER_GMRES,  # noqa: F401
                     MDP_INNER_RICHARDSON, MDP_INNER_BICGSTAB, MDP_INNER_TFQMR, MDP_MINIMIZE_COST, MDP_MAXIMIZE_REWARD,
                     MDP_VALIDATE_NONE, MDP_VALIDATE_HOST, MDP_VALIDATE_DEVICE,
                     MDP_LAUNCH_AUTO, MDP_LAUNCH_GRAPHS, MDP_LAUNCH_DIRECT,
                     MDP_BUILD_FP32, MDP_BUILD_FP16, MDP_OK,
                     MDP_W_MAXITER, MDPError)

__all__ = ["mdp_create", "mdp_create_from_rows", "mdp_bellman", "mdp_bellman_noalloc", "mdp_create_from_device_rows", "mdp_load_kernel", "mdp_policy_apply", "mdp_policy_eval", "mdp_solve",
           "mdp_solve_batch", "Server",
           "mdp_destroy", "mdp_info", "mdp_autotune", "mdp_profile", "mdp_profile_read",
           "mdp_last_error", "MDP", "MDPError"]


def _ptr(a, dtype, n=None, name="array"):
    """Pointer of a numpy array or torch tensor with the given dtype."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
            raise TypeError(f"{name}: need a C-contiguous {np.dtype(dtype)} array")
        if n is not None and a.size < n:
            raise ValueError(f"{name}: need {n} elements, got {a.size}")
        return a.ctypes.data
    import torch
    if isinstance(a, torch.Tensor):
        tdt = {np.float64: torch.float64, np.int32: torch.int32, np.int64: torch.int64}[dtype]
        if a.dtype != tdt or not a.is_contiguous():
            raise TypeError(f"{name}: need a contiguous {tdt} tensor")
        if n is not None and a.numel() < n:
            raise ValueError(f"{name}: need {n} elements, got {a.numel()}")
        return a.data_ptr()
    raise TypeError(f"{name}: numpy array or torch tensor expected")


def mdp_last_error():
    return native.load().mdp_last_error().decode()


def _validate_mode(validate):
    """True/False, or one of "host", "device", "none" (MDP_VALIDATE_*)."""
    modes = {True: native.MDP_VALIDATE_HOST, False: native.MDP_VALIDATE_NONE,
             "host": native.MDP_VALIDATE_HOST, "device": native.MDP_VALIDATE_DEVICE,
             "none": native.MDP_VALIDATE_NONE}
    if validate not in modes:
        raise ValueError(f"validate must be True, False, 'host', 'device' or 'none', not {validate!r}")
    return modes[validate]


def mdp_create(S, A, row_ptr, col, val, cost, gamma, stream=None, device=-1, validate=True,
               low_precision=0, lanes_per_row=0, col_blocks=-1, objective=0):
    """objective: native.MDP_MINIMIZE_COST (cost holds costs) or
    native.MDP_MAXIMIZE_REWARD (cost holds rewards; values come back in
    reward terms).  validate: see _validate_mode."""
    lib = native.load()
    o = native.CreateOpts()
    lib.mdp_default_create_opts(C.byref(o))
    o.col_blocks = col_blocks
    o.objective = objective
    o.stream = stream
    o.device = device
    o.validate = _validate_mode(validate)
    o.low_precision = low_precision
    o.lanes_per_row = lanes_per_row
    h = C.c_void_p()
    nnz = None
    native.check(lib.mdp_create(int(S), int(A), _ptr(row_ptr, np.int64, S * A + 1, "row_ptr"),
                                _ptr(col, np.int32, nnz, "col"), _ptr(val, np.float64, nnz, "val"),
                                _ptr(cost, np.float64, S * A, "cost"), float(gamma), C.byref(o),
                                C.byref(h)))
    return h


def mdp_create_from_rows(S, A, k_max, fn, gamma, stream=None, device=-1, validate=True,
                         low_precision=0, lanes_per_row=0, col_blocks=-1, objective=0):
    """Create a handle from a row function (mdp_create_from_rows in the C
    ABI).  fn(s_begin, s_end, col, val, length, cost) fills, for the states
    [s_begin, s_end), numpy views shaped (rows, k_max) for col (int32) and val
    (float64) and (rows,) for length (int32) and cost (float64), where rows =
    (s_end - s_begin) * A; it is called from several threads at once."""
    lib = native.load()
    o = native.CreateOpts()
    lib.mdp_default_create_opts(C.byref(o))
    o.stream, o.device, o.validate = stream, device, _validate_mode(validate)
    o.low_precision, o.lanes_per_row = low_precision, lanes_per_row
    o.col_blocks, o.objective = col_blocks, objective

    def cb(user, s0, s1, k, colp, valp, lenp, costp):
        try:
            n = int(s1 - s0) * A
            fn(int(s0), int(s1), np.ctypeslib.as_array(colp, shape=(n, k)),
               np.ctypeslib.as_array(valp, shape=(n, k)), np.ctypeslib.as_array(lenp, shape=(n,)),
               np.ctypeslib.as_array(costp, shape=(n,)))
            return 0
        except Exception:  # reported to the library as a failed range
            return 1

    cfn = native.ROWS_FN(cb)
    h = C.c_void_p()
    native.check(lib.mdp_create_from_rows(int(S), int(A), int(k_max), cfn, None, float(gamma),
                                          C.byref(o), C.byref(h)))
    return h


def mdp_destroy(h):
    return native.check(native.load().mdp_destroy(h))


def mdp_load_kernel(path, name):
    """hipFunction_t of kernel `name` in the code object at `path`."""
    k = C.c_void_p()
    native.check(native.load().mdp_load_kernel(os.fsencode(path), name.encode(), C.byref(k)))
    return k


def mdp_create_from_device_rows(S, A, k_max, kernel, user, gamma, stream=None, device=-1,
                                validate="device", low_precision=0, lanes_per_row=0, col_blocks=-1,
                                objective=0):
    """Create a handle from a row kernel run on the device (see
    mdp_device_rows_args in include/mdp.h).  user: a device pointer (int) or
    None, passed to the kernel unchanged."""
    lib = native.load()
    o = native.CreateOpts()
    lib.mdp_default_create_opts(C.byref(o))
    o.col_blocks, o.objective, o.stream, o.device = col_blocks, objective, stream, device
    o.validate, o.low_precision, o.lanes_per_row = _validate_mode(validate), low_precision, lanes_per_row
    h = C.c_void_p()
    native.check(lib.mdp_create_from_device_rows(int(S), int(A), int(k_max), kernel, user, float(gamma),
                                                 C.byref(o), C.byref(h)))
    return h


def mdp_info(h):
    S, A, nnz, L, b = C.c_int64(), C.c_int32(), C.c_int64(), C.c_int32(), C.c_int64()
    native.check(native.load().mdp_info(h, C.byref(S), C.byref(A), C.byref(nnz), C.byref(L),
                                        C.byref(b)))
    return dict(S=S.value, A=A.value, nnz=nnz.value, lanes_per_row=L.value, device_bytes=b.value)


def mdp_autotune(h):
    L = C.c_int32()
    native.check(native.load().mdp_autotune(h, C.byref(L)))
    return L.value


def mdp_profile(h, enable=True, kinds=None, every=1):
    """Record kernel durations: all classes (enable=True), the named classes
    (kinds, names as in native.KERNEL_KINDS), or stop (enable=False); with
    every > 1 only one launch in `every` of each class is timed."""
    mask = 0
    if enable:
        mask = -1 if kinds is None else sum(1 << native.KERNEL_KINDS.index(k) for k in kinds)
    return native.check(native.load().mdp_profile_sampled(h, mask, int(every)))


def mdp_profile_read(h):
    """Per kernel class: launches, summed ms, summed algorithmic bytes."""
    p = native.KernelProfile()
    p.struct_size = C.sizeof(native.KernelProfile)
    native.check(native.load().mdp_profile_read(h, C.byref(p)))
    return {k: dict(launches=p.launches[i], ms=p.ms[i], bytes=p.bytes[i])
            for i, k in enumerate(native.KERNEL_KINDS)}


def mdp_bellman(h, v, Tv=None, policy=None):
    res = C.c_double()
    native.check(native.load().mdp_bellman(h, _ptr(v, np.float64, name="v"),
                                            _ptr(Tv, np.float64, name="Tv"),
                                            _ptr(policy, np.int32, name="policy"), C.byref(res)))
    return res.value


def mdp_bellman_noalloc(S, A, nnz, row_ptr, col, val, cost, gamma, v, Tv=None, policy=None,
                        res_inf=None, lanes_per_row=0, stream=None):
    """The allocation-free sweep on caller device tensors (mdp_bellman_noalloc):
    row_ptr int64, col int32, val/cost/v/Tv/res_inf float64, policy int32, all
    on the current device.  Only enqueues work on `stream` (a raw hipStream_t
    handle, e.g. torch.cuda.current_stream().cuda_stream; None: the null stream)."""
    rows = int(S) * int(A)
    return native.check(native.load().mdp_bellman_noalloc(
        int(S), int(A), int(nnz), _ptr(row_ptr, np.int64, rows + 1, "row_ptr"),
        _ptr(col, np.int32, nnz, "col"), _ptr(val, np.float64, nnz, "val"),
        _ptr(cost, np.float64, rows, "cost"), float(gamma), _ptr(v, np.float64, S, "v"),
        _ptr(Tv, np.float64, S, "Tv"), _ptr(policy, np.int32, S, "policy"),
        _ptr(res_inf, np.float64, 1, "res_inf"), int(lanes_per_row), stream))


def mdp_policy_apply(h, policy, x, y, mode=0):
    return native.check(native.load().mdp_policy_apply(h, _ptr(policy, np.int32, name="policy"),
                                                        _ptr(x, np.float64, name="x"),
                                                        _ptr(y, np.float64, name="y"), int(mode)))


def _stats(history_cap=0):
    st = native.Stats()
    st.struct_size = C.sizeof(native.Stats)
    hist = None
    if history_cap:
        hist = (C.c_double * history_cap)()
        st.history = C.cast(hist, C.POINTER(C.c_double))
        st.history_cap = history_cap
    return st, hist


def _stats_dict(st, hist):
    d = {k: getattr(st, k) for k, _ in native.Stats._fields_ if k not in ("history", "struct_size")}
    if hist is not None:
        d["history"] = list(hist[:st.history_len])
    return d


def mdp_policy_eval(h, policy, v, v0=None, inner=MDP_INNER_GMRES, restart=30, precision=MDP_FP64,
                    rtol=1e-10, max_iter=10000, sync_every=0, precond_degree=1, gs_passes=1,
                    policy_copy=-1):
    lib = native.load()
    o = native.EvalOpts()
    lib.mdp_default_eval_opts(C.byref(o))
    o.inner, o.restart, o.precision, o.rtol, o.max_iter = inner, restart, precision, rtol, max_iter
    o.sync_every, o.precond_degree, o.gs_passes = sync_every, precond_degree, gs_passes
    o.policy_copy = policy_copy
    st, hist = _stats()
    status = native.check(lib.mdp_policy_eval(h, _ptr(policy, np.int32, name="policy"),
                                              _ptr(v0, np.float64, name="v0"),
                                              _ptr(v, np.float64, name="v"), C.byref(o),
                                              C.byref(st)))
    d = _stats_dict(st, hist)
    d["status"] = status
    return d


def mdp_solve(h, v, policy, v0=None, inner=MDP_INNER_GMRES, restart=30, precision=MDP_FP64,
              alpha=1e-4, atol=1e-8, rtol_cert=0.0, max_outer=1000, max_inner=10000,
              sync_every=0, history_cap=1024, precond_degree=1, gs_passes=1, policy_copy=-1):
    lib = native.load()
    o = native.SolveOpts()
    lib.mdp_default_solve_opts(C.byref(o))
    o.inner, o.restart, o.precision, o.alpha, o.atol = inner, restart, precision, alpha, atol
    o.rtol_cert, o.max_outer, o.max_inner, o.sync_every = rtol_cert, max_outer, max_inner, sync_every
    o.precond_degree, o.gs_passes, o.policy_copy = precond_degree, gs_passes, policy_copy
    st, hist = _stats(history_cap)
    status = native.check(lib.mdp_solve(h, _ptr(v0, np.float64, name="v0"),
                                        _ptr(v, np.float64, name="v"),
                                        _ptr(policy, np.int32, name="policy"), C.byref(o),
                                        C.byref(st)))
    d = _stats_dict(st, hist)
    d["status"] = status
    return d


def _solve_opts(lib, inner=MDP_INNER_GMRES, restart=30, precision=MDP_FP64, alpha=1e-4, atol=1e-8,
                rtol_cert=0.0, max_outer=1000, max_inner=10000, sync_every=0, launch=0, precond_degree=1,
                gs_passes=1, policy_copy=-1):
    o = native.SolveOpts()
    lib.mdp_default_solve_opts(C.byref(o))
    o.inner, o.restart, o.precision, o.alpha, o.atol = inner, restart, precision, alpha, atol
    o.rtol_cert, o.max_outer, o.max_inner, o.sync_every = rtol_cert, max_outer, max_inner, sync_every
    o.launch, o.precond_degree, o.gs_passes, o.policy_copy = launch, precond_degree, gs_passes, policy_copy
    return o


def mdp_solve_batch(handles, vs, pis, v0s=None, history_cap=1024, **opts):
    """Solve several MDPs together; vs/pis are per-handle outputs.  Returns
    (status, list of per-MDP stats dicts)."""
    lib = native.load()
    n = len(handles)
    o = _solve_opts(lib, **opts)
    H = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    V = (C.c_void_p * n)(*[_ptr(x, np.float64, name="v") for x in vs])
    P = (C.c_void_p * n)(*[_ptr(x, np.int32, name="policy") for x in pis])
    V0 = None if v0s is None else (C.c_void_p * n)(*[_ptr(x, np.float64, name="v0") for x in v0s])
    stats = (native.Stats * n)()
    hists = []
    for i in range(n):
        stats[i].struct_size = C.sizeof(native.Stats)
        if history_cap:
            hb = (C.c_double * history_cap)()
            hists.append(hb)
            stats[i].history = C.cast(hb, C.POINTER(C.c_double))
            stats[i].history_cap = history_cap
        else:
            hists.append(None)
    status = native.check(lib.mdp_solve_batch(H, n, V0, V, P, C.byref(o), stats))
    return status, [_stats_dict(stats[i], hists[i]) for i in range(n)]


class MDP:
    """Owning wrapper of a handle (numpy in, numpy out)."""

    def __init__(self, S, A, row_ptr, col, val, cost, gamma, **create_kw):
        self.S, self.A, self.gamma = int(S), int(A), float(gamma)
        self.h = mdp_create(S, A, row_ptr, col, val, cost, gamma, **create_kw)

    @classmethod
    def from_instance(cls, inst, **kw):
        return cls(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, inst.cost, inst.gamma, **kw)

    def close(self):
        if self.h is not None:
            mdp_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return mdp_info(self.h)

    def bellman(self, v):
        Tv = np.empty(self.S)
        pi = np.empty(self.S, np.int32)
        res = mdp_bellman(self.h, np.ascontiguousarray(v, np.float64), Tv, pi)
        return Tv, pi, res

    def policy_apply(self, policy, x, mode=0):
        y = np.empty(self.S)
        mdp_policy_apply(self.h, np.ascontiguousarray(policy, np.int32),
                         np.ascontiguousarray(x, np.float64), y, mode)
        return y

    def policy_eval(self, policy, v0=None, **kw):
        v = np.empty(self.S)
        st = mdp_policy_eval(self.h, np.ascontiguousarray(policy, np.int32), v,
                             None if v0 is None else np.ascontiguousarray(v0, np.float64), **kw)
        return v, st

    def solve(self, v0=None, **kw):
        v = np.empty(self.S)
        pi = np.empty(self.S, np.int32)
        st = mdp_solve(self.h, v, pi, None if v0 is None else np.ascontiguousarray(v0, np.float64),
                       **kw)
        return v, pi, st


class Server:
    """Continuous-batching solve server (mdp_server_* in include/mdp.h)."""

    def __init__(self, hbm_budget_bytes=64 << 30, max_batch=256, device=-1, stream=None,
                 admit_threads=4, retire_threads=4, autotune=False, split_nnz=None, trace_path=None,
                 **solve_opts):
        lib = native.load()
        o = native.ServerOpts()
        lib.mdp_default_server_opts(C.byref(o))
        o.hbm_budget_bytes, o.max_batch, o.device, o.stream = hbm_budget_bytes, max_batch, device, stream
        o.admit_threads, o.retire_threads, o.autotune = admit_threads, retire_threads, int(bool(autotune))
        if split_nnz is not None:
            o.split_nnz = split_nnz
        if trace_path is not None:
            o.trace_path = os.fsencode(trace_path)
        solve_opts.setdefault("precision", MDP_MIXED_FP32)
        o.solve = _solve_opts(lib, **solve_opts)
        self.s = C.c_void_p()
        native.check(lib.mdp_server_create(C.byref(o), C.byref(self.s)))
        self.S = {}

    def submit(self, inst, borrow=False):
        """Queue a solve.  borrow=True skips the host copy: the instance's
        arrays must stay alive and unchanged until wait() returns (the
        server keeps a reference to them until then)."""
        rid = C.c_int64()
        fn = native.load().mdp_server_submit_borrowed if borrow else native.load().mdp_server_submit
        native.check(fn(self.s, inst.S, inst.A, _ptr(inst.row_ptr, np.int64),
                        _ptr(inst.col, np.int32), _ptr(inst.val, np.float64),
                        _ptr(inst.cost, np.float64), inst.gamma, C.byref(rid)))
        self.S[rid.value] = (inst.S, inst if borrow else None)
        return rid.value

    def poll(self, rid):
        d = C.c_int32()
        native.check(native.load().mdp_server_poll(self.s, rid, C.byref(d)))
        return bool(d.value)

    def wait(self, rid):
        S, _keep = self.S[rid]
        v = np.empty(S)
        pi = np.empty(S, np.int32)
        st = native.RequestStats()
        st.struct_size = C.sizeof(native.RequestStats)
        try:
            status = native.check(native.load().mdp_server_wait(self.s, rid, v.ctypes.data,
                                                                pi.ctypes.data, C.byref(st)))
        finally:
            del self.S[rid]
        d = {k: getattr(st, k) for k, _ in native.RequestStats._fields_ if k != "struct_size"}
        d["status"] = status
        return v, pi, d

    def info(self):
        q, r, b, n = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        native.check(native.load().mdp_server_info(self.s, C.byref(q), C.byref(r), C.byref(b),
                                                   C.byref(n)))
        return dict(queued=q.value, resident=r.value, resident_bytes=b.value, rounds=n.value)

    def close(self):
        if self.s is not None and self.s.value:
            native.check(native.load().mdp_server_destroy(self.s))
        self.s = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
