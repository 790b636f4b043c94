"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and its host-side validation rejects bad MDPs before touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2502_14474_amd import native
from workloads import config1

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "mdp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mdp_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = native.load()
    names = _header_functions()
    assert "mdp_create" in names and "mdp_solve" in names and len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(native.SIGNATURES), "binding and header disagree"


def test_version_and_defaults():
    lib = native.load()
    assert b"gfx950" in lib.mdp_version()
    o = native.SolveOpts()
    lib.mdp_default_solve_opts(C.byref(o))
    assert o.struct_size == C.sizeof(native.SolveOpts)
    assert o.restart == 30 and o.alpha == 1e-4 and o.atol == 1e-8 and o.inner == 0
    e = native.EvalOpts()
    lib.mdp_default_eval_opts(C.byref(e))
    assert e.struct_size == C.sizeof(native.EvalOpts) and e.max_iter == 10000
    c = native.CreateOpts()
    lib.mdp_default_create_opts(C.byref(c))
    assert c.validate == 1 and c.device == -1
    # the binding's structs have the C layout's size (the library fills struct_size)
    assert c.struct_size == C.sizeof(native.CreateOpts)
    so = native.ServerOpts()
    lib.mdp_default_server_opts(C.byref(so))
    assert so.struct_size == C.sizeof(native.ServerOpts)
    assert so.solve.struct_size == C.sizeof(native.SolveOpts) and so.solve.precision == 1
    assert so.admit_threads == 4 and so.retire_threads == 4 and so.max_batch == 256


def _create(S, A, rp, col, val, cost, gamma, **kw):
    lib = native.load()
    o = native.CreateOpts()
    lib.mdp_default_create_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    h = C.c_void_p()
    st = lib.mdp_create(S, A, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                        cost.ctypes.data, gamma, C.byref(o), C.byref(h))
    return st, lib.mdp_last_error().decode(), h


def _small():
    inst = config1(S=20, A=3, k=4, seed=2)
    return (inst.S, inst.A, inst.row_ptr.copy(), inst.col.copy(), inst.val.copy(),
            inst.cost.copy(), inst.gamma)


@pytest.mark.parametrize("mutate,expect", [
    (lambda a: a.update(gamma=1.0), "gamma"),
    (lambda a: a.update(gamma=-0.1), "gamma"),
    (lambda a: a.update(gamma=float("nan")), "gamma"),
    (lambda a: a.update(S=0), "at least 1"),
    (lambda a: a["cost"].__setitem__(5, np.nan), "non-finite cost"),
    (lambda a: a["col"].__setitem__(3, 20), "column index"),
    (lambda a: a["col"].__setitem__(3, -1), "column index"),
    (lambda a: a["val"].__setitem__(7, -0.01), "negative"),
    (lambda a: a["val"].__setitem__(7, a["val"][7] + 1e-6), "sum to 1"),
    (lambda a: a["rp"].__setitem__(4, a["rp"][3]), "row_ptr"),
    (lambda a: a["rp"].__setitem__(0, 1), "row_ptr[0]"),
])
def test_validation_rejects_bad_mdp(mutate, expect):
    S, A, rp, col, val, cost, gamma = _small()
    a = dict(S=S, A=A, rp=rp, col=col, val=val, cost=cost, gamma=gamma)
    mutate(a)
    st, msg, h = _create(a["S"], A, a["rp"], a["col"], a["val"], a["cost"], a["gamma"])
    assert st == native.MDP_E_INVAL, (st, msg)
    assert expect in msg
    assert not h.value


@pytest.mark.parametrize("mode", [0, 2])
def test_row_ptr_checked_on_host_in_every_validation_mode(mode):
    # row_ptr decides which memory the kernels touch, so its structure is
    # checked on the host even when entries are unchecked or checked on the device
    S, A, rp, col, val, cost, gamma = _small()
    rp[4] = rp[3]
    st, msg, h = _create(S, A, rp, col, val, cost, gamma, validate=mode)
    assert st == native.MDP_E_INVAL and "row_ptr" in msg and not h.value


def test_bad_options_rejected():
    S, A, rp, col, val, cost, gamma = _small()
    st, msg, _ = _create(S, A, rp, col, val, cost, gamma, validate=3)
    assert st == native.MDP_E_INVAL and "validate" in msg
    st, msg, _ = _create(S, A, rp, col, val, cost, gamma, lanes_per_row=12)
    assert st == native.MDP_E_INVAL and "lanes_per_row" in msg
    st, msg, _ = _create(S, A, rp, col, val, cost, gamma, low_precision=8)
    assert st == native.MDP_E_INVAL
    st, msg, _ = _create(S, 9000, rp, col, val, cost, gamma)
    assert st == native.MDP_E_NOTSUP


def test_server_rejects_unknown_launch_mode():
    lib = native.load()
    o = native.ServerOpts()
    lib.mdp_default_server_opts(C.byref(o))
    assert o.solve.launch == native.MDP_LAUNCH_AUTO
    o.solve.launch = 5
    srv = C.c_void_p()
    assert lib.mdp_server_create(C.byref(o), C.byref(srv)) == native.MDP_E_INVAL
    assert "launch" in lib.mdp_last_error().decode() and not srv.value


def test_null_handle_calls_fail_cleanly():
    lib = native.load()
    res = C.c_double()
    v = np.zeros(4)
    assert lib.mdp_bellman(None, v.ctypes.data, None, None, C.byref(res)) == native.MDP_E_INVAL
    assert lib.mdp_solve(None, None, v.ctypes.data, v.ctypes.data, None, None) == native.MDP_E_INVAL
    assert lib.mdp_destroy(None) == native.MDP_OK
    assert "handle" in lib.mdp_last_error().decode().lower()


def test_valid_create_without_gpu_reports_device_error():
    """With no GPU the library must fail loudly (no CPU fallback)."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    S, A, rp, col, val, cost, gamma = _small()
    st, msg, h = _create(S, A, rp, col, val, cost, gamma)
    assert st in (native.MDP_E_DEVICE, native.MDP_E_NOMEM), (st, msg)
    assert not h.value


def _rows_from(inst, k_max):
    def fn(s0, s1, col, val, length, cost):
        r0, r1 = s0 * inst.A, s1 * inst.A
        for i, r in enumerate(range(r0, r1)):
            a, b = inst.row_ptr[r], inst.row_ptr[r + 1]
            col[i, :b - a] = inst.col[a:b]
            val[i, :b - a] = inst.val[a:b]
            length[i] = b - a
            cost[i] = inst.cost[r]
    return fn


def test_create_from_rows_reports_row_function_failures():
    """A failing row function or a row longer than k_max is refused on the
    host, before any device work."""
    import paper_2502_14474_amd as m
    inst = config1(S=50, seed=1)

    def broken(s0, s1, col, val, length, cost):
        raise RuntimeError("simulator failed")
    with pytest.raises(m.MDPError) as ei:
        m.mdp_create_from_rows(inst.S, inst.A, 10, broken, inst.gamma)
    assert ei.value.status == native.MDP_E_INVAL and "row function" in str(ei.value)

    def too_long(s0, s1, col, val, length, cost):
        _rows_from(inst, 10)(s0, s1, col, val, length, cost)
        length[0] = 11
    with pytest.raises(m.MDPError) as ei:
        m.mdp_create_from_rows(inst.S, inst.A, 10, too_long, inst.gamma)
    assert ei.value.status == native.MDP_E_INVAL and "k_max" in str(ei.value)


def test_sizes_the_kernels_cannot_index_are_refused():
    """S >= 2^29 (32-bit byte offsets into float64 vectors) and nnz above
    2^31 - 4096 (int32 entry loops) are refused on the host before any array
    past row_ptr[S*A] is read; the small dummy arrays here are never touched."""
    lib = native.load()
    dummy_i64 = np.zeros(4, dtype=np.int64)
    dummy_i32 = np.zeros(4, dtype=np.int32)
    dummy_f64 = np.zeros(4)
    h = C.c_void_p()
    # S = 2^29, A = 1: refused by its state count alone, row_ptr is not read
    st = lib.mdp_create(1 << 29, 1, dummy_i64.ctypes.data, dummy_i32.ctypes.data,
                        dummy_f64.ctypes.data, dummy_f64.ctypes.data, 0.9, None, C.byref(h))
    assert st == native.MDP_E_NOTSUP and "2^29" in lib.mdp_last_error().decode() and not h.value
    # one state, one action, nnz claimed at 2^31 - 4095: refused from row_ptr[S*A]
    rp = np.array([0, (1 << 31) - 4095], dtype=np.int64)
    st = lib.mdp_create(1, 1, rp.ctypes.data, dummy_i32.ctypes.data, dummy_f64.ctypes.data,
                        dummy_f64.ctypes.data, 0.9, None, C.byref(h))
    assert st == native.MDP_E_NOTSUP and "2^31 - 4096" in lib.mdp_last_error().decode()
    # the same limits hold for row functions and for server submissions
    import paper_2502_14474_amd as m
    with pytest.raises(m.MDPError) as ei:
        m.mdp_create_from_rows(1 << 29, 1, 4, lambda *a: None, 0.9)
    assert ei.value.status == native.MDP_E_NOTSUP
    o = native.ServerOpts()
    lib.mdp_default_server_opts(C.byref(o))
    srv = C.c_void_p()
    st = lib.mdp_server_create(C.byref(o), C.byref(srv))
    if st != native.MDP_OK:
        pytest.skip("no server without a GPU: " + lib.mdp_last_error().decode())
    try:
        rid = C.c_int64()
        st = lib.mdp_server_submit(srv, 1 << 29, 1, dummy_i64.ctypes.data, dummy_i32.ctypes.data,
                                   dummy_f64.ctypes.data, dummy_f64.ctypes.data, 0.9, C.byref(rid))
        assert st == native.MDP_E_NOTSUP
        st = lib.mdp_server_submit(srv, 1, 1, rp.ctypes.data, dummy_i32.ctypes.data,
                                   dummy_f64.ctypes.data, dummy_f64.ctypes.data, 0.9, C.byref(rid))
        assert st == native.MDP_E_NOTSUP
    finally:
        lib.mdp_server_destroy(srv)


def test_new_option_defaults_and_entry_point_checks():
    """Defaults of the options added for the preconditioner, CGS2, size-classed
    serving and server autotuning, and the host-side refusals of the
    allocation-free sweep and of device construction (all before any GPU call)."""
    lib = native.load()
    o = native.SolveOpts()
    lib.mdp_default_solve_opts(C.byref(o))
    assert o.precond_degree == 1 and o.gs_passes == 1
    e = native.EvalOpts()
    lib.mdp_default_eval_opts(C.byref(e))
    assert e.precond_degree == 1 and e.gs_passes == 1
    so = native.ServerOpts()
    lib.mdp_default_server_opts(C.byref(so))
    assert so.autotune == 0 and so.split_nnz == 1 << 24
    so.split_nnz = -1
    srv = C.c_void_p()
    assert lib.mdp_server_create(C.byref(so), C.byref(srv)) == native.MDP_E_INVAL
    so.split_nnz = 0
    so.solve.precond_degree = 2
    assert lib.mdp_server_create(C.byref(so), C.byref(srv)) == native.MDP_E_NOTSUP
    so.solve.precond_degree = 1
    so.solve.gs_passes = 2
    assert lib.mdp_server_create(C.byref(so), C.byref(srv)) == native.MDP_E_NOTSUP
    # allocation-free sweep: more sweep tiles than its scratch holds, bad lanes
    assert lib.mdp_bellman_noalloc(70000 * 1024, 1, 70000 * 1024, None, None, None, None, 0.9, None, None,
                                   None, None, 0, None) == native.MDP_E_NOTSUP
    assert lib.mdp_bellman_noalloc(100, 2, 400, None, None, None, None, 0.9, None, None, None, None, 3,
                                   None) == native.MDP_E_INVAL
    assert lib.mdp_bellman_noalloc(100, 2, 100, None, None, None, None, 0.9, None, None, None, None, 0,
                                   None) == native.MDP_E_INVAL  # fewer entries than rows
    # device construction: argument checks come before any allocation or launch
    h = C.c_void_p()
    fake = C.c_void_p(1)
    assert lib.mdp_create_from_device_rows(100, 2, 4, None, None, 0.9, None, C.byref(h)) == native.MDP_E_INVAL
    for k_max in (0, 5000):
        assert lib.mdp_create_from_device_rows(100, 2, k_max, fake, None, 0.9, None, C.byref(h)) == native.MDP_E_INVAL
    assert lib.mdp_create_from_device_rows(1 << 26, 16, 32, fake, None, 0.9, None,
                                           C.byref(h)) == native.MDP_E_NOTSUP
    assert b"2^34" in lib.mdp_last_error()
    k = C.c_void_p()
    assert lib.mdp_load_kernel(b"/nonexistent.hsaco", b"k", C.byref(k)) in (native.MDP_E_INVAL, native.MDP_E_DEVICE)
