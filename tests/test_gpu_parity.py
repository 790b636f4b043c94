"""GPU parity: the HIP path through the C ABI against the CPU oracle, on the
same seeded inputs.  Tolerances follow the floating-point arithmetic of each
step (stated next to each check)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import (MDPInstance, config1, config2, config3, config4, deterministic_chain,
                       random_dense_mdp)

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _mdp(inst, **kw):
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    import paper_2502_14474_amd as m
    print(f"[case] {inst.name} S={inst.S} A={inst.A} nnz={inst.nnz} {kw}", flush=True)
    sys.stdout.flush()
    return m.MDP.from_instance(inst, **kw)


def _row_bound(inst, v):
    """Per-row rounding bound of Q(s,a) = g + gamma * sum p v for two
    different summation orders of k terms: 2 (k + 2) eps (|g| + gamma max|v|)."""
    k = np.diff(inst.row_ptr).astype(np.float64)
    return 2.0 * (k + 2.0) * EPS * (np.abs(inst.cost) + inst.gamma * np.max(np.abs(v)))


def _check_bellman(inst, h, v):
    Tv, pi, res = h.bellman(v)
    Q = oracle.q_values(inst, v)
    bnd = _row_bound(inst, v).reshape(inst.S, inst.A).max(axis=1)
    Tv_ref = Q.min(axis=1)
    assert np.all(np.abs(Tv - Tv_ref) <= bnd), np.max(np.abs(Tv - Tv_ref) / bnd)
    part = np.partition(Q, 1, axis=1) if inst.A > 1 else None
    gap = (part[:, 1] - part[:, 0]) if inst.A > 1 else np.full(inst.S, np.inf)
    clear = gap > 2 * bnd
    ref_pi = Q.argmin(axis=1)
    assert np.array_equal(pi[clear], ref_pi[clear])
    # everywhere: the chosen action is optimal within the rounding bound
    assert np.all(Q[np.arange(inst.S), pi] - Tv_ref <= 2 * bnd)
    ref_res = np.max(np.abs(Tv_ref - v))
    assert abs(res - ref_res) <= np.max(bnd) + 0.0
    return Tv, pi, res


INSTANCES = {
    "c1": lambda: config1(),
    "c2twin": lambda: config2(S=20000, A=8, seed=1),
    "c3twin": lambda: config3(H=64, W=80, seed=1),
    "c4twin": lambda: config4(S=12000, A=16, seed=1),
    "ragged": lambda: random_dense_mdp(37, 3, 0.95, seed=5, density=0.3),
}


@pytest.mark.parametrize("name", list(INSTANCES))
@pytest.mark.parametrize("lanes", [0, 2, 64])
def test_bellman_sweep_matches_oracle(name, lanes):
    inst = INSTANCES[name]()
    rng = np.random.default_rng(7)
    with _mdp(inst, lanes_per_row=lanes) as h:
        for scale in (0.0, 1.0, 100.0):
            v = scale * rng.standard_normal(inst.S)
            _check_bellman(inst, h, v)


def test_bellman_exact_ties_take_lowest_action():
    # config-3 absorbing cells have A identical rows: ties must resolve to action 0
    inst = config3(H=40, W=40, seed=2)
    absorbing = inst.meta["obstacle"].copy()
    absorbing[inst.meta["goal"]] = True
    rng = np.random.default_rng(1)
    with _mdp(inst) as h:
        _, pi, _ = h.bellman(rng.standard_normal(inst.S))
    assert np.all(pi[absorbing] == 0)


@pytest.mark.parametrize("name", ["c1", "c2twin", "c3twin", "ragged"])
def test_policy_apply_matches_oracle(name):
    inst = INSTANCES[name]()
    rng = np.random.default_rng(3)
    pi = rng.integers(0, inst.A, inst.S).astype(np.int32)
    x = rng.standard_normal(inst.S)
    Ppi, gpi = oracle.policy_system(inst, pi)
    k = np.diff(Ppi.indptr).astype(np.float64)
    bnd = 2.0 * (k + 2) * EPS * (np.abs(x) + np.abs(gpi) + inst.gamma * np.max(np.abs(x)))
    with _mdp(inst) as h:
        y0 = h.policy_apply(pi, x, mode=0)
        y1 = h.policy_apply(pi, x, mode=1)
    assert np.all(np.abs(y0 - (x - inst.gamma * (Ppi @ x))) <= bnd)
    assert np.all(np.abs(y1 - (gpi + inst.gamma * (Ppi @ x))) <= bnd)
    # row-stochastic: P_pi 1 = 1, so (I - gamma P_pi) 1 = 1 - gamma
    with _mdp(inst) as h:
        ones = h.policy_apply(pi, np.ones(inst.S), mode=0)
    assert np.max(np.abs(ones - (1 - inst.gamma))) <= 64 * EPS


@pytest.mark.parametrize("S,A,density", [(700, 3, 0.3), (1000, 8, 0.02), (5, 512, 0.5), (3, 1024, 0.7),
                                           (2, 1025, 0.7), (130, 7, 0.9)])
def test_stored_row_order_shapes(S, A, density):
    # Rows are copied into tiles of floor(1024/A) states, action-major inside a
    # tile; these shapes cover full and ragged last tiles, tiles of 1023 and
    # 1024 rows, one-state tiles, and rows longer than the copy's lane groups.
    inst = random_dense_mdp(S, A, 0.9, seed=S + A, density=density)
    rng = np.random.default_rng(S)
    pi = rng.integers(0, A, S).astype(np.int32)
    x = rng.standard_normal(S)
    Ppi, gpi = oracle.policy_system(inst, pi)
    k = np.diff(Ppi.indptr).astype(np.float64)
    bnd = 2.0 * (k + 2) * EPS * (np.abs(x) + np.abs(gpi) + inst.gamma * np.max(np.abs(x)))
    with _mdp(inst) as h:
        _check_bellman(inst, h, x)
        y1 = h.policy_apply(pi, x, mode=1)
    assert np.all(np.abs(y1 - (gpi + inst.gamma * (Ppi @ x))) <= bnd)


def _create_status(inst, validate):
    import ctypes as C
    from paper_2502_14474_amd import native
    lib = native.load()
    o = native.CreateOpts()
    lib.mdp_default_create_opts(C.byref(o))
    o.validate = validate
    h = C.c_void_p()
    st = lib.mdp_create(inst.S, inst.A, inst.row_ptr.ctypes.data, inst.col.ctypes.data, inst.val.ctypes.data,
                        inst.cost.ctypes.data, inst.gamma, C.byref(o), C.byref(h))
    msg = lib.mdp_last_error().decode()
    if h.value:
        lib.mdp_destroy(h)
    return st, msg


def _mutated(inst, edits):
    bad = MDPInstance(inst.S, inst.A, inst.row_ptr.copy(), inst.col.copy(), inst.val.copy(), inst.cost.copy(),
                      inst.gamma, name=inst.name)
    for arr, idx, value in edits:
        getattr(bad, arr)[idx] = value(getattr(bad, arr)[idx]) if callable(value) else value
    return bad


VALIDATION_CASES = {
    "col_high": [("col", 3, 10 ** 6)],
    "col_negative": [("col", 3, -1)],
    "val_negative": [("val", 7, -0.01)],
    "val_nan": [("val", 7, np.nan)],
    "val_inf": [("val", 7, np.inf)],
    "row_sum": [("val", 7, lambda x: x + 1e-6)],
    "cost_inf": [("cost", 5, np.inf)],
    "cost_beats_entry": [("val", 2, -1.0), ("cost", 900, np.nan)],
    "lowest_row_wins": [("val", -3, -1.0), ("col", 40, -5), ("val", 1000, lambda x: x * 2)],
    "tail_only": [("val", -1, lambda x: x + 1e-3)],
}


@pytest.mark.parametrize("case", sorted(VALIDATION_CASES))
@pytest.mark.parametrize("A", [1, 3, 8])
def test_device_validation_matches_host(case, A):
    # rows > 1024 * 256 for A = 8, so the device check runs grid-stride over
    # several rows per thread; A = 1 keeps the natural row order
    inst = config1(S=40000, A=A, k=6, seed=4)
    bad = _mutated(inst, VALIDATION_CASES[case])
    st_h, msg_h = _create_status(bad, 1)
    st_d, msg_d = _create_status(bad, 2)
    print(f"[case] {case} A={A}: {msg_h}", flush=True)
    assert st_h == -1 and st_d == -1
    assert msg_d == msg_h


def test_device_validation_accepts_valid_mdp():
    import paper_2502_14474_amd as m
    inst = config2(S=20000, A=8, seed=2)
    v = np.random.default_rng(0).standard_normal(inst.S)
    with _mdp(inst, validate="host") as h1, _mdp(inst, validate="device") as h2:
        a, b = h1.bellman(v), h2.bellman(v)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    with pytest.raises(ValueError):
        m.MDP.from_instance(inst, validate="sometimes")


def test_policy_apply_rejects_bad_policy():
    import paper_2502_14474_amd as m
    inst = config1(S=50, seed=3)
    with _mdp(inst) as h:
        pi = np.zeros(inst.S, np.int32)
        pi[7] = inst.A
        with pytest.raises(m.MDPError) as e:
            h.policy_apply(pi, np.zeros(inst.S))
        assert e.value.status == m.native.MDP_E_INVAL


@pytest.mark.parametrize("name", ["c1", "c2twin", "c4twin"])
@pytest.mark.parametrize("inner", [0, 1, 2, 3])
def test_policy_eval_matches_exact_solve(name, inner):
    inst = INSTANCES[name]()
    rng = np.random.default_rng(4)
    pi = rng.integers(0, inst.A, inst.S).astype(np.int32)
    v_ref, _ = oracle.evaluate_policy(inst, pi)
    # TFQMR stops on an upper bound tau sqrt(m+1) of the residual, which stays
    # above the rounding floor of 1e-13: it gets 1e-11
    rtol = 1e-11 if inner == 3 else 1e-13
    with _mdp(inst) as h:
        v, st = h.policy_eval(pi, inner=inner, rtol=rtol, max_iter=20000)
    err = np.max(np.abs(v - v_ref)) / np.max(np.abs(v_ref))
    # relative residual 1e-13 in the 2-norm (GMRES, BiCGSTAB; TFQMR: its upper
    # bound on it) or successive differences (Richardson) bounds the error by
    # about cond * 1e-13
    assert err <= 1e-9, (err, st)
    assert st["status"] == 0, st


def test_gmres_exact_in_few_steps_small_system():
    # GMRES with m >= S terminates with the exact solution in at most S steps
    inst = random_dense_mdp(12, 2, 0.9, seed=9, density=0.5)
    pi = np.zeros(inst.S, np.int32)
    v_ref = np.linalg.solve(np.eye(inst.S) - inst.gamma * oracle.policy_system(inst, pi)[0].toarray(),
                            oracle.policy_system(inst, pi)[1])
    with _mdp(inst) as h:
        v, st = h.policy_eval(pi, restart=16, rtol=1e-14, max_iter=16)
    assert st["inner_iters"] <= inst.S
    assert np.max(np.abs(v - v_ref)) <= 1e-12 * np.max(np.abs(v_ref))


def _solve_parity(inst, rel_tol, **kw):
    ref = oracle.policy_iteration(inst, method="auto" if inst.S <= 2500 else "certified")
    vstar = ref["v"]
    with _mdp(inst) as h:
        v, pi, st = h.solve(**kw)
    assert st["status"] == 0, st
    err = np.max(np.abs(v - vstar)) / np.max(np.abs(vstar))
    assert err <= rel_tol, (err, st)
    Q = oracle.q_values(inst, vstar)
    delta = np.max(np.abs(v - vstar))
    tau = max(1e-9, 2 * inst.gamma * (delta + 1e-11 * np.max(np.abs(vstar))))
    pp = oracle.policy_parity(inst, Q, pi, ref["pi"], tau)
    assert pp["mismatch_outside_band"] == 0 and pp["not_tau_optimal"] == 0, pp
    return v, pi, st


@pytest.mark.parametrize("name", ["c1", "c2twin", "c4twin"])
def test_solve_fp64_gmres(name):
    inst = INSTANCES[name]()
    _solve_parity(inst, 1e-9, rtol_cert=1e-10)


def test_solve_fp64_maze_gmres():
    inst = config3(H=48, W=48, seed=4)
    ref = oracle.policy_iteration(inst, method="sparse")
    with _mdp(inst) as h:
        v, pi, st = h.solve(rtol_cert=1e-10)
    assert st["status"] == 0, st
    assert np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"])) <= 1e-9
    obst = inst.meta["obstacle"]
    assert np.allclose(v[obst], 10 / (1 - inst.gamma), rtol=1e-9)
    assert abs(v[inst.meta["goal"]]) <= 1e-9 * np.max(np.abs(v))


@pytest.mark.parametrize("name", ["c1", "c2twin"])
def test_solve_fp64_richardson(name):
    inst = INSTANCES[name]()
    _solve_parity(inst, 1e-9, inner=1, rtol_cert=1e-10, max_inner=500)


@pytest.mark.parametrize("inner", [2, 3])
@pytest.mark.parametrize("name", ["c1", "c2twin", "c4twin", "ragged"])
def test_solve_fp64_bicgstab_tfqmr(name, inner):
    inst = INSTANCES[name]()
    _solve_parity(inst, 1e-9, inner=inner, rtol_cert=1e-10)


@pytest.mark.parametrize("inner", [2, 3])
def test_solve_maze_bicgstab_tfqmr(inner):
    """gamma = 0.999 and absorbing cells: the inner systems are the hardest of
    the workloads (I - gamma P_pi close to singular)."""
    inst = config3(H=48, W=48, seed=4)
    _solve_parity(inst, 1e-9, inner=inner, rtol_cert=1e-10, max_inner=20000)


@pytest.mark.parametrize("inner", [2, 3])
def test_short_recurrence_solvers_reject_mixed_precision(inner):
    import paper_2502_14474_amd as m
    inst = INSTANCES["c1"]()
    with _mdp(inst) as h:
        with pytest.raises(m.MDPError) as ei:
            h.solve(inner=inner, precision=m.MDP_MIXED_FP32)
    assert ei.value.status == m.native.MDP_E_NOTSUP


def test_richardson_one_step_is_value_iteration_bitwise():
    inst = config1(S=400, seed=6)
    with _mdp(inst) as h:
        v_vi = np.zeros(inst.S)
        for _ in range(25):
            Tv, pi_vi, res = h.bellman(v_vi)
            v_vi = Tv
        v, pi, st = h.solve(inner=1, max_inner=1, max_outer=25, atol=1e-300)
    assert st["bellman_sweeps"] == 26 and st["status"] == 1
    assert np.array_equal(v, v_vi)


def test_solve_is_deterministic():
    inst = INSTANCES["c2twin"]()
    with _mdp(inst) as h:
        a = h.solve()
        b = h.solve()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2]["inner_iters"] == b[2]["inner_iters"]


@pytest.mark.parametrize("precision,tol", [(1, 1e-8), (2, 1e-8)])
@pytest.mark.parametrize("name", ["c1", "c4twin", "c3twin", "ragged"])
def test_solve_mixed_precision(name, precision, tol):
    # c3twin and ragged have rows of different lengths (the packed float32
    # copy with per-row offsets, and lanes past short rows)
    inst = INSTANCES[name]()
    _solve_parity(inst, tol, precision=precision, rtol_cert=1e-9)


def test_edge_single_state_and_gamma_zero():
    g = np.array([0.7, 0.3, 0.9, 0.3])
    inst = MDPInstance(1, 4, np.arange(5, dtype=np.int64), np.zeros(4, np.int32), np.ones(4), g, 0.99)
    with _mdp(inst) as h:
        v, pi, st = h.solve(atol=1e-12)
    assert pi[0] == 1 and abs(v[0] - 0.3 / 0.01) <= 1e-9 * 30
    inst0 = config1(S=200, seed=2, gamma=0.0)
    with _mdp(inst0) as h:
        v, pi, st = h.solve()
    Q = inst0.cost.reshape(inst0.S, inst0.A)
    # gamma = 0: v* = min_a g(s, a); the evaluation step (I x = g_pi) rounds at
    # most a few units in the last place through the normalised Krylov vector
    assert np.all(np.abs(v - Q.min(axis=1)) <= 4 * EPS * np.abs(Q.min(axis=1)))
    assert np.array_equal(pi, Q.argmin(axis=1))


def test_edge_single_action_and_chain():
    inst = config1(S=300, A=1, k=5, seed=3)
    ref = oracle.policy_iteration(inst)
    with _mdp(inst) as h:
        v, pi, st = h.solve(atol=1e-12)
    assert np.all(pi == 0) and np.max(np.abs(v - ref["v"])) <= 1e-9 * np.max(np.abs(ref["v"]))
    ch = deterministic_chain(50, c_adv=1.5, c_stay=2.0, gamma=0.95)
    with _mdp(ch) as h:
        v, pi, st = h.solve(atol=1e-12)
    s = np.arange(50)
    expect = 1.5 * (1 - 0.95 ** (49 - s)) / (1 - 0.95)
    assert np.max(np.abs(v - expect)) <= 1e-9 * np.max(expect) and np.all(pi == 0)


def test_device_pointer_round_trip():
    """torch device tensors in and out through the C ABI."""
    import torch
    import paper_2502_14474_amd as m
    inst = config1(S=500, seed=4)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    h = m.mdp_create(inst.S, inst.A, t(inst.row_ptr), t(inst.col), t(inst.val), t(inst.cost),
                     inst.gamma)
    try:
        v = torch.zeros(inst.S, dtype=torch.float64, device=dev)
        pi = torch.zeros(inst.S, dtype=torch.int32, device=dev)
        st = m.mdp_solve(h, v, pi, rtol_cert=1e-10)
        torch.cuda.synchronize()
    finally:
        m.mdp_destroy(h)
    ref = oracle.policy_iteration(inst)
    assert st["status"] == 0
    assert np.max(np.abs(v.cpu().numpy() - ref["v"])) <= 1e-9 * np.max(np.abs(ref["v"]))
    assert np.array_equal(pi.cpu().numpy(), ref["pi"])


@pytest.mark.parametrize("mode", ["host", "device"])
def test_validation_of_device_pointer_inputs(mode):
    """Device inputs: the host check copies them back, the device check reads
    the uploaded copy; both reject a bad probability with the message the host
    check gives for the same arrays in host memory."""
    import torch
    import paper_2502_14474_amd as m
    bad = _mutated(config1(S=3000, A=6, k=7, seed=8), [("val", 1234, -0.25)])
    with pytest.raises(m.MDPError) as ref:
        m.mdp_create(bad.S, bad.A, bad.row_ptr, bad.col, bad.val, bad.cost, bad.gamma, validate="host")
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    with pytest.raises(m.MDPError) as e:
        m.mdp_create(bad.S, bad.A, t(bad.row_ptr), t(bad.col), t(bad.val), t(bad.cost), bad.gamma,
                     validate=mode)
    assert e.value.status == m.native.MDP_E_INVAL and str(e.value) == str(ref.value)


def test_reused_device_memory_gives_fresh_results():
    """Handle memory is recycled through the library's pool: a handle created
    where a larger, different one lived must compute exactly what a handle of
    the same MDP computed before it (no state leaks from freed memory)."""
    import paper_2502_14474_amd as m
    small = config2(S=20000, A=8, seed=3)
    v = np.random.default_rng(2).standard_normal(small.S)
    with _mdp(small) as h:
        ref = h.bellman(v), h.solve(alpha=1e-2)
    for seed in (4, 5):
        big = config2(S=60000, A=8, seed=seed)
        with _mdp(big, low_precision=m.MDP_BUILD_FP32) as hb:
            hb.solve(alpha=1e-2, precision=m.MDP_MIXED_FP32)
        with _mdp(small) as h:
            got = h.bellman(v), h.solve(alpha=1e-2)
        assert all(np.array_equal(a, b) for a, b in zip(got[0][:2], ref[0][:2])) and got[0][2] == ref[0][2]
        assert np.array_equal(got[1][0], ref[1][0]) and np.array_equal(got[1][1], ref[1][1])


def test_autotune_remembers_width_per_class(tmp_path, monkeypatch):
    """The autotuner picks one of the candidate widths, stores it under the
    handle's class key and a later handle of that class starts from it; the
    tuned handle's sweep still matches the oracle."""
    import json
    import paper_2502_14474_amd as m
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MDP_TUNE_CACHE", str(cache))
    inst = config2(S=20000, A=8, seed=3)
    with _mdp(inst) as h:
        L = m.mdp_autotune(h.h)
        assert L in (2, 4, 8, 16, 32, 64)
        assert h.info()["lanes_per_row"] == L
        _check_bellman(inst, h, np.random.default_rng(0).standard_normal(inst.S))
    stored = json.loads(cache.read_text())
    assert len(stored) == 1
    (key, val), = stored.items()
    assert key.startswith("gfx") and key.endswith(":A8_k16_n20") and val == L  # 2.56M and 640K nonzeros
    with _mdp(config2(S=5000, A=8, seed=4)) as h2:
        assert h2.info()["lanes_per_row"] == L
    with _mdp(config2(S=5000, A=8, seed=4), lanes_per_row=2) as h3:
        assert h3.info()["lanes_per_row"] == 2


CB_CASES = {
    "c4twin_b4": (lambda: config4(S=12000, A=16, seed=1), 4),
    "c4twin_b7": (lambda: config4(S=12000, A=16, seed=2), 7),
    "c2twin_b3": (lambda: config2(S=20000, A=8, seed=1), 3),
    "ragged_b2": (lambda: random_dense_mdp(37, 3, 0.95, seed=5, density=0.3), 2),
}


@pytest.mark.parametrize("name", sorted(CB_CASES))
def test_colblocked_sweep_matches_oracle(name):
    """The column-blocked sweep (forced on small instances, slices of uneven
    width included) against the oracle's sweep, with the rounding bound of two
    summation orders."""
    make, blocks = CB_CASES[name]
    inst = make()
    v = 3.0 * np.random.default_rng(4).standard_normal(inst.S)
    with _mdp(inst, col_blocks=blocks) as h:
        _check_bellman(inst, h, v)
        # a second sweep on the same copy (the running sums are overwritten per pass)
        _check_bellman(inst, h, -v)


@pytest.mark.parametrize("precision", [0, 1])
def test_colblocked_solve_certified(precision):
    """Whole solves over the blocked sweep reach the oracle's fixed point."""
    import paper_2502_14474_amd as m
    inst = config4(S=12000, A=16, seed=1)
    kw = dict(col_blocks=5)
    if precision:
        kw["low_precision"] = m.MDP_BUILD_FP32
    with _mdp(inst, **kw) as h:
        v, pi, st = h.solve(alpha=1e-2, precision=precision, rtol_cert=1e-10 if precision == 0 else 1e-9)
    assert st["status"] == 0, st
    Tv, pi_ref, res = oracle.bellman(inst, v)
    rel = res / (1.0 - inst.gamma) / np.max(np.abs(Tv))
    assert rel <= (1e-9 if precision == 0 else 1e-8)


@pytest.mark.parametrize("deg", [1, 3])
@pytest.mark.parametrize("name", ["c2twin_b3", "c4twin_b7", "ragged_b2"])
def test_colblocked_policy_products_match_exact_solve(name, deg):
    """float64 GMRES on handles that carry the column-blocked copy (the
    sweeps run over it, the Arnoldi products over the XCD-partitioned copy of
    P_pi, the preconditioner's products over the plain rows), with and
    without the polynomial preconditioner, against the oracle's exact policy
    evaluation."""
    make, blocks = CB_CASES[name]
    inst = make()
    rng = np.random.default_rng(8)
    pi = rng.integers(0, inst.A, inst.S).astype(np.int32)
    v_ref, _ = oracle.evaluate_policy(inst, pi)
    with _mdp(inst, col_blocks=blocks) as h:
        v, st = h.policy_eval(pi, rtol=1e-13, max_iter=20000, precond_degree=deg)
    err = np.max(np.abs(v - v_ref)) / np.max(np.abs(v_ref))
    assert st["status"] == 0, st
    assert err <= 1e-9, (err, st)


def test_colblocks_option_rules():
    """Forced blocks cost device memory, the automatic rule leaves small
    matrices alone, and unsupported rows are refused."""
    import paper_2502_14474_amd as m
    inst = config2(S=20000, A=8, seed=1)
    with _mdp(inst, col_blocks=0) as h0, _mdp(inst, col_blocks=-1) as ha, _mdp(inst, col_blocks=2) as h2:
        assert ha.info()["device_bytes"] == h0.info()["device_bytes"]
        assert h2.info()["device_bytes"] > h0.info()["device_bytes"] + inst.nnz * 12
    dense = random_dense_mdp(300, 2, 0.9, seed=3, density=1.0)  # 300 entries per row
    with pytest.raises(m.MDPError) as ei:
        m.MDP.from_instance(dense, col_blocks=1)
    assert ei.value.status == m.native.MDP_E_NOTSUP


def test_maximize_reward_matches_brute_force():
    """Reward maximisation against the oracle's enumeration of all policies."""
    import paper_2502_14474_amd as m
    inst = random_dense_mdp(5, 3, 0.9, seed=7, density=0.6)
    best, vals = oracle.brute_force(inst, maximize=True)
    with _mdp(inst, objective=m.MDP_MAXIMIZE_REWARD) as h:
        v, pi, st = h.solve(rtol_cert=1e-12, atol=1e-12)
    assert st["status"] == 0, st
    np.testing.assert_allclose(v, best, rtol=1e-10, atol=1e-10)
    v_pi = dict((tuple(p.tolist()), vv) for p, vv in vals)[tuple(pi.tolist())]
    np.testing.assert_allclose(v_pi, best, rtol=1e-10, atol=1e-10)


def test_maximize_is_negated_minimize_bitwise():
    """Rewards r maximised and costs -r minimised run the same arithmetic: every
    value vector agrees bit for bit up to its sign, policies exactly."""
    import paper_2502_14474_amd as m
    inst = config2(S=20000, A=8, seed=1)
    neg = MDPInstance(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, -inst.cost, inst.gamma)
    x = np.random.default_rng(3).standard_normal(inst.S)
    pol = np.random.default_rng(4).integers(0, inst.A, inst.S).astype(np.int32)
    with _mdp(neg, objective=m.MDP_MAXIMIZE_REWARD) as hmax, _mdp(inst) as hmin:
        vmax, pmax, _ = hmax.solve(alpha=1e-2)
        vmin, pmin, _ = hmin.solve(alpha=1e-2)
        assert np.array_equal(vmax, -vmin) and np.array_equal(pmax, pmin)
        Tmax, qmax, rmax = hmax.bellman(-x)
        Tmin, qmin, rmin = hmin.bellman(x)
        assert np.array_equal(Tmax, -Tmin) and np.array_equal(qmax, qmin) and rmax == rmin
        for mode in (0, 1):
            assert np.array_equal(hmax.policy_apply(pol, -x, mode), -hmin.policy_apply(pol, x, mode))
        emax, _ = hmax.policy_eval(pol, rtol=1e-10)
        emin, _ = hmin.policy_eval(pol, rtol=1e-10)
        assert np.array_equal(emax, -emin)


def test_bicgstab_edge_cases():
    """BiCGSTAB on the degenerate systems: one state (A x = g with A = 1 - gamma
    p_ss), gamma = 0 (A = I), and a warm start close to the solution."""
    import paper_2502_14474_amd as m
    one = MDPInstance(1, 2, np.array([0, 1, 2]), np.array([0, 0], np.int32), np.array([1.0, 1.0]),
                      np.array([0.7, 0.3]), 0.9)
    with _mdp(one) as h:
        v, pi, st = h.solve(inner=m.MDP_INNER_BICGSTAB, atol=1e-12)
    assert st["status"] == 0 and pi[0] == 1
    assert abs(v[0] - 0.3 / (1 - 0.9)) <= 4 * EPS * 3.0
    inst = random_dense_mdp(40, 3, 0.0, seed=2, density=0.3)
    with _mdp(inst) as h:
        v, pi, st = h.solve(inner=m.MDP_INNER_BICGSTAB)
    assert st["status"] == 0
    np.testing.assert_array_equal(v, inst.cost.reshape(inst.S, inst.A).min(axis=1))
    inst = config1(S=300, seed=3)
    pol = np.random.default_rng(1).integers(0, inst.A, inst.S).astype(np.int32)
    v_ref, _ = oracle.evaluate_policy(inst, pol)
    v0 = v_ref + 1e-3 * np.random.default_rng(2).standard_normal(inst.S)
    with _mdp(inst) as h:
        v, st = h.policy_eval(pol, v0=v0, inner=m.MDP_INNER_BICGSTAB, rtol=1e-12)
    assert st["status"] == 0, st
    assert np.max(np.abs(v - v_ref)) <= 1e-10 * np.max(np.abs(v_ref))


def test_colblocked_with_maximize_and_bicgstab():
    """The options compose: a blocked sweep, reward maximisation and BiCGSTAB
    together reach the oracle's fixed point of the negated problem."""
    import paper_2502_14474_amd as m
    inst = config4(S=12000, A=16, seed=3)
    neg = MDPInstance(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, -inst.cost, inst.gamma)
    with _mdp(neg, col_blocks=4, objective=m.MDP_MAXIMIZE_REWARD) as h:
        v, pi, st = h.solve(inner=m.MDP_INNER_BICGSTAB, alpha=1e-2, rtol_cert=1e-10)
    assert st["status"] == 0, st
    Tv, pi_ref, res = oracle.bellman(inst, -v)
    rel = res / (1.0 - inst.gamma) / np.max(np.abs(Tv))
    assert rel <= 1e-9


@pytest.mark.parametrize("name", ["c2twin", "ragged"])
def test_create_from_rows_equals_create(name):
    """A handle built from a row function (called on several threads) holds the
    same MDP as one built from the arrays: sweeps and solves agree bit for bit."""
    import paper_2502_14474_amd as m
    inst = INSTANCES[name]()
    k_max = int(np.max(np.diff(inst.row_ptr)))

    def fn(s0, s1, col, val, length, cost):
        for i, r in enumerate(range(s0 * inst.A, s1 * inst.A)):
            a, b = inst.row_ptr[r], inst.row_ptr[r + 1]
            col[i, :b - a] = inst.col[a:b]
            val[i, :b - a] = inst.val[a:b]
            length[i] = b - a
            cost[i] = inst.cost[r]

    v = np.random.default_rng(6).standard_normal(inst.S)
    hr = m.mdp_create_from_rows(inst.S, inst.A, k_max, fn, inst.gamma)
    try:
        with _mdp(inst) as h:
            Tv, pi, res = h.bellman(v)
            Tv2 = np.empty(inst.S)
            pi2 = np.empty(inst.S, np.int32)
            res2 = m.mdp_bellman(hr, v, Tv2, pi2)
            assert np.array_equal(Tv, Tv2) and np.array_equal(pi, pi2) and res == res2
            x, p1, _ = h.solve(alpha=1e-2)
            x2 = np.empty(inst.S)
            p2 = np.empty(inst.S, np.int32)
            m.mdp_solve(hr, x2, p2, alpha=1e-2)
            assert np.array_equal(x, x2) and np.array_equal(p1, p2)
    finally:
        m.mdp_destroy(hr)
