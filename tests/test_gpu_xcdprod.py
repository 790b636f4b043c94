"""The Arnoldi products on a per-policy copy of P_pi (policy_copy): on handles
that carry the column-blocked copy the copy is cut into column slices (one per
XCD), on other large handles it is P_pi stored contiguously.  Policy
evaluations and solves through it must match the oracle, match the products
through row_ptr to rounding, be deterministic, and follow policy changes on
the same handle."""
import sys

import numpy as np
import pytest

import oracle
from workloads import config2, config3, config4, random_dense_mdp

pytestmark = pytest.mark.gpu

CASES = {
    "c4twin_b7": (lambda: config4(S=12000, A=16, seed=2), 7),
    "c2twin_b3": (lambda: config2(S=20000, A=8, seed=1), 3),
    "ragged_b2": (lambda: random_dense_mdp(37, 3, 0.95, seed=5, density=0.3), 2),
    # 9999 states: no multiple of the 1024-state tiles nor of the 8 slices
    "tail_b1": (lambda: config4(S=9999, A=3, k=5, seed=4), 1),
}


def _mdp(inst, **kw):
    import paper_2502_14474_amd as m
    print(f"[case] {inst.name} S={inst.S} A={inst.A} nnz={inst.nnz} {kw}", flush=True)
    sys.stdout.flush()
    return m.MDP.from_instance(inst, **kw)


@pytest.mark.parametrize("deg", [1, 3])
@pytest.mark.parametrize("name", sorted(CASES))
def test_partitioned_products_match_oracle_and_plain_products(name, deg):
    make, blocks = CASES[name]
    inst = make()
    pi = np.random.default_rng(8).integers(0, inst.A, inst.S).astype(np.int32)
    v_ref, _ = oracle.evaluate_policy(inst, pi)
    scale = np.max(np.abs(v_ref))
    out = {}
    with _mdp(inst, col_blocks=blocks) as h:
        for xcd in (-1, 0, -1):
            v, st = h.policy_eval(pi, rtol=1e-13, max_iter=20000, precond_degree=deg, policy_copy=xcd)
            assert st["status"] == 0, st
            assert np.max(np.abs(v - v_ref)) / scale <= 1e-9, (xcd, st)
            if xcd in out:  # the same copy and policy again: bit for bit
                assert np.array_equal(v, out[xcd])
            out[xcd] = v
    assert np.max(np.abs(out[-1] - out[0])) / scale <= 1e-10


def test_partitioned_products_follow_policy_changes():
    """Evaluations of different policies on one handle, and a solve (whose
    sweeps change the policy between evaluations) on the same handle."""
    inst = config4(S=12000, A=16, seed=3)
    rng = np.random.default_rng(2)
    p1 = rng.integers(0, inst.A, inst.S).astype(np.int32)
    p2 = rng.integers(0, inst.A, inst.S).astype(np.int32)
    with _mdp(inst, col_blocks=4) as h:
        vs = []
        for p in (p1, p2, p1):
            v, st = h.policy_eval(p, rtol=1e-13, max_iter=20000)
            assert st["status"] == 0, st
            vs.append(v)
        v, pi, st = h.solve(alpha=1e-2, rtol_cert=1e-10)
    for p, vv in zip((p1, p2, p1), vs):
        ref, _ = oracle.evaluate_policy(inst, p)
        assert np.max(np.abs(vv - ref)) / np.max(np.abs(ref)) <= 1e-9
    assert np.array_equal(vs[0], vs[2])
    assert st["status"] == 0, st
    ref = oracle.policy_iteration(inst, method="certified")
    err = np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"]))
    assert err <= 1e-9, err
    Q = oracle.q_values(inst, ref["v"])
    tau = max(1e-9, 2 * inst.gamma * (np.max(np.abs(v - ref["v"])) + 1e-11 * np.max(np.abs(ref["v"]))))
    pp = oracle.policy_parity(inst, Q, pi, ref["pi"], tau)
    assert pp["mismatch_outside_band"] == 0 and pp["not_tau_optimal"] == 0, pp


def test_partitioned_products_in_two_passes():
    """A vector of more than 8 x 4 MB: 16 slices, two passes per product.  The
    oracle's sweep-free check at this size: the partitioned and the plain
    products give the same evaluation to rounding, and the evaluation solves
    the policy's linear system (residual checked on the host)."""
    inst = config4(S=4_300_001, A=2, k=4, seed=6, workers=8)
    pi = np.random.default_rng(5).integers(0, inst.A, inst.S).astype(np.int32)
    with _mdp(inst, col_blocks=16) as h:
        va, sa = h.policy_eval(pi, rtol=1e-12, max_iter=5000, policy_copy=-1)
        vb, sb = h.policy_eval(pi, rtol=1e-12, max_iter=5000, policy_copy=0)
    assert sa["status"] == 0 and sb["status"] == 0
    scale = np.max(np.abs(vb))
    assert np.max(np.abs(va - vb)) / scale <= 1e-10
    # v = g_pi + gamma P_pi v, row by row on the host
    rows = np.arange(inst.S) * inst.A + pi
    lo, hi = inst.row_ptr[rows], inst.row_ptr[rows + 1]
    k = hi - lo
    idx = np.repeat(lo, k) + (np.arange(k.sum()) - np.repeat(np.cumsum(k) - k, k))
    pv = np.add.reduceat(inst.val[idx] * va[inst.col[idx]], np.cumsum(k) - k)
    res = va - (inst.cost[rows] + inst.gamma * pv)
    assert np.max(np.abs(res)) / scale <= 1e-9


@pytest.mark.parametrize("blocks", [3, 8])
def test_blocked_sweep_one_launch_equals_pass_by_pass(blocks, monkeypatch):
    """The blocked sweep with all slices in one launch (one slice per XCD,
    parts added afterwards in slice order; enabled by a limit on the parts
    buffer) against the same sweep run one pass per slice with a running sum
    (the default): bit for bit, and both against the oracle's sweep."""
    inst = config4(S=12000, A=16, seed=7)
    v = 2.0 * np.random.default_rng(6).standard_normal(inst.S)
    outs = []
    for limit in (str(1 << 34), None):
        if limit is None:
            monkeypatch.delenv("MDP_CB_PARTS_MAX_BYTES", raising=False)
        else:
            monkeypatch.setenv("MDP_CB_PARTS_MAX_BYTES", limit)
        with _mdp(inst, col_blocks=blocks) as h:
            outs.append(h.bellman(v))
    (Tv0, pi0, r0), (Tv1, pi1, r1) = outs
    assert np.array_equal(Tv0, Tv1) and np.array_equal(pi0, pi1) and r0 == r1
    Q = oracle.q_values(inst, v)
    assert np.max(np.abs(Tv0 - Q.min(axis=1))) <= 1e-12 * np.max(np.abs(Q))


@pytest.mark.parametrize("name", ["c4twin_b7", "tail_b1"])
def test_partitioned_products_in_mixed_solves(name):
    """Mixed float32 solves (float32 basis gathered from the sliced copy, slice
    parts summed in float64, float64 refinement) against the oracle, with and
    without the partitioned products."""
    import paper_2502_14474_amd as m
    make, blocks = CASES[name]
    inst = make()
    ref = oracle.policy_iteration(inst, method="certified")
    scale = np.max(np.abs(ref["v"]))
    Q = oracle.q_values(inst, ref["v"])
    with _mdp(inst, col_blocks=blocks) as h:
        for xcd in (-1, 0):
            v, pi, st = h.solve(alpha=1e-2, precision=m.MDP_MIXED_FP32, rtol_cert=1e-10, policy_copy=xcd)
            assert st["status"] == 0, (xcd, st)
            err = np.max(np.abs(v - ref["v"]))
            assert err / scale <= 1e-9, (xcd, err / scale)
            tau = max(1e-9, 2 * inst.gamma * (err + 1e-11 * scale))
            pp = oracle.policy_parity(inst, Q, pi, ref["pi"], tau)
            assert pp["mismatch_outside_band"] == 0 and pp["not_tau_optimal"] == 0, (xcd, pp)


WHOLE = {
    # no column-blocked copy, at least 2^17 states, short rows: the contiguous copy
    "c2_140k": lambda: config2(S=140_000, A=2, n_band=4, n_jump=2, seed=3),
    "maze_370": lambda: config3(H=370, W=370, gamma=0.95, seed=2),
}


def _policy_residual(inst, pi, v):
    """max |v - (g_pi + gamma P_pi v)| on the host, from the CSR arrays."""
    rows = np.arange(inst.S) * inst.A + pi
    lo, hi = inst.row_ptr[rows], inst.row_ptr[rows + 1]
    k = hi - lo
    idx = np.repeat(lo, k) + (np.arange(k.sum()) - np.repeat(np.cumsum(k) - k, k))
    pv = np.add.reduceat(inst.val[idx] * v[inst.col[idx]], np.cumsum(k) - k)
    return np.max(np.abs(v - (inst.cost[rows] + inst.gamma * pv)))


@pytest.mark.parametrize("name", sorted(WHOLE))
def test_contiguous_policy_copy_solves_the_policy_system(name):
    """At these sizes the oracle's certified solves take minutes, so the
    evaluations are checked against the policy's linear system itself (its
    residual, on the host), the two product paths against each other, and a
    mixed solve against the Bellman equation (the oracle's Q values)."""
    import paper_2502_14474_amd as m
    inst = WHOLE[name]()
    assert inst.S >= 1 << 17
    pi = np.random.default_rng(9).integers(0, inst.A, inst.S).astype(np.int32)
    out = {}
    with _mdp(inst) as h:
        for copy in (-1, 0, -1):
            v, st = h.policy_eval(pi, rtol=1e-13, max_iter=20000, policy_copy=copy)
            assert st["status"] == 0, st
            scale = np.max(np.abs(v))
            assert _policy_residual(inst, pi, v) <= 1e-10 * scale, copy
            if copy in out:
                assert np.array_equal(v, out[copy])
            out[copy] = v
        v, p, st = h.solve(alpha=1e-2, precision=m.MDP_MIXED_FP32, atol=1e-9, rtol_cert=1e-10)
    assert np.max(np.abs(out[-1] - out[0])) <= 1e-10 * np.max(np.abs(out[0]))
    assert st["status"] == 0, st
    Q = oracle.q_values(inst, v)
    assert np.max(np.abs(Q.min(axis=1) - v)) <= 2e-9
    chosen = Q[np.arange(inst.S), p]
    assert np.all(chosen - Q.min(axis=1) <= 1e-9 * max(1.0, np.max(np.abs(v))))


def test_contiguous_policy_copy_in_preconditioned_evaluations():
    """The polynomial preconditioner's Horner products run on the copy too."""
    inst = WHOLE["maze_370"]()
    pi = np.random.default_rng(4).integers(0, inst.A, inst.S).astype(np.int32)
    out = {}
    with _mdp(inst) as h:
        for copy in (-1, 0):
            v, st = h.policy_eval(pi, rtol=1e-13, max_iter=20000, precond_degree=4, policy_copy=copy)
            assert st["status"] == 0, st
            assert _policy_residual(inst, pi, v) <= 1e-10 * np.max(np.abs(v)), copy
            out[copy] = v
    assert np.max(np.abs(out[-1] - out[0])) <= 1e-10 * np.max(np.abs(out[0]))


def test_contiguous_policy_copy_in_mixed_preconditioned_solves():
    """Mixed float32 solves with the polynomial preconditioner: the float32
    Horner steps and Arnoldi products run on the contiguous copy in one launch
    each; the solve meets the Bellman equation (the oracle's Q values) and its
    policy is greedy for its values."""
    import paper_2502_14474_amd as m
    inst = WHOLE["maze_370"]()
    with _mdp(inst) as h:
        v, p, st = h.solve(alpha=1e-2, precision=m.MDP_MIXED_FP32, precond_degree=4, atol=1e-9,
                           rtol_cert=1e-10)
    assert st["status"] == 0, st
    Q = oracle.q_values(inst, v)
    assert np.max(np.abs(Q.min(axis=1) - v)) <= 2e-9
    chosen = Q[np.arange(inst.S), p]
    assert np.all(chosen - Q.min(axis=1) <= 1e-9 * max(1.0, np.max(np.abs(v))))


@pytest.mark.parametrize("inner", [2, 3])  # BiCGSTAB, TFQMR
@pytest.mark.parametrize("name", ["c4twin_b7", "maze_370"])
def test_policy_copy_in_short_recurrence_solvers(name, inner):
    """BiCGSTAB and TFQMR run their products y = x - gamma P_pi x on the copy
    too (sliced on a column-blocked handle, contiguous on a large short-row
    one): the evaluation satisfies the policy's system, repeats bit for bit,
    and agrees with the products through row_ptr to rounding."""
    if name in CASES:
        make, blocks = CASES[name]
        inst, kw = make(), {"col_blocks": blocks}
    else:
        inst, kw = WHOLE[name](), {}
    pi = np.random.default_rng(6).integers(0, inst.A, inst.S).astype(np.int32)
    out = {}
    with _mdp(inst, **kw) as h:
        for copy in (-1, 0, -1):
            v, st = h.policy_eval(pi, rtol=1e-13, max_iter=20000, inner=inner, policy_copy=copy)
            assert st["status"] == 0, (copy, st)
            assert _policy_residual(inst, pi, v) <= 1e-10 * np.max(np.abs(v)), copy
            if copy in out:
                assert np.array_equal(v, out[copy])
            out[copy] = v
    assert np.max(np.abs(out[-1] - out[0])) <= 1e-10 * np.max(np.abs(out[0]))


@pytest.mark.parametrize("inner", [2, 3])
def test_short_recurrence_solves_on_the_sliced_copy(inner):
    """Whole solves with BiCGSTAB / TFQMR on a column-blocked twin: the copy is
    formed again for every new policy of the outer iteration, and the solve
    matches the oracle's exact policy iteration (values and policy parity)."""
    make, blocks = CASES["c4twin_b7"]
    inst = make()
    with _mdp(inst, col_blocks=blocks) as h:
        v, pi, st = h.solve(alpha=1e-2, rtol_cert=1e-10, inner=inner)
    assert st["status"] == 0, st
    ref = oracle.policy_iteration(inst, method="certified")
    err = np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"]))
    assert err <= 1e-9, err
    Q = oracle.q_values(inst, ref["v"])
    tau = max(1e-9, 2 * inst.gamma * (np.max(np.abs(v - ref["v"])) + 1e-11 * np.max(np.abs(ref["v"]))))
    pp = oracle.policy_parity(inst, Q, pi, ref["pi"], tau)
    assert pp["mismatch_outside_band"] == 0 and pp["not_tau_optimal"] == 0, pp


def test_streamed_sweep_on_short_rows():
    """Handles with short rows (no blocked copy) stream each tile's rows in the
    float64 sweep: against the oracle's Q values within the rounding bound of
    two summation orders, bit for bit the one-slice blocked sweep (the same
    fma chain per row), and against the row-by-row sweep (col_blocks = 0)."""
    inst = WHOLE["maze_370"]()
    v = 3.0 * np.random.default_rng(2).standard_normal(inst.S)
    outs = {}
    for cb in (-1, 1, 0):
        with _mdp(inst, col_blocks=cb) as h:
            outs[cb] = h.bellman(v)
    Q = oracle.q_values(inst, v)
    Tv_ref = Q.min(axis=1)
    bound = 8 * 2.2e-16 * (np.abs(inst.cost).max() + inst.gamma * np.abs(v).max()) * 4
    for cb, (Tv, pi, r) in outs.items():
        assert np.max(np.abs(Tv - Tv_ref)) <= bound, cb
    assert np.array_equal(outs[-1][0], outs[1][0]) and np.array_equal(outs[-1][1], outs[1][1])
    assert outs[-1][2] == outs[1][2]
