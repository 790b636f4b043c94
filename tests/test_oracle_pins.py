"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, hand-derived examples, brute-force enumeration, textbook
invariants (contraction, monotone policy iteration, MacQueen bounds),
metamorphic relations, and library routines in special cases."""
import json
import os

import numpy as np
import pytest

import oracle
from workloads import (MDPInstance, config1, config2, config3, config4, deterministic_chain,
                       random_dense_mdp)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        d = json.load(f)
    inst = MDPInstance(d["S"], d["A"], np.asarray(d["row_ptr"], np.int64),
                       np.asarray(d["col"], np.int32), np.asarray(d["val"], np.float64),
                       np.asarray(d["cost"], np.float64), float(d["gamma"]), name=name)
    return inst, d


def single_state(g, gamma):
    A = len(g)
    return MDPInstance(1, A, np.arange(A + 1, dtype=np.int64), np.zeros(A, np.int32),
                       np.ones(A), np.asarray(g, np.float64), gamma, name="single")


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("gamma", [0.0, 0.5, 0.9, 0.999])
def test_single_state_closed_form(gamma):
    g = [0.7, 0.3, 0.9, 0.3]
    r = oracle.policy_iteration(single_state(g, gamma))
    assert r["pi"][0] == 1  # lowest index among the tied minima 0.3
    np.testing.assert_allclose(r["v"][0], 0.3 / (1.0 - gamma), rtol=1e-14)


@pytest.mark.parametrize("n,gamma", [(12, 0.9), (40, 0.99)])
def test_chain_closed_form(n, gamma):
    inst = deterministic_chain(n, c_adv=1.5, c_stay=2.0, gamma=gamma)
    r = oracle.policy_iteration(inst)
    s = np.arange(n)
    expect = 1.5 * (1.0 - gamma ** (n - 1 - s)) / (1.0 - gamma)
    np.testing.assert_allclose(r["v"], expect, rtol=1e-12, atol=1e-12)
    assert np.all(r["pi"] == 0)  # advance; the absorbing end ties at 0 -> lowest index


@pytest.mark.parametrize("name", ["two_state_hand.json", "two_state_tie.json"])
def test_golden_hand_examples(name):
    inst, d = _load_golden(name)
    r = oracle.policy_iteration(inst)
    np.testing.assert_allclose(r["v"], d["v_star"], rtol=0, atol=1e-13)
    assert r["pi"].tolist() == d["pi_star"]
    Q = oracle.q_values(inst, np.asarray(d["v_star"]))
    np.testing.assert_array_equal(Q, np.asarray(d["q_star"]))
    Tv, pi, res = oracle.bellman(inst, np.asarray(d["v_star"]))
    assert res == 0.0 and pi.tolist() == d["pi_star"]


def test_maze_absorbing_closed_forms():
    inst = config3(H=30, W=30, seed=3)
    r = oracle.policy_iteration(inst, method="sparse")
    obst = inst.meta["obstacle"]
    goal = inst.meta["goal"]
    assert abs(r["v"][goal]) <= 1e-12 * np.abs(r["v"]).max()
    np.testing.assert_allclose(r["v"][obst], 10.0 / (1.0 - inst.gamma), rtol=1e-12)
    assert r["res"] <= 1e-10


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("S,A,seed", [(2, 3, 0), (3, 3, 1), (4, 4, 2), (5, 3, 3), (5, 2, 4)])
def test_brute_force_enumeration(S, A, seed):
    inst = random_dense_mdp(S, A, gamma=0.9, seed=seed, density=0.6)
    best, vals = oracle.brute_force(inst)
    r = oracle.policy_iteration(inst)
    np.testing.assert_allclose(r["v"], best, rtol=1e-12, atol=1e-12)
    # the returned policy is in the optimal set: its value equals v*
    v_pi = dict((tuple(p.tolist()), v) for p, v in vals)[tuple(r["pi"].tolist())]
    np.testing.assert_allclose(v_pi, best, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("S,A,seed", [(3, 3, 1), (4, 3, 2)])
def test_brute_force_maximize(S, A, seed):
    """Maximising rewards r gives v* = -(v* minimising costs -r), and a single
    state reaches max_a r(a) / (1 - gamma)."""
    inst = random_dense_mdp(S, A, gamma=0.9, seed=seed, density=0.6)
    best_max, _ = oracle.brute_force(inst, maximize=True)
    neg = MDPInstance(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, -inst.cost, inst.gamma)
    best_min, _ = oracle.brute_force(neg)
    np.testing.assert_allclose(best_max, -best_min, rtol=1e-12, atol=1e-12)
    one = random_dense_mdp(1, 4, gamma=0.8, seed=3)
    v1, _ = oracle.brute_force(one, maximize=True)
    np.testing.assert_allclose(v1, [one.cost.max() / (1 - 0.8)], rtol=1e-12)


# ---------------------------------------------------------------- invariants

def test_policy_iteration_trajectory_config1():
    inst = config1()
    r = oracle.policy_iteration(inst, check_monotone=True)
    assert r["res"] <= 1e-10
    assert r["iters"] < 20
    lo, hi = oracle.macqueen_bounds(inst, r["v"])
    assert np.all(lo - 1e-12 <= r["v"]) and np.all(r["v"] <= hi + 1e-12)


@pytest.mark.parametrize("make", [lambda: config1(S=300, seed=5),
                                  lambda: config2(S=3000, A=4, seed=1),
                                  lambda: config4(S=3000, A=4, seed=2)])
def test_macqueen_bounds_bracket(make):
    inst = make()
    r = oracle.policy_iteration(inst)
    rng = np.random.default_rng(0)
    for scale in (1.0, 10.0):
        v = r["v"] + scale * rng.standard_normal(inst.S)
        lo, hi = oracle.macqueen_bounds(inst, v)
        tol = 1e-9 * max(1.0, np.abs(r["v"]).max())
        assert np.all(lo <= r["v"] + tol) and np.all(r["v"] <= hi + tol)


def test_contraction_of_T():
    inst = config1(S=200, seed=3)
    rng = np.random.default_rng(1)
    P = oracle.to_csr(inst)
    for _ in range(5):
        u, w = rng.standard_normal(inst.S), rng.standard_normal(inst.S)
        Tu, _, _ = oracle.bellman(inst, u, P)
        Tw, _, _ = oracle.bellman(inst, w, P)
        assert np.max(np.abs(Tu - Tw)) <= inst.gamma * np.max(np.abs(u - w)) * (1 + 1e-12)


def test_evaluation_methods_agree_and_match_fixed_point():
    inst = config2(S=2000, A=4, seed=4)
    pi = np.random.default_rng(2).integers(0, inst.A, inst.S).astype(np.int32)
    vd, rd = oracle.evaluate_policy(inst, pi, method="dense")
    vc, rc = oracle.evaluate_policy(inst, pi, method="certified")
    vf = oracle.evaluate_policy_fixed_point(inst, pi)
    scale = np.abs(vd).max()
    assert np.max(np.abs(vd - vc)) <= 1e-11 * scale
    assert np.max(np.abs(vd - vf)) <= 1e-11 * scale
    assert rd <= 1e-12 * scale and rc <= 1e-12 * scale


def test_vi_and_mpi_reach_same_fixed_point():
    inst = config1(S=400, seed=7)
    r = oracle.policy_iteration(inst)
    v_vi, pi_vi, res_vi, _ = oracle.value_iteration(inst, tol=1e-11)
    v_m, pi_m, res_m, _ = oracle.modified_policy_iteration(inst, m=5, tol=1e-11)
    bound = 1e-11 / (1 - inst.gamma)
    assert np.max(np.abs(v_vi - r["v"])) <= 2 * bound
    assert np.max(np.abs(v_m - r["v"])) <= 2 * bound
    assert np.array_equal(pi_vi, r["pi"]) and np.array_equal(pi_m, r["pi"])


def test_mpi_one_step_is_value_iteration():
    inst = config1(S=200, seed=8)
    a = oracle.modified_policy_iteration(inst, m=1, tol=1e-9)
    b = oracle.value_iteration(inst, tol=1e-9)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[3] == b[3]


# ---------------------------------------------------------------- metamorphic

def _with(inst, **kw):
    d = dict(S=inst.S, A=inst.A, row_ptr=inst.row_ptr, col=inst.col, val=inst.val,
             cost=inst.cost, gamma=inst.gamma, name=inst.name)
    d.update(kw)
    return MDPInstance(**d)


def test_metamorphic_cost_shift_and_scale():
    inst = config1(S=300, seed=11)
    r = oracle.policy_iteration(inst)
    c, lam = 2.5, 3.0
    r2 = oracle.policy_iteration(_with(inst, cost=inst.cost + c))
    np.testing.assert_allclose(r2["v"], r["v"] + c / (1 - inst.gamma), rtol=1e-11)
    assert np.array_equal(r2["pi"], r["pi"])
    r3 = oracle.policy_iteration(_with(inst, cost=lam * inst.cost))
    np.testing.assert_allclose(r3["v"], lam * r["v"], rtol=1e-11)
    assert np.array_equal(r3["pi"], r["pi"])


def _permute_states(inst, perm):
    """State s of the new MDP is state perm[s] of the old one."""
    S, A = inst.S, inst.A
    inv = np.empty(S, np.int64)
    inv[perm] = np.arange(S)
    rows, cols, vals, costs, ptr = [], [], [], [], [0]
    for s_new in range(S):
        s_old = perm[s_new]
        for a in range(A):
            r = s_old * A + a
            c = inv[inst.col[inst.row_ptr[r]:inst.row_ptr[r + 1]]]
            v = inst.val[inst.row_ptr[r]:inst.row_ptr[r + 1]]
            o = np.argsort(c)
            cols.append(c[o])
            vals.append(v[o])
            costs.append(inst.cost[r])
            ptr.append(ptr[-1] + len(c))
    return _with(inst, row_ptr=np.asarray(ptr, np.int64), col=np.concatenate(cols).astype(np.int32),
                 val=np.concatenate(vals), cost=np.asarray(costs))


def test_metamorphic_state_relabelling():
    inst = config1(S=150, seed=12)
    r = oracle.policy_iteration(inst)
    perm = np.random.default_rng(3).permutation(inst.S)
    r2 = oracle.policy_iteration(_permute_states(inst, perm))
    np.testing.assert_allclose(r2["v"], r["v"][perm], rtol=1e-12)
    assert np.array_equal(r2["pi"], r["pi"][perm])


def test_metamorphic_action_permutation():
    inst = config1(S=150, A=4, seed=13)
    r = oracle.policy_iteration(inst)
    sigma = np.array([2, 0, 3, 1])  # new action a is old action sigma[a]
    S, A = inst.S, inst.A
    rows_old = (np.arange(S)[:, None] * A + sigma[None, :]).reshape(-1)
    ptr = [0]
    cols, vals = [], []
    for r_old in rows_old:
        cols.append(inst.col[inst.row_ptr[r_old]:inst.row_ptr[r_old + 1]])
        vals.append(inst.val[inst.row_ptr[r_old]:inst.row_ptr[r_old + 1]])
        ptr.append(ptr[-1] + len(cols[-1]))
    inst2 = _with(inst, row_ptr=np.asarray(ptr, np.int64), col=np.concatenate(cols),
                  val=np.concatenate(vals), cost=inst.cost[rows_old])
    r2 = oracle.policy_iteration(inst2)
    np.testing.assert_allclose(r2["v"], r["v"], rtol=1e-12)
    Q = oracle.q_values(inst, r["v"])
    part = np.partition(Q, 1, axis=1)
    clear = (part[:, 1] - part[:, 0]) > 1e-9
    assert np.array_equal(sigma[r2["pi"]][clear], r["pi"][clear])


# ---------------------------------------------------------------- fp16 copy

def test_fp16_row_correction_special_values():
    # probabilities exactly representable in fp16 need no correction
    inst = deterministic_chain(5)
    h, c = oracle.fp16_with_row_correction(inst)
    assert np.all(c == 0.0) and np.all(h.astype(np.float64) == inst.val)
    inst2 = _with(single_state([1.0, 2.0], 0.9), row_ptr=np.array([0, 3, 6], np.int64),
                  col=np.zeros(6, np.int32), val=np.array([0.1, 0.2, 0.7, 0.25, 0.25, 0.5]))
    h2, c2 = oracle.fp16_with_row_correction(inst2)
    # 0.1, 0.2 and 0.7 round in fp16 to 1638/16384, 1638/8192 and 1434/2048
    expect0 = 1.0 - (1638 / 16384 + 1638 / 8192 + 1434 / 2048)
    assert c2[0] == expect0 and c2[1] == 0.0


# ---------------------------------------------------------------- planted mistakes

def _pin_suite():
    """A compact set of the pins above; returns the number that fail."""
    fails = 0
    checks = [lambda: test_single_state_closed_form(0.9),
              lambda: test_chain_closed_form(12, 0.9),
              lambda: test_golden_hand_examples("two_state_hand.json"),
              lambda: test_golden_hand_examples("two_state_tie.json"),
              lambda: test_brute_force_enumeration(3, 3, 1)]
    for c in checks:
        try:
            c()
        except Exception:
            fails += 1
    return fails


def _mut_q_no_gamma(inst, v, P=None):
    P = oracle.to_csr(inst) if P is None else P
    return (inst.cost + (P @ np.asarray(v, np.float64))).reshape(inst.S, inst.A)


def _mut_q_sign(inst, v, P=None):
    P = oracle.to_csr(inst) if P is None else P
    return (inst.cost - inst.gamma * (P @ np.asarray(v, np.float64))).reshape(inst.S, inst.A)


def _mut_q_transposed(inst, v, P=None):
    P = oracle.to_csr(inst) if P is None else P
    # P^T has shape S x S*A; apply it to a state-major v reshaped per action
    Pt = P.T.tocsr()
    w = np.zeros(inst.S * inst.A)
    w[:inst.S] = Pt[:, :inst.S] @ np.asarray(v, np.float64)[:inst.S] if inst.S * inst.A >= inst.S else 0
    return (inst.cost + inst.gamma * w).reshape(inst.S, inst.A)


def _mut_policy_rows_shift(inst, pi, P=None):
    import scipy.sparse as sp  # noqa: F401
    P = oracle.to_csr(inst) if P is None else P
    rows = (np.arange(inst.S, dtype=np.int64) * inst.A + np.asarray(pi, np.int64) + 1) % (inst.S * inst.A)
    return P[rows], inst.cost[rows]


@pytest.mark.parametrize("target,mutant", [
    ("q_values", _mut_q_no_gamma),
    ("q_values", _mut_q_sign),
    ("q_values", _mut_q_transposed),
    ("policy_system", _mut_policy_rows_shift),
])
def test_planted_mistakes_are_caught(monkeypatch, target, mutant):
    from oracle import mdp_oracle
    assert _pin_suite() == 0
    monkeypatch.setattr(mdp_oracle, target, mutant)
    assert _pin_suite() >= 1


def test_planted_argmax_is_caught(monkeypatch):
    from oracle import mdp_oracle

    def bellman_max(inst, v, P=None):
        Q = mdp_oracle.q_values(inst, v, P)
        return Q.max(axis=1), Q.argmax(axis=1).astype(np.int32), float(
            np.max(np.abs(Q.max(axis=1) - v)))
    monkeypatch.setattr(mdp_oracle, "bellman", bellman_max)
    assert _pin_suite() >= 1


def test_policy_parity_rule():
    Q = np.array([[1.0, 1.0 + 1e-12, 3.0], [2.0, 1.0, 5.0]])
    pi_star = np.array([0, 1])
    ok = oracle.policy_parity(None, Q, np.array([1, 1]), pi_star, tau=1e-9)
    assert ok["mismatch_outside_band"] == 0 and ok["not_tau_optimal"] == 0 and ok["ties_1e9"] == 1
    bad = oracle.policy_parity(None, Q, np.array([0, 0]), pi_star, tau=1e-9)
    assert bad["mismatch_outside_band"] == 1 and bad["not_tau_optimal"] == 1


def test_q_values_states_matches_full_q():
    inst = config2(S=2000, A=4, seed=9)
    v = np.random.default_rng(2).standard_normal(inst.S)
    states = np.array([0, 5, 1999, 777])
    Q = oracle.q_values(inst, v)
    np.testing.assert_allclose(oracle.q_values_states(inst, v, states), Q[states], rtol=1e-13,
                               atol=1e-13)


@pytest.mark.parametrize("block_rows", [1, 7, 1 << 22])
def test_bellman_streamed_matches_statewise_definition(block_rows):
    """The block-streamed sweep against the state-by-state definition (a dot
    product per stored row) on ragged and banded instances, for block sizes
    that cut rows of one state apart and that hold the whole matrix."""
    for inst in (random_dense_mdp(23, 3, 0.9, seed=4, density=0.4), config2(S=600, A=3, seed=2)):
        v = np.random.default_rng(8).standard_normal(inst.S)
        Tv, pi, res = oracle.bellman_streamed(inst, v, block_rows=block_rows)
        Tv2, pi2, res2 = oracle.bellman_streamed(inst, v, block_rows=block_rows, workers=3)
        assert np.array_equal(Tv, Tv2) and np.array_equal(pi, pi2) and res == res2
        Q = oracle.q_values_states(inst, v, np.arange(inst.S))
        np.testing.assert_allclose(Tv, Q.min(axis=1), rtol=1e-13, atol=1e-13)
        part = np.partition(Q, 1, axis=1)
        clear = part[:, 1] - part[:, 0] > 1e-12
        assert np.array_equal(pi[clear], Q.argmin(axis=1)[clear])
        assert abs(res - np.max(np.abs(Q.min(axis=1) - v))) <= 1e-13


def test_bellman_streamed_rejects_empty_rows():
    inst = random_dense_mdp(5, 2, 0.9, seed=1)
    rp = inst.row_ptr.copy()
    rp[3] = rp[2]  # row 2 loses its entries
    bad = MDPInstance(inst.S, inst.A, rp, inst.col, inst.val, inst.cost, inst.gamma)
    with pytest.raises(ValueError):
        oracle.bellman_streamed(bad, np.zeros(inst.S))
