"""Oracle parity of the mixed-precision paths that the default serving and
batching configuration runs: the server (mixed float32 with float64
refinement, its default) on requests of the serving workload across its whole
state range, mdp_solve_batch in mixed float32, and the full 2000 x 2000 maze in
mixed float32.

Small requests are compared with the oracle's exact policy iteration
(relative value error <= 1e-8 and the policy parity rule).  Requests too large
for that are certified by the oracle's own Bellman sweep at the returned
values, ||v - v*|| <= ||T v - v|| / (1 - gamma), plus a state-by-state check of
the greedy actions on a sample."""
import sys
import time

import numpy as np
import pytest

import oracle
from workloads import config1, config2, config3, config4, config5_instance, config5_requests

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
MIXED_REL = 1e-8


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_check(inst, v, pi, rel_limit, label):
    """Exact policy iteration on the CPU; relative value error and policy parity."""
    t = time.time()
    ref = oracle.policy_iteration(inst, method="auto" if inst.S <= 2500 else "certified")
    rel = np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"]))
    Q = oracle.q_values(inst, ref["v"])
    delta = np.max(np.abs(v - ref["v"]))
    tau = max(1e-9, 2.0 * inst.gamma * (delta + 1e-12 * np.max(np.abs(ref["v"]))))
    pp = oracle.policy_parity(inst, Q, pi, ref["pi"], tau)
    _log(f"[oracle] {label}: S={inst.S} A={inst.A} nnz={inst.nnz} gamma={inst.gamma} rel {rel:.2e} "
         f"tau {tau:.1e} parity {pp} ({time.time() - t:.1f}s)")
    assert rel <= rel_limit, (label, rel)
    assert pp["mismatch_outside_band"] == 0 and pp["not_tau_optimal"] == 0, (label, pp)


def _certified_check(inst, v, pi, rel_limit, label, n_sample=1500):
    """Full-size certificate from the oracle's sweep, and the greedy actions on
    a sample of states recomputed from the oracle's Q row by row."""
    t = time.time()
    Tv, pi_ref, res = oracle.bellman_streamed(inst, v, workers=8)
    rel = res / (1.0 - inst.gamma) / np.max(np.abs(Tv))
    _log(f"[cert] {label}: S={inst.S} A={inst.A} nnz={inst.nnz} gamma={inst.gamma} residual {res:.2e} "
         f"certified rel <= {rel:.2e} ({time.time() - t:.1f}s)")
    assert rel <= rel_limit, (label, rel)
    rng = np.random.default_rng(inst.S)
    states = np.sort(rng.choice(inst.S, size=min(n_sample, inst.S), replace=False))
    Q = oracle.q_values_states(inst, v, states)
    k = np.diff(inst.row_ptr).reshape(inst.S, inst.A)[states].max(axis=1)
    g = np.abs(inst.cost).reshape(inst.S, inst.A)[states].max(axis=1)
    bnd = 2.0 * (k + 2.0) * EPS * (g + inst.gamma * np.max(np.abs(v)))
    part = np.partition(Q, 1, axis=1)  # every instance here has A >= 2
    clear = (part[:, 1] - part[:, 0]) > 2 * bnd
    assert np.array_equal(pi[states][clear], Q.argmin(axis=1)[clear]), label
    assert np.array_equal(pi[states][clear], pi_ref[states][clear]), label


def _serving_requests():
    """Requests of the serving workload's law spread over S in [1e3, 1e6]:
    every gamma, short and long rows, and one explicit request at the corner
    the default mixed path finds hardest (gamma = 0.999, k = 32 columns of which
    16 long jumps, A = 16)."""
    reqs = config5_requests(3000, seed=21)
    picks = []

    def take(pred):
        for r in reqs:
            if all(r["id"] != p["id"] for p in picks) and pred(r):
                picks.append(r)
                return
        raise AssertionError("no request of the stream matches")

    take(lambda r: r["S"] < 1e4 and r["gamma"] == 0.999 and r["k"] >= 17)
    take(lambda r: r["S"] < 1e4 and r["gamma"] == 0.9)
    take(lambda r: 1e4 <= r["S"] < 5e4 and r["gamma"] == 0.999)
    take(lambda r: 1e4 <= r["S"] < 5e4 and r["gamma"] == 0.99 and r["k"] >= 17)
    take(lambda r: 1e5 <= r["S"] < 3e5 and r["gamma"] == 0.999)
    take(lambda r: r["S"] >= 6e5 and r["k"] >= 17 and r["A"] <= 6)
    corner = dict(id=-1, S=30000, A=16, k=32, gamma=0.999, gap=1.0, seed=987654)
    return picks + [corner]


def test_server_default_mixed_matches_oracle_across_the_state_range():
    import paper_2502_14474_amd as m
    reqs = _serving_requests()
    t = time.time()
    insts = [config5_instance(r, workers=16) for r in reqs]
    _log(f"[case] server, default mixed float32: {len(insts)} requests, S "
         f"{[i.S for i in insts]}, generated in {time.time() - t:.1f}s")
    assert any(i.gamma == 0.999 for i in insts) and any(i.nnz // i.rows >= 17 for i in insts)
    assert min(i.S for i in insts) < 1e4 and max(i.S for i in insts) >= 6e5
    # no precision argument: the server's default, mixed float32
    with m.Server(alpha=1e-2, rtol_cert=1e-9, max_batch=8) as srv:
        ids = [srv.submit(inst, borrow=True) for inst in insts]
        outs = [srv.wait(i) for i in ids]
    for inst, (v, pi, st), r in zip(insts, outs, reqs):
        label = f"request S={inst.S} A={inst.A} k={r['k']} gamma={inst.gamma}"
        assert st["status"] == 0, (label, st)
        if inst.S <= 50000:
            _oracle_check(inst, v, pi, MIXED_REL, label)
        else:
            _certified_check(inst, v, pi, MIXED_REL, label)


def test_batch_mixed_fp32_matches_oracle():
    import paper_2502_14474_amd as m
    reqs = [r for r in config5_requests(400, seed=13) if r["S"] <= 20000][:3]
    insts = [config5_instance(r) for r in reqs]
    insts += [config1(S=600, A=4, k=8, seed=31), config2(S=6000, A=4, seed=32),
              config3(H=30, W=40, seed=33), config4(S=4000, A=6, seed=34)]
    _log(f"[case] batch mixed fp32 of {len(insts)} MDPs")
    handles = [m.mdp_create(i.S, i.A, i.row_ptr, i.col, i.val, i.cost, i.gamma,
                            low_precision=m.MDP_BUILD_FP32) for i in insts]
    try:
        vs = [np.empty(i.S) for i in insts]
        pis = [np.empty(i.S, np.int32) for i in insts]
        status, sts = m.mdp_solve_batch(handles, vs, pis, precision=m.MDP_MIXED_FP32, alpha=1e-2,
                                        rtol_cert=1e-9, max_inner=20000)
    finally:
        for h in handles:
            m.mdp_destroy(h)
    assert status == 0
    for k, (inst, v, pi) in enumerate(zip(insts, vs, pis)):
        _oracle_check(inst, v, pi, MIXED_REL, f"batch member {k} ({inst.name})")


def test_config3_full_maze_mixed_fp32():
    """The 2000 x 2000 maze (gamma = 0.999) in mixed float32: certified by the
    oracle's sweep at full size, absorbing cells at their closed forms."""
    import paper_2502_14474_amd as m
    t = time.time()
    inst = config3()
    _log(f"[case] config3 full mixed fp32 S={inst.S} nnz={inst.nnz} generated in {time.time() - t:.1f}s")
    with m.MDP.from_instance(inst, validate=False, low_precision=m.MDP_BUILD_FP32) as h:
        v, pi, st = h.solve(alpha=1e-2, precision=m.MDP_MIXED_FP32, rtol_cert=1e-9, max_inner=20000)
    assert st["status"] == 0, st
    _log(f"[case] config3 mixed solve: {st['time_ms']:.1f} ms, sweeps {st['bellman_sweeps']}, "
         f"inner {st['inner_iters']}, refinements {st['refinements']}")
    obst, goal = inst.meta["obstacle"], inst.meta["goal"]
    scale = 10.0 / (1.0 - inst.gamma)
    assert np.max(np.abs(v[obst] - scale)) <= MIXED_REL * scale
    assert abs(v[goal]) <= MIXED_REL * scale
    _certified_check(inst, v, pi, MIXED_REL, "config3 mixed fp32")
