"""Batched solves: every MDP must come out bitwise the same alone and in the
batch (same kernels bodies, tiling, reduction order and decisions), and match
the oracle."""
import numpy as np
import pytest

import oracle
from workloads import config1, config2, config3, config4, config5_instance, config5_requests

pytestmark = pytest.mark.gpu


def _mix():
    reqs = [r for r in config5_requests(400, seed=3) if r["S"] <= 30000][:5]
    insts = [config5_instance(r) for r in reqs]
    insts += [config1(S=700, A=3, k=6, seed=4), config2(S=9000, A=4, seed=5),
              config3(H=40, W=50, seed=6), config4(S=5000, A=8, seed=7)]
    return insts


@pytest.mark.parametrize("precision,launch", [(0, 1), (1, 1), (0, 2), (1, 2)])
def test_batch_bitwise_equals_alone(precision, launch):
    # launch 1: Arnoldi steps replayed from captured HIP graphs; 2: direct launches
    import paper_2502_14474_amd as m
    insts = _mix()
    print(f"[case] batch of {len(insts)} MDPs precision={precision} launch={launch}", flush=True)
    handles = [m.mdp_create(i.S, i.A, i.row_ptr, i.col, i.val, i.cost, i.gamma,
                            low_precision=1 if precision else 0) for i in insts]
    try:
        alone = []
        for inst, h in zip(insts, handles):
            v = np.empty(inst.S)
            pi = np.empty(inst.S, np.int32)
            st = m.mdp_solve(h, v, pi, precision=precision, alpha=1e-2, max_inner=20000)
            alone.append((v, pi, st))
        vs = [np.empty(i.S) for i in insts]
        pis = [np.empty(i.S, np.int32) for i in insts]
        status, sts = m.mdp_solve_batch(handles, vs, pis, precision=precision, alpha=1e-2,
                                        max_inner=20000, launch=launch)
        # a second call leases the cached engine and replays its graphs
        vs2 = [np.empty(i.S) for i in insts]
        pis2 = [np.empty(i.S, np.int32) for i in insts]
        status2, _ = m.mdp_solve_batch(handles, vs2, pis2, precision=precision, alpha=1e-2,
                                       max_inner=20000, launch=launch)
    finally:
        for h in handles:
            m.mdp_destroy(h)
    assert status == 0 and status2 == 0
    assert all(np.array_equal(a, b) for a, b in zip(vs, vs2))
    assert all(np.array_equal(a, b) for a, b in zip(pis, pis2))
    for k, (inst, (v, pi, st)) in enumerate(zip(insts, alone)):
        assert st["status"] == 0
        assert np.array_equal(vs[k], v), (k, inst.name, np.max(np.abs(vs[k] - v)))
        assert np.array_equal(pis[k], pi), k
        for key in ("outer_iters", "inner_iters", "bellman_sweeps", "policy_applies"):
            assert sts[k][key] == st[key], (k, key, sts[k][key], st[key])
        assert sts[k]["history"] == st["history"]


@pytest.mark.parametrize("precision,launch", [(0, 2), (1, 1)])
def test_batch_bitwise_equals_alone_many_tiles(precision, launch):
    """MDPs of more than 256 product tiles (each thread of the dot and norm
    sums then adds several partials, the last stride ragged) against one of
    fewer: alone and in the batch the results stay bitwise equal."""
    import paper_2502_14474_amd as m
    insts = [config2(S=140000, A=4, seed=11),   # 274 tiles
             config4(S=300000, A=4, seed=12),   # 586 tiles
             config2(S=100000, A=4, seed=13)]   # 196 tiles
    print(f"[case] many-tile batch precision={precision} launch={launch}", flush=True)
    handles = [m.mdp_create(i.S, i.A, i.row_ptr, i.col, i.val, i.cost, i.gamma,
                            low_precision=1 if precision else 0) for i in insts]
    try:
        alone = []
        for inst, h in zip(insts, handles):
            v = np.empty(inst.S)
            pi = np.empty(inst.S, np.int32)
            st = m.mdp_solve(h, v, pi, precision=precision, alpha=1e-2, max_inner=20000, policy_copy=0)
            alone.append((v, pi, st))
        vs = [np.empty(i.S) for i in insts]
        pis = [np.empty(i.S, np.int32) for i in insts]
        status, sts = m.mdp_solve_batch(handles, vs, pis, precision=precision, alpha=1e-2,
                                        max_inner=20000, launch=launch)
    finally:
        for h in handles:
            m.mdp_destroy(h)
    assert status == 0
    for k, (inst, (v, pi, st)) in enumerate(zip(insts, alone)):
        assert st["status"] == 0
        assert np.array_equal(vs[k], v), (k, inst.name, np.max(np.abs(vs[k] - v)))
        assert np.array_equal(pis[k], pi), k
        assert sts[k]["inner_iters"] == st["inner_iters"]
        assert sts[k]["history"] == st["history"]


def test_batch_matches_oracle():
    import paper_2502_14474_amd as m
    insts = [config1(S=500, seed=s) for s in range(6)] + [config2(S=4000, A=3, seed=9)]
    handles = [m.mdp_create(i.S, i.A, i.row_ptr, i.col, i.val, i.cost, i.gamma) for i in insts]
    try:
        vs = [np.empty(i.S) for i in insts]
        pis = [np.empty(i.S, np.int32) for i in insts]
        status, sts = m.mdp_solve_batch(handles, vs, pis, rtol_cert=1e-10)
    finally:
        for h in handles:
            m.mdp_destroy(h)
    assert status == 0
    for inst, v, pi in zip(insts, vs, pis):
        ref = oracle.policy_iteration(inst, method="auto" if inst.S <= 2500 else "certified")
        assert np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"])) <= 1e-9
        Q = oracle.q_values(inst, ref["v"])
        pp = oracle.policy_parity(inst, Q, pi, ref["pi"], 1e-9)
        assert pp["mismatch_outside_band"] == 0 and pp["not_tau_optimal"] == 0


def test_batch_rejects_bad_input():
    import paper_2502_14474_amd as m
    inst = config1(S=100, seed=1)
    h = m.mdp_create(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, inst.cost, inst.gamma)
    try:
        v, pi = np.empty(inst.S), np.empty(inst.S, np.int32)
        with pytest.raises(m.MDPError):
            m.mdp_solve_batch([h, h], [v, v], [pi, pi])
        with pytest.raises(m.MDPError):
            m.mdp_solve_batch([h], [v], [pi], inner=1)
    finally:
        m.mdp_destroy(h)


def test_concurrent_batches_lease_separate_engines():
    """Two host threads run batched solves at once (each leases its own cached
    engine); both give bitwise what the same batch gives alone."""
    import threading

    import paper_2502_14474_amd as m
    groups = [[config1(S=600, seed=s) for s in range(3)], [config2(S=5000, A=4, seed=s) for s in range(3)]]
    handles = [[m.mdp_create(i.S, i.A, i.row_ptr, i.col, i.val, i.cost, i.gamma) for i in g] for g in groups]
    try:
        def run(k, out):
            vs = [np.empty(i.S) for i in groups[k]]
            pis = [np.empty(i.S, np.int32) for i in groups[k]]
            status, _ = m.mdp_solve_batch(handles[k], vs, pis, alpha=1e-2)
            out[k] = (status, vs, pis)

        alone = {}
        for k in range(2):
            run(k, alone)
        together = {}
        threads = [threading.Thread(target=run, args=(k, together)) for k in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=60)
        assert not any(t.is_alive() for t in threads)
    finally:
        for g in handles:
            for h in g:
                m.mdp_destroy(h)
    for k in range(2):
        assert alone[k][0] == 0 and together[k][0] == 0
        assert all(np.array_equal(a, b) for a, b in zip(alone[k][1], together[k][1]))
        assert all(np.array_equal(a, b) for a, b in zip(alone[k][2], together[k][2]))
