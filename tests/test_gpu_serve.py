"""Serving: continuous batching.  Requests submitted while others run are
admitted as memory frees up; each result equals the request solved alone."""
import time

import numpy as np
import pytest

from workloads import config1, config2, config4, config5_instance, config5_requests

pytestmark = pytest.mark.gpu


def _requests():
    reqs = [r for r in config5_requests(300, seed=8) if r["S"] <= 40000][:8]
    insts = [config5_instance(r) for r in reqs]
    insts += [config1(S=800, seed=2), config2(S=7000, A=4, seed=3), config4(S=6000, A=6, seed=4)]
    return insts


def _alone(inst, precision):
    import paper_2502_14474_amd as m
    with m.MDP.from_instance(inst, low_precision=1 if precision == 1 else 0) as h:
        return h.solve(precision=precision, alpha=1e-2)


@pytest.mark.parametrize("precision,launch", [(1, 0), (0, 0), (1, 1), (1, 2)])
def test_server_results_equal_alone_with_staggered_arrivals(precision, launch):
    # launch 0: the default (direct launches for a server); 1: graph replays; 2: direct launches
    import paper_2502_14474_amd as m
    insts = _requests()
    print(f"[case] server precision={precision} launch={launch} with {len(insts)} requests", flush=True)
    ref = [_alone(i, precision) for i in insts]
    with m.Server(precision=precision, alpha=1e-2, max_batch=4, launch=launch) as srv:
        ids = []
        for k, inst in enumerate(insts):
            ids.append(srv.submit(inst, borrow=(k % 2 == 1)))
            if k % 3 == 2:
                time.sleep(0.01)  # later requests arrive while earlier ones run
        outs = [srv.wait(i) for i in ids]
        info = srv.info()
    assert info["resident"] == 0 and info["queued"] == 0 and info["rounds"] > 0
    for k, ((v, pi, st), (vr, pir, str_)) in enumerate(zip(outs, ref)):
        assert st["status"] == 0 and str_["status"] == 0
        assert np.array_equal(v, vr), (k, np.max(np.abs(v - vr)))
        assert np.array_equal(pi, pir), k
        assert st["bellman_sweeps"] == str_["bellman_sweeps"]
        assert st["inner_iters"] == str_["inner_iters"]
        assert st["submit_ms"] <= st["admit_ms"] <= st["finish_ms"]


def test_server_admission_under_small_budget():
    import paper_2502_14474_amd as m
    insts = [config1(S=3000, seed=s) for s in range(5)]
    # a budget that holds about one request at a time: all must still finish
    with m.Server(hbm_budget_bytes=3 << 20, max_batch=8, alpha=1e-2) as srv:
        ids = [srv.submit(i) for i in insts]
        outs = [srv.wait(i) for i in ids]
    for (v, pi, st), inst in zip(outs, insts):
        vr, pir, _ = _alone(inst, 1)
        assert np.array_equal(v, vr) and np.array_equal(pi, pir)
    # admissions are serialised by the budget
    admits = sorted(st["admit_ms"] for _, _, st in outs)
    finishes = sorted(st["finish_ms"] for _, _, st in outs)
    assert all(a >= f - 1e-6 for a, f in zip(admits[1:], finishes[:-1]))


def test_server_rejects_oversized_request():
    import paper_2502_14474_amd as m
    with m.Server(hbm_budget_bytes=1 << 16) as srv:
        with pytest.raises(m.MDPError) as e:
            srv.submit(config1(S=2000, seed=1))
        assert e.value.status == m.native.MDP_E_NOMEM


def test_server_borrowed_invalid_request_fails_at_wait():
    import paper_2502_14474_amd as m
    inst = config1(S=200, seed=3)
    bad = config1(S=200, seed=3)
    bad.val = bad.val.copy()
    bad.val[5] = -0.5
    with m.Server(alpha=1e-2) as srv:
        good = srv.submit(inst, borrow=True)
        rid = srv.submit(bad, borrow=True)
        with pytest.raises(m.MDPError) as e:
            srv.wait(rid)
        assert e.value.status == m.native.MDP_E_INVAL
        v, pi, st = srv.wait(good)
        assert st["status"] == 0


def test_server_beside_threads_that_create_and_destroy_handles():
    """Handles created, solved and destroyed on other host threads while a
    server captures graphs and admits and retires requests: every result equals
    the same solve alone (allocation, stream and control-slot recycling and the
    capture lock are shared across the library)."""
    import threading

    import paper_2502_14474_amd as m
    insts = _requests()[:6]
    ref = [_alone(i, 1) for i in insts]
    side = [config2(S=5000 + 700 * t, A=4, seed=20 + t) for t in range(3)]
    side_ref = [_alone(i, 0) for i in side]
    errors = []

    def churn(t):
        try:
            for _ in range(4):
                v, pi, st = _alone(side[t], 0)
                if not (np.array_equal(v, side_ref[t][0]) and np.array_equal(pi, side_ref[t][1])):
                    errors.append(f"thread {t}: result differs")
        except Exception as e:  # reported below
            errors.append(f"thread {t}: {e}")

    print(f"[case] server beside 3 churning threads, {len(insts)} requests", flush=True)
    with m.Server(precision=1, alpha=1e-2, max_batch=3) as srv:
        threads = [threading.Thread(target=churn, args=(t,)) for t in range(3)]
        for th in threads:
            th.start()
        ids = [srv.submit(inst, borrow=(k % 2 == 0)) for k, inst in enumerate(insts * 2)]
        outs = [srv.wait(i) for i in ids]
        for th in threads:
            th.join(timeout=90)
        assert not any(th.is_alive() for th in threads)
    assert not errors, errors
    for k, (v, pi, st) in enumerate(outs):
        vr, pir, _ = ref[k % len(insts)]
        assert st["status"] == 0 and np.array_equal(v, vr) and np.array_equal(pi, pir), k


def test_server_autotunes_each_new_class_once(tmp_path, monkeypatch):
    """autotune=True: the first request of each class times the lane widths at
    admission and stores the winner; every request of the class then runs
    with it, so each result equals mdp_solve on a handle created afterwards
    (which starts from the stored width)."""
    import json
    import paper_2502_14474_amd as m
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MDP_TUNE_CACHE", str(cache))
    insts = [config1(S=3000, A=4, k=10, seed=s) for s in range(3)]  # one class, three requests
    insts += [config2(S=7000, A=8, seed=3), config4(S=6000, A=6, k=24, seed=4)]
    print(f"[case] server autotune over {len(insts)} requests", flush=True)
    with m.Server(precision=1, alpha=1e-2, max_batch=4, autotune=True) as srv:
        ids = [srv.submit(i) for i in insts]
        outs = [srv.wait(i) for i in ids]
    widths = json.loads(cache.read_text())
    assert len(widths) == 3, widths  # three classes, each stored once
    assert all(v in (2, 4, 8, 16, 32, 64) for v in widths.values())
    for k, (inst, (v, pi, st)) in enumerate(zip(insts, outs)):
        vr, pir, str_ = _alone(inst, 1)
        assert st["status"] == 0 and str_["status"] == 0
        assert np.array_equal(v, vr) and np.array_equal(pi, pir), k


@pytest.mark.parametrize("precision", [1, 0])
def test_server_size_classes_give_the_alone_results(precision):
    """Two workers (size classes): requests up to split_nnz nonzeros on one,
    larger ones on the other, each on its own stream and engine; every result
    still equals the request solved alone, bit for bit."""
    import paper_2502_14474_amd as m
    insts = _requests()
    split = int(np.median([i.nnz for i in insts]))
    assert any(i.nnz <= split for i in insts) and any(i.nnz > split for i in insts)
    print(f"[case] server size classes, split at {split} nonzeros, precision={precision}", flush=True)
    ref = [_alone(i, precision) for i in insts]
    with m.Server(precision=precision, alpha=1e-2, max_batch=6, split_nnz=split) as srv:
        ids = []
        for k, inst in enumerate(insts):
            ids.append(srv.submit(inst, borrow=(k % 2 == 0)))
            if k % 4 == 3:
                time.sleep(0.005)
        outs = [srv.wait(i) for i in ids]
        info = srv.info()
    assert info["resident"] == 0 and info["queued"] == 0
    for k, ((v, pi, st), (vr, pir, str_)) in enumerate(zip(outs, ref)):
        assert st["status"] == 0 and str_["status"] == 0
        assert np.array_equal(v, vr) and np.array_equal(pi, pir), k
        assert st["inner_iters"] == str_["inner_iters"]


def test_server_small_requests_pass_a_large_head_that_does_not_fit():
    """Budget for one large request plus small ones: a second large request at
    the head of the queue waits for room while the small ones behind it are
    admitted; every result still equals the request solved alone."""
    import paper_2502_14474_amd as m
    big = [config2(S=200000, A=8, seed=s) for s in (5, 6)]
    small = [config1(S=3000, seed=s) for s in range(4)]
    insts = big + small
    print(f"[case] server head-of-line bypass: 2 large ({big[0].nnz} nnz) + 4 small", flush=True)
    with m.Server(hbm_budget_bytes=700 << 20, max_batch=8, alpha=1e-2, split_nnz=0) as srv:
        ids = [srv.submit(i) for i in insts]
        outs = [srv.wait(i) for i in ids]
    admit = [o[2]["admit_ms"] for o in outs]
    assert max(admit[2:]) <= admit[1], admit
    for inst, (v, pi, st) in zip(insts, outs):
        vr, pir, _ = _alone(inst, 1)
        assert st["status"] == 0 and np.array_equal(v, vr) and np.array_equal(pi, pir)
