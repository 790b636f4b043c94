"""MDP construction on the device (mdp_create_from_device_rows): the row kernel
of tests/kernels/band_hash_rows.hip fills the rows on the GPU; the same MDP
rebuilt on the host by the numpy twin below goes through mdp_create.  The two
handles must hold bitwise the same MDP (same sweep and solve, bit for bit),
and the solve must match the oracle."""
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import MDPInstance

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CODE_OBJECT = os.path.join(ROOT, "tests", "kernels", "band_hash_rows.hsaco")
U64 = np.uint64


def _splitmix64(x):
    # SplitMix64 as Vigna publishes it; uint64 arrays wrap modulo 2^64
    z = x + U64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> U64(30))) * U64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> U64(27))) * U64(0x94D049BB133111EB)
    return z ^ (z >> U64(31))


def _h(seed, r, t):
    return _splitmix64(U64(seed) ^ (r.astype(U64) * U64(1000003) + np.asarray(t).astype(U64)))


def band_hash_instance(S, A, k_max, seed, gamma):
    """The MDP the row kernel writes (its header comment gives the rules)."""
    rows = S * A
    r = np.arange(rows, dtype=np.int64)
    s = r // A
    length = 1 + (_h(seed, r, 0) % U64(k_max)).astype(np.int64)
    shift = (_h(seed, r, 1) % U64(5)).astype(np.int64)
    j = np.arange(k_max, dtype=np.int64)
    cols = (s[:, None] + 3 * j[None, :] + shift[:, None]) % S
    w = (_h(seed, r[:, None], 100 + j[None, :]) >> U64(11)).astype(np.float64) * 2.0 ** -53 + 2.0 ** -10
    valid = j[None, :] < length[:, None]
    key = np.where(valid, cols, np.iinfo(np.int64).max)
    order = np.argsort(key, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, 1)
    w = np.where(valid, np.take_along_axis(w, order, 1), 0.0)  # valid entries sort first
    total = np.cumsum(w, axis=1)[:, -1]  # the sum in sorted order, one term at a time
    val = w / total[:, None]
    row_ptr = np.concatenate([[0], np.cumsum(length)]).astype(np.int64)
    cost = (_h(seed, r, 999) >> U64(11)).astype(np.float64) * 2.0 ** -53
    return MDPInstance(S, A, row_ptr, cols[valid].astype(np.int32), val[valid], cost, gamma,
                       name="band-hash", meta=dict(seed=seed))


def _kernel():
    import paper_2502_14474_amd as m
    assert os.path.isfile(CODE_OBJECT), f"{CODE_OBJECT} is not built; run __graft_entry__.build()"
    return m.mdp_load_kernel(CODE_OBJECT, "band_hash_rows")


def _device_handle(S, A, k_max, seed, gamma, **kw):
    import torch
    import paper_2502_14474_amd as m
    seed_dev = torch.tensor([seed], dtype=torch.int64, device="cuda:0")
    print(f"[case] device rows S={S} A={A} k_max={k_max} seed={seed} {kw}", flush=True)
    sys.stdout.flush()
    h = m.mdp_create_from_device_rows(S, A, k_max, _kernel(), seed_dev.data_ptr(), gamma, **kw)
    torch.cuda.synchronize()
    return h


@pytest.mark.parametrize("S,A,k_max,gamma", [(20000, 4, 12, 0.95), (3001, 7, 32, 0.99)])
def test_device_rows_equal_host_rows_bitwise(S, A, k_max, gamma):
    import paper_2502_14474_amd as m
    seed = 20250214 + S
    inst = band_hash_instance(S, A, k_max, seed, gamma)
    hd = _device_handle(S, A, k_max, seed, gamma)
    hh = m.mdp_create(S, A, inst.row_ptr, inst.col, inst.val, inst.cost, gamma)
    try:
        assert m.mdp_info(hd)["nnz"] == inst.nnz
        rng = np.random.default_rng(1)
        v = rng.standard_normal(S)
        outs = []
        for h in (hd, hh):
            Tv = np.empty(S)
            pi = np.empty(S, np.int32)
            res = m.mdp_bellman(h, v, Tv, pi)
            vs = np.empty(S)
            ps = np.empty(S, np.int32)
            st = m.mdp_solve(h, vs, ps, alpha=1e-2, rtol_cert=1e-10)
            outs.append((Tv, pi, res, vs, ps, st))
        (Tv0, pi0, r0, v0, p0, s0), (Tv1, pi1, r1, v1, p1, s1) = outs
        assert np.array_equal(Tv0, Tv1) and np.array_equal(pi0, pi1) and r0 == r1
        assert np.array_equal(v0, v1) and np.array_equal(p0, p1)
        assert s0["inner_iters"] == s1["inner_iters"] and s0["status"] == 0
    finally:
        m.mdp_destroy(hd)
        m.mdp_destroy(hh)
    # and the solve is the oracle's
    ref = oracle.policy_iteration(inst, method="auto" if S <= 2500 else "certified")
    err = np.max(np.abs(v0 - ref["v"])) / np.max(np.abs(ref["v"]))
    assert err <= 1e-9, err
    Q = oracle.q_values(inst, ref["v"])
    tau = max(1e-9, 2 * gamma * (np.max(np.abs(v0 - ref["v"])) + 1e-11 * np.max(np.abs(ref["v"]))))
    pp = oracle.policy_parity(inst, Q, p0, ref["pi"], tau)
    assert pp["mismatch_outside_band"] == 0 and pp["not_tau_optimal"] == 0, pp


def test_device_rows_reject_lengths_beyond_k_max():
    # the kernel draws len up to its own k_max argument; a k_max of 1 is legal
    # (every row one entry), so plant the failure in the host-side contract
    # instead: k_max outside [1, 4096] is refused before any launch
    import paper_2502_14474_amd as m
    for bad in (0, 5000):
        with pytest.raises(m.MDPError) as e:
            m.mdp_create_from_device_rows(100, 2, bad, _kernel(), None, 0.9)
        assert e.value.status == m.native.MDP_E_INVAL


def test_device_rows_single_entry_rows_and_validation_modes():
    import paper_2502_14474_amd as m
    S, A, k_max, gamma, seed = 5000, 3, 1, 0.9, 7
    inst = band_hash_instance(S, A, k_max, seed, gamma)
    assert inst.nnz == S * A  # every row one entry with probability 1
    for validate in ("device", "host", "none"):
        h = _device_handle(S, A, k_max, seed, gamma, validate=validate)
        try:
            v = np.empty(S)
            p = np.empty(S, np.int32)
            st = m.mdp_solve(h, v, p, rtol_cert=1e-10)
        finally:
            m.mdp_destroy(h)
        ref = oracle.policy_iteration(inst, method="certified")
        assert st["status"] == 0
        assert np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"])) <= 1e-9
