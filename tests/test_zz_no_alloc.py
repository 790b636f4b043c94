"""The allocation-free sweep (mdp_bellman_noalloc) against mdp_bellman on a
handle of the same MDP: bitwise equal Tv, policy and residual with the
handle's lanes per row, on two calls in a row (the second with a smaller
MDP), plus the oracle's Q values within the per-row rounding bound.  Every
call goes through the C ABI."""
import sys

import numpy as np
import pytest

import oracle
from workloads import config2, config4, random_dense_mdp

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _device_arrays(inst, dev):
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    return t(inst.row_ptr.astype(np.int64)), t(inst.col), t(inst.val), t(inst.cost)


def _run_pair(inst, seed):
    """mdp_bellman on a handle, then mdp_bellman_noalloc on the same arrays
    and v; returns both results as host arrays."""
    import torch
    import paper_2502_14474_amd as m
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    v_h = 5.0 * rng.standard_normal(inst.S)
    v = torch.from_numpy(v_h).to(dev)
    _log(f"[case] no-alloc sweep {inst.name} S={inst.S} A={inst.A} nnz={inst.nnz}")
    h = m.mdp_create(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, inst.cost, inst.gamma)
    try:
        lanes = m.mdp_info(h)["lanes_per_row"]
        Tv_ref = torch.empty(inst.S, dtype=torch.float64, device=dev)
        pi_ref = torch.empty(inst.S, dtype=torch.int32, device=dev)
        res_ref = m.mdp_bellman(h, v, Tv_ref, pi_ref)
    finally:
        m.mdp_destroy(h)
    rp, col, val, cost = _device_arrays(inst, dev)
    Tv = torch.full((inst.S,), np.nan, dtype=torch.float64, device=dev)
    pi = torch.full((inst.S,), -1, dtype=torch.int32, device=dev)
    res = torch.full((1,), np.nan, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    m.mdp_bellman_noalloc(inst.S, inst.A, inst.nnz, rp, col, val, cost, inst.gamma, v, Tv, pi, res,
                          lanes_per_row=lanes, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    return (v_h, Tv_ref.cpu().numpy(), pi_ref.cpu().numpy(), res_ref,
            Tv.cpu().numpy(), pi.cpu().numpy(), float(res.cpu().numpy()[0]))


def _check_oracle(inst, v, Tv, pi, res):
    Q = oracle.q_values(inst, v)
    k = np.diff(inst.row_ptr).astype(np.float64)
    bnd = (2.0 * (k + 2.0) * EPS * (np.abs(inst.cost) + inst.gamma * np.max(np.abs(v)))
           ).reshape(inst.S, inst.A).max(axis=1)
    ref = Q.min(axis=1)
    assert np.all(np.abs(Tv - ref) <= bnd)
    if inst.A > 1:
        part = np.partition(Q, 1, axis=1)
        clear = (part[:, 1] - part[:, 0]) > 2 * bnd
        assert np.array_equal(pi[clear], Q.argmin(axis=1)[clear])
    assert abs(res - np.max(np.abs(ref - v))) <= np.max(bnd)


def test_noalloc_sweep_equals_handle_sweep_on_two_calls():
    first = config2(S=50000, A=8, seed=3)
    second = config4(S=3000, A=16, k=24, seed=4)  # smaller, and other A and row length
    for inst, seed in ((first, 1), (second, 2)):
        v, Tv_ref, pi_ref, res_ref, Tv, pi, res = _run_pair(inst, seed)
        assert np.array_equal(Tv, Tv_ref), inst.name
        assert np.array_equal(pi, pi_ref), inst.name
        assert res == res_ref, (res, res_ref)
        _check_oracle(inst, v, Tv, pi, res)


def test_noalloc_sweep_ragged_rows_and_optional_outputs():
    import torch
    import paper_2502_14474_amd as m
    inst = random_dense_mdp(37, 3, 0.95, seed=5, density=0.3)
    v, Tv_ref, pi_ref, res_ref, Tv, pi, res = _run_pair(inst, 7)
    assert np.array_equal(Tv, Tv_ref) and np.array_equal(pi, pi_ref) and res == res_ref
    _check_oracle(inst, v, Tv, pi, res)
    # only the policy requested: the same policy
    dev = torch.device("cuda:0")
    rp, col, val, cost = _device_arrays(inst, dev)
    pi2 = torch.full((inst.S,), -1, dtype=torch.int32, device=dev)
    h = m.mdp_create(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, inst.cost, inst.gamma)
    lanes = m.mdp_info(h)["lanes_per_row"]
    m.mdp_destroy(h)
    m.mdp_bellman_noalloc(inst.S, inst.A, inst.nnz, rp, col, val, cost, inst.gamma,
                          torch.from_numpy(v).to(dev), None, pi2, None, lanes_per_row=lanes)
    torch.cuda.synchronize()
    assert np.array_equal(pi2.cpu().numpy(), pi_ref)


def test_noalloc_sweep_rejects_host_memory_and_oversized_mdps():
    import torch
    import paper_2502_14474_amd as m
    from paper_2502_14474_amd import native
    inst = config2(S=2000, A=4, seed=9)
    dev = torch.device("cuda:0")
    rp, col, val, cost = _device_arrays(inst, dev)
    v_host = np.zeros(inst.S)
    with pytest.raises(m.MDPError) as e:
        m.mdp_bellman_noalloc(inst.S, inst.A, inst.nnz, rp, col, val, cost, inst.gamma, v_host)
    assert e.value.status == native.MDP_E_INVAL
    # more sweep tiles than the scratch holds: refused before any array is read
    lib = native.load()
    st = lib.mdp_bellman_noalloc(70000 * 1024, 1, 70000 * 1024, None, None, None, None, 0.9, None, None,
                                 None, None, 0, None)
    assert st == native.MDP_E_NOTSUP, lib.mdp_last_error()
    assert b"65536" in lib.mdp_last_error()
