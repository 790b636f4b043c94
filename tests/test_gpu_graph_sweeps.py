"""Bellman sweeps replayed from a captured HIP graph through the
allocation-free sweep (value iteration v <- T v, two buffers): every replay,
with eager work and synchronisations between replays, must give bitwise the
result of the same sweeps launched eagerly."""
import numpy as np
import pytest

import oracle
from workloads import config1

pytestmark = pytest.mark.gpu


def test_graph_of_noalloc_sweeps_replays_bitwise():
    import torch
    import paper_2502_14474_amd as m
    inst = config1(S=1000, A=4, k=10, seed=3)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    rp, col, val, cost = t(inst.row_ptr.astype(np.int64)), t(inst.col), t(inst.val), t(inst.cost)
    h = m.mdp_create(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, inst.cost, inst.gamma)
    lanes = m.mdp_info(h)["lanes_per_row"]
    m.mdp_destroy(h)
    n = 20  # sweeps per replay (pairs a -> b -> a)
    va = torch.zeros(inst.S, dtype=torch.float64, device=dev)
    vb = torch.zeros_like(va)
    pi = torch.zeros(inst.S, dtype=torch.int32, device=dev)
    res = torch.zeros(1, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)

    def sweeps(x, y, count, stream):
        for _ in range(count // 2):
            m.mdp_bellman_noalloc(inst.S, inst.A, inst.nnz, rp, col, val, cost, inst.gamma, x, y, pi, res,
                                  lanes_per_row=lanes, stream=stream)
            m.mdp_bellman_noalloc(inst.S, inst.A, inst.nnz, rp, col, val, cost, inst.gamma, y, x, pi, res,
                                  lanes_per_row=lanes, stream=stream)

    # eager reference: 3 x n sweeps from 0, recorded after every n
    ref = []
    ea, eb = torch.zeros_like(va), torch.zeros_like(va)
    with torch.cuda.stream(s):
        for _ in range(3):
            sweeps(ea, eb, n, s.cuda_stream)
            ref.append((ea.clone(), pi.clone(), res.clone()))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        sweeps(va, vb, n, s.cuda_stream)
    va.zero_()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        # eager work between replays
        scratch = torch.randn(4096, device=dev).sum().item()
        assert np.isfinite(scratch)
        assert torch.equal(va, ref[k][0]), k
        assert torch.equal(pi, ref[k][1]), k
        assert torch.equal(res, ref[k][2]), k
    # and the iterate is value iteration's: the oracle's 3n sweeps from 0
    v = np.zeros(inst.S)
    for _ in range(3 * n):
        v, p, r = oracle.bellman(inst, v)
    got = va.cpu().numpy()
    assert np.max(np.abs(got - v)) <= 1e-12 * max(1.0, np.max(np.abs(v)))
