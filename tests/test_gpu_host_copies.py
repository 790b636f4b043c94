"""Host memory of every kind at the boundary: the same MDP handed over as
pageable numpy arrays, as page-locked host arrays and as device arrays must
give the same handle, and results copied out to pageable and page-locked
arrays must agree bit for bit.  Pageable memory goes through the library's
pinned blocks in pieces, so the arrays here span several blocks and end in a
ragged piece."""
import numpy as np
import pytest

from workloads import MDPInstance, config2

pytestmark = pytest.mark.gpu


def _pinned(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory().numpy()


def test_pageable_pinned_and_device_inputs_build_the_same_mdp():
    import torch
    import paper_2502_14474_amd as m
    # 9.6M entries: 38 MB of columns and 77 MB of values, not block multiples
    inst = config2(S=300_001, A=4, n_band=6, n_jump=2, seed=11)
    print(f"[case] host copies: S={inst.S} nnz={inst.nnz}", flush=True)
    pinned = MDPInstance(inst.S, inst.A, _pinned(inst.row_ptr), _pinned(inst.col), _pinned(inst.val),
                         _pinned(inst.cost), inst.gamma)
    dev = [torch.from_numpy(a).to("cuda:0") for a in (inst.row_ptr, inst.col, inst.val, inst.cost)]
    torch.cuda.synchronize()
    outs = []
    for kind in ("pageable", "pinned", "device"):
        if kind == "pageable":
            h = m.mdp_create(inst.S, inst.A, inst.row_ptr, inst.col, inst.val, inst.cost, inst.gamma)
        elif kind == "pinned":
            h = m.mdp_create(inst.S, inst.A, pinned.row_ptr, pinned.col, pinned.val, pinned.cost, inst.gamma)
        else:
            h = m.mdp_create(inst.S, inst.A, *dev, inst.gamma)
        try:
            rng = np.random.default_rng(3)
            v = rng.standard_normal(inst.S)
            res = []
            for out_kind in ("pageable", "pinned"):
                Tv = np.empty(inst.S) if out_kind == "pageable" else _pinned(np.empty(inst.S))
                pi = np.empty(inst.S, np.int32) if out_kind == "pageable" else _pinned(np.empty(inst.S, np.int32))
                r = m.mdp_bellman(h, v if out_kind == "pageable" else _pinned(v), Tv, pi)
                res.append((Tv.copy(), pi.copy(), r))
            assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
            assert res[0][2] == res[1][2]
            outs.append(res[0])
        finally:
            m.mdp_destroy(h)
    for Tv, pi, r in outs[1:]:
        assert np.array_equal(Tv, outs[0][0]) and np.array_equal(pi, outs[0][1]) and r == outs[0][2]
    # and the sweep is the definition: Tv(s) = min_a g(s,a) + gamma * P(s,a,:) v
    q = inst.cost + inst.gamma * np.add.reduceat(inst.val * v[inst.col], inst.row_ptr[:-1])
    q = q.reshape(inst.S, inst.A)
    assert np.max(np.abs(outs[0][0] - q.min(axis=1))) <= 1e-12 * np.max(np.abs(q))
