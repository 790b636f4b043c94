"""Checks of the seeded input generators (no method arithmetic involved)."""
import numpy as np
import pytest

from workloads import config1, config2, config3, config4, config5_instance, config5_requests


def _check_csr(inst, k=None):
    rows = inst.S * inst.A
    rp = inst.row_ptr
    assert rp.shape == (rows + 1,) and rp[0] == 0 and np.all(np.diff(rp) >= 1)
    assert inst.col.dtype == np.int32 and inst.val.dtype == np.float64
    assert inst.col.min() >= 0 and inst.col.max() < inst.S
    assert np.all(inst.val >= 0) and np.all(np.isfinite(inst.cost))
    sums = np.add.reduceat(inst.val, rp[:-1])
    assert np.max(np.abs(sums - 1.0)) <= 1e-12
    # sorted unique columns inside every row
    d = np.diff(inst.col.astype(np.int64))
    inner = np.ones(inst.nnz - 1, bool)
    inner[rp[1:-1] - 1] = False
    assert np.all(d[inner] > 0)
    if k is not None:
        assert np.all(np.diff(rp) == k)


def test_config1_shape_and_determinism():
    a, b = config1(), config1()
    _check_csr(a, k=10)
    assert a.S == 1000 and a.A == 4 and a.nnz == 40000 and a.gamma == 0.9
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    c = config1(seed=1)
    assert not np.array_equal(a.col, c.col)


def test_config2_band_and_jumps():
    inst = config2(S=5000, A=3, seed=2)
    _check_csr(inst, k=16)
    s_of_row = np.repeat(np.arange(inst.S), inst.A)
    cols = inst.col.reshape(-1, 16).astype(np.int64)
    off = (cols - s_of_row[:, None]) % inst.S
    off = np.where(off > inst.S // 2, off - inst.S, off)
    in_band = np.abs(off) <= 64
    assert np.all(in_band.sum(axis=1) >= 14)


def test_config2_independent_of_worker_count():
    a = config2(S=300_000, A=2, workers=1, chunk_states=65536)
    b = config2(S=300_000, A=2, workers=4, chunk_states=65536)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert np.array_equal(a.cost, b.cost)


def test_config3_maze_structure():
    inst = config3(H=40, W=30, seed=1)
    _check_csr(inst)
    S, A = inst.S, inst.A
    obst, goal = inst.meta["obstacle"], inst.meta["goal"]
    assert not obst[goal]
    absorbing = obst.copy()
    absorbing[goal] = True
    for s in np.nonzero(absorbing)[0][:50]:
        for a in range(A):
            r = s * A + a
            lo, hi = inst.row_ptr[r], inst.row_ptr[r + 1]
            assert hi - lo == 1 and inst.col[lo] == s and inst.val[lo] == 1.0
    assert np.all(np.diff(inst.row_ptr) <= 5)
    c = inst.cost.reshape(S, A)
    assert np.all(c[obst] == 10.0) and np.all(c[goal] == 0.0)
    free = ~absorbing
    assert np.all(c[free] == 1.0)
    # interior free cell, action N: 0.8 to the north neighbour
    W = 30
    s = next(s for s in range(W + 1, S - W - 1) if free[s] and 0 < s % W < W - 1)
    r = s * A + 1
    cols = inst.col[inst.row_ptr[r]:inst.row_ptr[r + 1]]
    vals = inst.val[inst.row_ptr[r]:inst.row_ptr[r + 1]]
    assert dict(zip(cols.tolist(), vals.tolist()))[s - W] == 0.8


def test_config4_twin():
    inst = config4(S=4000, A=4, seed=3)
    _check_csr(inst, k=24)
    assert inst.gamma == 0.995 and np.all(inst.cost > 0)


def test_config5_stream():
    reqs = config5_requests(200, seed=1)
    S = np.array([r["S"] for r in reqs])
    A = np.array([r["A"] for r in reqs])
    k = np.array([r["k"] for r in reqs])
    assert S.min() >= 1000 and S.max() <= 1_000_000
    assert A.min() >= 2 and A.max() <= 16 and k.min() >= 4 and k.max() <= 32
    assert set(r["gamma"] for r in reqs) <= {0.9, 0.99, 0.999}
    small = next(r for r in reqs if r["S"] < 20000)
    inst = config5_instance(small)
    _check_csr(inst, k=small["k"])
    assert inst.gamma == small["gamma"]
