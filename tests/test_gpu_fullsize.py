"""Parity at the full workload sizes, in the launch configuration the bench
times: sampled outputs recomputed one by one by the oracle, and properties
that hold at any size (MacQueen's bounds computed by the oracle's Bellman
operator, closed-form values of absorbing maze cells)."""
import sys
import time

import numpy as np
import pytest

import oracle
from workloads import config2, config3, config4

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c2():
    t = time.time()
    inst = config2()
    _log(f"[case] config2 full S={inst.S} nnz={inst.nnz} generated in {time.time() - t:.1f}s")
    return inst


def _sampled_bellman_check(inst, Tv, pi, v, rng, n=2000):
    states = np.sort(rng.choice(inst.S, size=n, replace=False))
    Q = oracle.q_values_states(inst, v, states)
    k = np.diff(inst.row_ptr).reshape(inst.S, inst.A)[states].max(axis=1)
    g = np.abs(inst.cost).reshape(inst.S, inst.A)[states].max(axis=1)
    bnd = 2.0 * (k + 2.0) * EPS * (g + inst.gamma * np.max(np.abs(v)))
    ref = Q.min(axis=1)
    assert np.all(np.abs(Tv[states] - ref) <= bnd)
    part = np.partition(Q, 1, axis=1)
    clear = (part[:, 1] - part[:, 0]) > 2 * bnd
    assert np.array_equal(pi[states][clear], Q.argmin(axis=1)[clear])
    return states


def test_config2_full_bellman_sampled(c2):
    import paper_2502_14474_amd as m
    rng = np.random.default_rng(11)
    v = 10.0 * rng.standard_normal(c2.S)
    with m.MDP.from_instance(c2, validate=False) as h:
        Tv, pi, res = h.bellman(v)
    _sampled_bellman_check(c2, Tv, pi, v, rng)
    assert res >= np.max(np.abs(Tv - v)) * (1 - 1e-15)


def test_config2_full_solve_certified(c2):
    """The bench's solve, then a certificate from the oracle's own Bellman
    sweep at full size: ||v - v*|| <= ||T v - v|| / (1 - gamma)."""
    import paper_2502_14474_amd as m
    with m.MDP.from_instance(c2, validate=False) as h:
        v, pi, st = h.solve(alpha=1e-2, rtol_cert=1e-10)
    assert st["status"] == 0, st
    P = oracle.to_csr(c2)
    Tv, pi_ref, res = oracle.bellman(c2, v, P)
    bound = res / (1.0 - c2.gamma)
    rel = bound / np.max(np.abs(Tv))
    _log(f"[cert] oracle residual {res:.3e}, certified relative error <= {rel:.3e}")
    assert rel <= 1e-9
    lo, hi = oracle.macqueen_bounds(c2, v, P)
    assert np.all(lo <= v + bound) and np.all(v <= hi + bound)
    Q = oracle.q_values(c2, v, P)
    part = np.partition(Q, 1, axis=1)
    gap = part[:, 1] - part[:, 0]
    tau = max(1e-9, 2 * c2.gamma * 2 * bound)
    assert np.all(pi[gap > tau] == pi_ref[gap > tau])
    assert np.all(Q[np.arange(c2.S), pi] - Q.min(axis=1) <= tau)


def test_config2_full_mixed_fp32(c2):
    import paper_2502_14474_amd as m
    with m.MDP.from_instance(c2, validate=False, low_precision=m.MDP_BUILD_FP32) as h:
        v, pi, st = h.solve(alpha=1e-2, precision=m.MDP_MIXED_FP32, rtol_cert=1e-9)
    assert st["status"] == 0, st
    Tv, pi_ref, res = oracle.bellman(c2, v)
    rel = res / (1.0 - c2.gamma) / np.max(np.abs(Tv))
    _log(f"[cert] mixed fp32: oracle residual {res:.3e}, certified relative error <= {rel:.3e}")
    assert rel <= 1e-8


def test_config3_full_maze():
    import paper_2502_14474_amd as m
    t = time.time()
    inst = config3()
    _log(f"[case] config3 full S={inst.S} nnz={inst.nnz} generated in {time.time() - t:.1f}s")
    with m.MDP.from_instance(inst, validate=False) as h:
        v, pi, st = h.solve(alpha=1e-2, rtol_cert=1e-10, max_inner=20000)
    assert st["status"] == 0, st
    _log(f"[case] config3 solve: {st['time_ms']:.1f} ms, sweeps {st['bellman_sweeps']}, inner {st['inner_iters']}")
    obst, goal = inst.meta["obstacle"], inst.meta["goal"]
    assert np.max(np.abs(v[obst] - 10.0 / (1.0 - inst.gamma))) <= 1e-9 * 1e4
    assert abs(v[goal]) <= 1e-9 * 1e4
    Tv, pi_ref, res = oracle.bellman(inst, v)
    rel = res / (1.0 - inst.gamma) / np.max(np.abs(Tv))
    _log(f"[cert] config3: oracle residual {res:.3e}, certified relative error <= {rel:.3e}")
    assert rel <= 1e-9
    rng = np.random.default_rng(5)
    _sampled_bellman_check(inst, Tv, pi, v, rng)


@pytest.mark.parametrize("inner,deg", [(2, 1), (0, 4)])  # BiCGSTAB; GMRES with the d = 4 polynomial
def test_config3_full_maze_other_inner_solvers(inner, deg):
    """The maze's products on the contiguous copy in one launch each (the
    Krylov product and the preconditioner's Horner steps): BiCGSTAB, and GMRES
    preconditioned, certified by the oracle's sweep at full size."""
    import paper_2502_14474_amd as m
    inst = config3()
    _log(f"[case] config3 full, inner={inner} precond_degree={deg}")
    with m.MDP.from_instance(inst, validate=False) as h:
        v, pi, st = h.solve(alpha=1e-2, rtol_cert=1e-10, max_inner=20000, inner=inner, precond_degree=deg)
    assert st["status"] == 0, st
    _log(f"[case] config3 solve: {st['time_ms']:.1f} ms, sweeps {st['bellman_sweeps']}, inner {st['inner_iters']}")
    Tv, pi_ref, res = oracle.bellman(inst, v)
    rel = res / (1.0 - inst.gamma) / np.max(np.abs(Tv))
    _log(f"[cert] config3 inner={inner}: certified relative error <= {rel:.3e}")
    assert rel <= 1e-9


@pytest.fixture(scope="module")
def c4():
    t = time.time()
    inst = config4()
    _log(f"[case] config4 full S={inst.S} nnz={inst.nnz} generated in {time.time() - t:.1f}s")
    return inst


def _certify(inst, v, limit, label):
    t = time.time()
    Tv, pi_ref, res = oracle.bellman_streamed(inst, v, workers=8)
    _log(f"[cert] {label}: oracle sweep in {time.time() - t:.1f}s")
    rel = res / (1.0 - inst.gamma) / np.max(np.abs(Tv))
    _log(f"[cert] {label}: oracle residual {res:.3e}, certified relative error <= {rel:.3e}")
    assert rel <= limit
    return Tv


def test_config4_full_solve_fp64_and_sampled_sweep(c4):
    """1.5G nonzeros: the float64 solve certified by the oracle's own sweep at
    full size, and the GPU sweep at the solution checked state by state on a
    sample."""
    import paper_2502_14474_amd as m
    inst = c4
    with m.MDP.from_instance(inst, validate=False) as h:
        v, pi, st = h.solve(alpha=1e-2, rtol_cert=1e-10)
        assert st["status"] == 0, st
        Tv_gpu, pi_gpu, _ = h.bellman(v)
    _certify(inst, v, 1e-9, "config4 fp64")
    _sampled_bellman_check(inst, Tv_gpu, pi_gpu, v, np.random.default_rng(7))


def test_config4_full_bicgstab_on_the_sliced_copy(c4):
    """BiCGSTAB's products y = x - gamma P_pi x on the XCD-sliced copy at full
    size, certified by the oracle's streamed sweep."""
    import paper_2502_14474_amd as m
    with m.MDP.from_instance(c4, validate=False) as h:
        v, pi, st = h.solve(alpha=1e-2, rtol_cert=1e-10, inner=2)
    assert st["status"] == 0, st
    _certify(c4, v, 1e-9, "config4 bicgstab")


def test_config4_full_mixed_fp16(c4):
    """The float16 copy with its per-row sum correction, float32 inner solves
    and float64 refinement reach the mixed-precision target at full size."""
    import paper_2502_14474_amd as m
    inst = c4
    with m.MDP.from_instance(inst, validate=False, low_precision=m.MDP_BUILD_FP16) as h:
        v, pi, st = h.solve(alpha=1e-2, precision=m.MDP_MIXED_FP16, rtol_cert=1e-9)
    assert st["status"] == 0, st
    _certify(inst, v, 1e-8, "config4 mixed fp16")


def test_config4_full_mixed_fp32_packed_copy(c4):
    """The packed float32 copy holds 2*nnz = 3.07e9 words here, past the
    int32 range: its build and its row loads form word indices in 64 bits.
    The mixed solve reaches the target and its sweep at the solution agrees
    with the float64 handle's."""
    import paper_2502_14474_amd as m
    inst = c4
    assert 2 * inst.nnz > 2 ** 31
    print("[case] config 4 mixed fp32 with the packed copy", flush=True)
    with m.MDP.from_instance(inst, validate=False, low_precision=m.MDP_BUILD_FP32) as h:
        v, pi, st = h.solve(alpha=1e-2, precision=m.MDP_MIXED_FP32, rtol_cert=1e-9)
    assert st["status"] == 0, st
    _certify(inst, v, 1e-8, "config4 mixed fp32")
