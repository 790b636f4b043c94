"""GPU parity of the polynomial preconditioner (precond_degree d >= 2): GMRES
on (I - gamma P_pi) M^-1 with M^-1 = sum_{i<d} (gamma P_pi)^i, against the
oracle's exact policy evaluation and exact policy iteration.  The
preconditioner changes the Krylov space, not the solution, so the bars are
those of the unpreconditioned solver."""
import sys

import numpy as np
import pytest

import oracle
from workloads import config1, config2, config3, config4, random_dense_mdp

pytestmark = pytest.mark.gpu

INSTANCES = {
    "c1": lambda: config1(),
    "c2twin": lambda: config2(S=20000, A=8, seed=1),
    "c3twin": lambda: config3(H=64, W=80, seed=1),
    "c4twin": lambda: config4(S=12000, A=16, seed=1),
    "ragged": lambda: random_dense_mdp(37, 3, 0.95, seed=5, density=0.3),
}


def _mdp(inst, **kw):
    import paper_2502_14474_amd as m
    print(f"[case] {inst.name} S={inst.S} A={inst.A} nnz={inst.nnz} {kw}", flush=True)
    sys.stdout.flush()
    return m.MDP.from_instance(inst, **kw)


@pytest.mark.parametrize("deg", [2, 4, 8])
@pytest.mark.parametrize("name", ["c1", "c2twin", "c3twin", "c4twin"])
def test_precond_policy_eval_matches_exact_solve(name, deg):
    inst = INSTANCES[name]()
    rng = np.random.default_rng(6)
    pi = rng.integers(0, inst.A, inst.S).astype(np.int32)
    v_ref, _ = oracle.evaluate_policy(inst, pi)
    with _mdp(inst) as h:
        v, st = h.policy_eval(pi, rtol=1e-13, max_iter=20000, precond_degree=deg)
    err = np.max(np.abs(v - v_ref)) / np.max(np.abs(v_ref))
    assert st["status"] == 0, st
    assert err <= 1e-9, (err, st)
    # d products with P_pi per Arnoldi step, plus d - 1 per cycle end and one per restart
    assert st["policy_applies"] >= deg * st["inner_iters"]


def test_precond_cuts_arnoldi_steps_on_the_maze():
    inst = INSTANCES["c3twin"]()
    rng = np.random.default_rng(2)
    pi = rng.integers(0, inst.A, inst.S).astype(np.int32)
    with _mdp(inst) as h:
        _, st1 = h.policy_eval(pi, rtol=1e-8, max_iter=20000)
        _, st4 = h.policy_eval(pi, rtol=1e-8, max_iter=20000, precond_degree=4)
    # (gamma P)^4 clusters the spectrum of the Krylov operator closer to 1
    assert st4["inner_iters"] < st1["inner_iters"], (st1, st4)


def test_precond_degree_one_is_the_plain_solver_bitwise():
    inst = INSTANCES["c2twin"]()
    with _mdp(inst) as h:
        v0, p0, s0 = h.solve(alpha=1e-2)
        v1, p1, s1 = h.solve(alpha=1e-2, precond_degree=1)
        v2, p2, s2 = h.solve(alpha=1e-2, precond_degree=0)
    assert np.array_equal(v0, v1) and np.array_equal(v0, v2)
    assert np.array_equal(p0, p1) and np.array_equal(p0, p2)
    assert s0["inner_iters"] == s1["inner_iters"] == s2["inner_iters"]


def _solve_parity(inst, rel_tol, **kw):
    ref = oracle.policy_iteration(inst, method="auto" if inst.S <= 2500 else "certified")
    vstar = ref["v"]
    with _mdp(inst) as h:
        v, pi, st = h.solve(**kw)
    assert st["status"] == 0, st
    err = np.max(np.abs(v - vstar)) / np.max(np.abs(vstar))
    assert err <= rel_tol, (err, st)
    Q = oracle.q_values(inst, vstar)
    delta = np.max(np.abs(v - vstar))
    tau = max(1e-9, 2 * inst.gamma * (delta + 1e-11 * np.max(np.abs(vstar))))
    pp = oracle.policy_parity(inst, Q, pi, ref["pi"], tau)
    assert pp["mismatch_outside_band"] == 0 and pp["not_tau_optimal"] == 0, pp
    return v, pi, st


@pytest.mark.parametrize("deg", [2, 4])
@pytest.mark.parametrize("name", ["c1", "c2twin", "c4twin", "ragged"])
def test_precond_solve_fp64(name, deg):
    _solve_parity(INSTANCES[name](), 1e-9, rtol_cert=1e-10, precond_degree=deg)


@pytest.mark.parametrize("precision", [1, 2])
@pytest.mark.parametrize("name", ["c4twin", "c3twin", "ragged"])
def test_precond_solve_mixed(name, precision):
    _solve_parity(INSTANCES[name](), 1e-8, precision=precision, rtol_cert=1e-9, precond_degree=4)


def test_precond_solve_maze_closed_forms():
    inst = config3(H=48, W=48, seed=4)
    ref = oracle.policy_iteration(inst, method="sparse")
    with _mdp(inst) as h:
        v, pi, st = h.solve(rtol_cert=1e-10, precond_degree=4)
    assert st["status"] == 0, st
    assert np.max(np.abs(v - ref["v"])) / np.max(np.abs(ref["v"])) <= 1e-9
    obst = inst.meta["obstacle"]
    assert np.allclose(v[obst], 10 / (1 - inst.gamma), rtol=1e-9)
    assert abs(v[inst.meta["goal"]]) <= 1e-9 * np.max(np.abs(v))


def test_precond_gmres_exact_in_few_steps_small_system():
    # with m >= S, GMRES on the preconditioned operator still ends with the
    # exact solution within S steps
    inst = random_dense_mdp(12, 2, 0.9, seed=9, density=0.5)
    pi = np.zeros(inst.S, np.int32)
    Ppi, gpi = oracle.policy_system(inst, pi)
    v_ref = np.linalg.solve(np.eye(inst.S) - inst.gamma * Ppi.toarray(), gpi)
    with _mdp(inst) as h:
        v, st = h.policy_eval(pi, restart=16, rtol=1e-14, max_iter=16, precond_degree=3)
    assert st["inner_iters"] <= inst.S
    assert np.max(np.abs(v - v_ref)) <= 1e-12 * np.max(np.abs(v_ref))


def test_precond_option_rules():
    import paper_2502_14474_amd as m
    inst = INSTANCES["c1"]()
    pi = np.zeros(inst.S, np.int32)
    with _mdp(inst) as h:
        for inner in (1, 2, 3):
            with pytest.raises(m.MDPError) as e:
                h.policy_eval(pi, inner=inner, precond_degree=2)
            assert e.value.status == m.native.MDP_E_NOTSUP
        with pytest.raises(m.MDPError) as e:
            h.solve(inner=2, precond_degree=2)
        assert e.value.status == m.native.MDP_E_NOTSUP
        for bad in (-1, 17):
            with pytest.raises(m.MDPError) as e:
                h.solve(precond_degree=bad)
            assert e.value.status == m.native.MDP_E_INVAL
        v = np.empty(inst.S)
        p = np.empty(inst.S, np.int32)
        with pytest.raises(m.MDPError) as e:
            m.mdp_solve_batch([h.h], [v], [p], precond_degree=2)
        assert e.value.status == m.native.MDP_E_NOTSUP
