"""CPU oracle for the inexact-policy-iteration hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 reference
written from the paper's problem statement (finite-state, finite-action,
infinite-horizon discounted-cost MDP, solved by policy iteration; the paper's
"Problem Setting and Solution Methods" section).  Only the tests, the smoke
check and the bench's CPU-baseline leg may import it.  The GPU library never
calls it and shares no code with it.

Parity pins: every function here is pinned by CPU tests against closed forms,
brute force, textbook invariants or a library routine in a special case (see
tests/test_oracle_pins.py).  Iteration counts and intermediate iterates of the
inexact method are parity unpinned (they depend on rounding and on the inner
tolerance).
"""
from .mdp_oracle import (  # noqa: F401
    to_csr,
    q_values,
    q_values_states,
    bellman,
    bellman_streamed,
    policy_system,
    evaluate_policy,
    policy_iteration,
    brute_force,
    evaluate_policy_fixed_point,
    macqueen_bounds,
    value_iteration,
    modified_policy_iteration,
    fp16_with_row_correction,
    policy_parity,
)
