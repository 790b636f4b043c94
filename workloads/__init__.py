"""Seeded synthetic MDP instances shared by the CPU oracle, the tests and the bench.

This package only draws random numbers and lays them out as CSR arrays.  It holds
none of the solution method's arithmetic (no Bellman operator, no policy
evaluation), so both sides of a parity check can take their inputs from it.
"""
from .generators import (  # noqa: F401
    MDPInstance,
    SEED_BASE,
    config1,
    config2,
    config3,
    config4,
    config5_requests,
    config5_instance,
    random_dense_mdp,
    deterministic_chain,
)
