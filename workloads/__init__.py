"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds *inputs* only: system parameters, control coefficients,
initial and target density matrices.  It contains none of the method's
arithmetic (no Hamiltonian or Lindbladian, no B-splines, no time stepping,
no objective), so that the CPU oracle and the HIP path never share code that
computes a result.
"""
from .systems import (  # noqa: F401
    System,
    Problem,
    CONFIG_SEED_BASE,
    make_config,
    random_system,
    random_alpha,
    random_pure_states,
    basis_density_matrices,
    essential_embedding,
    cnot_essential,
    truncate_steps,
    with_random_states,
    observable_nm,
    ensemble_state,
    gate_initial_states,
    gate_weights,
    n_alpha,
)
