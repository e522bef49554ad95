"""Seeded synthetic inputs for the Schur refinement.

This package only draws and assembles test matrices and starting bases. It
holds none of the refinement's arithmetic, and both the GPU library's tests
and the CPU oracle read their inputs from it.
"""
from .generator import (  # noqa: F401
    cn,
    haar_unitary,
    gapped_eigenvalues,
    schur_test_matrix,
    lp_schur_start,
    hp_schur_start,
    hadamard_exact,
    perturbed_start,
    wilkinson_companion_dd,
    example3_matrix,
    batched_sizes,
    batched_inputs,
    real_schur_test_matrix,
    real_blocks_of,
    lp_real_schur_start,
    continuation_step_dd,
    continuation_perturbation,
    to_dd,
    round_mantissa,
)
