"""Seeded synthetic inputs for the ACSE residual path.

This package holds input generation only (integrals, occupations, orbital
rotations and 2-RDM blocks of the synthetic workloads); it contains none of the
residual, reconstruction or update arithmetic.  Both the GPU tests/bench and
the oracle take their inputs from here.
"""
from .generators import (hamiltonian, fermi_occupations, haar_orthogonal, named,
                         rdm_blocks, problem, batched_problems, CONFIGS)

__all__ = ["hamiltonian", "fermi_occupations", "haar_orthogonal", "rdm_blocks",
           "problem", "batched_problems", "CONFIGS", "named"]
