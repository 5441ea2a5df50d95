"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only draws numbers: one- and two-electron integrals, UCCSD
amplitudes, random Pauli rotations and sums, request arrival traces, and
the order in which the UCCSD excitations are applied.  It holds
none of the method's arithmetic (no Jordan-Wigner transform, no state vector,
no expectation value), so that the oracle and the GPU path can both consume
the same inputs while sharing no code that computes a result.
"""
from .integrals import synthetic_integrals
from .params import uniform_amplitudes
from .random_paulis import random_rotations, random_pauli_sum
from .arrivals import poisson_requests
from .ansatz import uccsd_excitation_order

__all__ = [
    "synthetic_integrals",
    "uniform_amplitudes",
    "random_rotations",
    "random_pauli_sum",
    "poisson_requests",
    "uccsd_excitation_order",
]
