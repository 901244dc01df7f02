"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This package holds only input generation: gate matrices of the circuit family,
the lattice circuit generator, output bitstrings and random complex tensors.
It contains none of the contraction method's arithmetic, and imports neither
the oracle nor the GPU library.
"""
from .circuits import (  # noqa: F401
    Gate, Circuit, gate_matrix, lattice_circuit, sqrt_x, sqrt_y, sqrt_w, fsim,
    random_fixed_bits, random_bitstrings, output_spec,
)
from .tensors import complex_normal, complex_normal_c64  # noqa: F401
