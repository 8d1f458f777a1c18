"""Seeded synthetic inputs for the sliced big-head contraction.

This package generates the *inputs* of the method and nothing else:
grid layouts and coupler patterns, the gate matrices of a random circuit,
the choice of open/fixed qubits with their fixed bits, and seeded samples of
slice ids.  It holds none of the method's arithmetic (no tensor network, no
contraction, no statistics), so both the oracle and the GPU library's tests
and benchmark may read from it without sharing any computation.

The circuit family follows the description of the Sycamore random circuits
(section "Simulation of the Sycamore circuits"): m cycles, each a layer of
single-qubit gates drawn from {sqrt(X), sqrt(Y), sqrt(W)} followed by fSim
gates on one of four coupler patterns, alternated in the sequence ABCDCDAB.
"""

from .gates import sqrt_x, sqrt_y, sqrt_w, fsim, SINGLE_QUBIT_GATES
from .layouts import Layout, rect_layout, diag54_layout, near_square_layout
from .generate import (Circuit, Gate, random_circuit, product_circuit,
                       choose_open_qubits, fixed_bits, sample_slice_ids,
                       workload)

__all__ = [
    "sqrt_x", "sqrt_y", "sqrt_w", "fsim", "SINGLE_QUBIT_GATES",
    "Layout", "rect_layout", "diag54_layout", "near_square_layout",
    "Circuit", "Gate", "random_circuit", "product_circuit",
    "choose_open_qubits", "fixed_bits", "sample_slice_ids", "workload",
]
