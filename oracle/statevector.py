"""Schroedinger state-vector simulation in complex128 (oracle).

The full-state method the paper contrasts with (introduction, first kind of
method): store all 2^n amplitudes and apply the gates one by one.

Convention: qubit q is bit (n-1-q) of the basis index (qubit 0 is the most
significant bit), so a bitstring printed in qubit-id order reads as the
binary index.

Pins: brute-force unitary for n <= 8; unit norm; product-state closed form.
"""

import ctypes
import os

import numpy as np


def apply_gate_numpy(psi, n, qubits, m):
    """Apply one gate to the state (returns a new array).

    The state is viewed as an n-axis tensor whose axis q is qubit q; the gate
    matrix (row = output, column = input, basis |q0 q1>) is contracted with
    the gate's axes."""
    t = psi.reshape((2,) * n)
    k = len(qubits)
    g = m.reshape((2,) * (2 * k))
    out = np.tensordot(g, t, axes=(list(range(k, 2 * k)), list(qubits)))
    # tensordot puts the gate's output axes first; move them back in place
    out = np.moveaxis(out, list(range(k)), list(qubits))
    return np.ascontiguousarray(out).reshape(-1)


def simulate_numpy(circuit):
    n = circuit.n_qubits
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    for g in circuit.gates:
        psi = apply_gate_numpy(psi, n, g.qubits, g.matrix)
    return psi


# --- plain C version (oracle/csrc/statevector.c) -------------------------

_LIB = None


def _lib_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "liboracle_sv.so")


def build_c(force=False):
    """Compile the C state vector with gcc -O2 -fopenmp (fp64, no fast-math)."""
    import subprocess
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "statevector.c")
    out = _lib_path()
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               src, "-o", out, "-lm"])
    return out


def _load():
    global _LIB
    if _LIB is None:
        path = _lib_path()
        if not os.path.exists(path):
            build_c()
        lib = ctypes.CDLL(path)
        lib.oracle_sv_run.argtypes = [ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
        lib.oracle_sv_run.restype = ctypes.c_int
        lib.oracle_sv_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def simulate_c(circuit):
    """Same simulation as simulate_numpy, in plain C with OpenMP."""
    lib = _load()
    n = circuit.n_qubits
    ng = len(circuit.gates)
    qs = np.full((ng, 2), -1, dtype=np.int32)
    mats = np.zeros((ng, 32), dtype=np.float64)
    for i, g in enumerate(circuit.gates):
        qs[i, :len(g.qubits)] = g.qubits
        flat = g.matrix.ravel()
        mats[i, 0:2 * flat.size:2] = flat.real
        mats[i, 1:2 * flat.size:2] = flat.imag
    psi = np.zeros(2 << n, dtype=np.float64)
    rc = lib.oracle_sv_run(n, ng, qs.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           mats.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           psi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise RuntimeError(f"oracle_sv_run failed ({rc})")
    return psi.view(np.complex128)


def c_threads():
    return int(_load().oracle_sv_threads())


def simulate(circuit):
    return simulate_numpy(circuit) if circuit.n_qubits <= 16 else simulate_c(circuit)


def amplitudes_from_state(psi, n, open_q, fixed_q, bits):
    """A[s2] for all s2: entries of psi whose fixed qubits equal s1.

    Output index: open qubits in ascending id, the first one the most
    significant bit (the bitstring order of the paper's Table III)."""
    t = psi.reshape((2,) * n)
    idx = [slice(None)] * n
    for q, b in zip(fixed_q, bits):
        idx[q] = int(b)
    sub = t[tuple(idx)]          # remaining axes: open qubits in ascending order
    return np.ascontiguousarray(sub).reshape(-1)
