"""Brute-force circuit unitary (oracle, n <= 8).

U is the ordered product of full 2^n x 2^n gate matrices, each built from
Kronecker products with identities (a two-qubit gate on non-adjacent qubits is
conjugated by the permutation that brings its qubits together).  The state is
psi = U e_0.  This shares nothing with the in-place update of `statevector`
and pins it on tiny circuits.
"""

import numpy as np


def _perm_matrix(n, order):
    """Permutation P with (P psi)[i] = psi[j], where the bits of i in qubit
    order `order` equal the bits of j in natural order."""
    dim = 1 << n
    p = np.zeros((dim, dim), dtype=np.complex128)
    for j in range(dim):
        bits = [(j >> (n - 1 - q)) & 1 for q in range(n)]
        i = 0
        for pos, q in enumerate(order):
            i |= bits[q] << (n - 1 - pos)
        p[i, j] = 1.0
    return p


def full_gate(n, qubits, m):
    if len(qubits) == 1:
        q = qubits[0]
        return np.kron(np.kron(np.eye(1 << q), m), np.eye(1 << (n - 1 - q)))
    q0, q1 = qubits
    rest = [q for q in range(n) if q not in (q0, q1)]
    order = [q0, q1] + rest                  # bring q0, q1 to the front
    p = _perm_matrix(n, order)
    big = np.kron(m, np.eye(1 << (n - 2)))
    return p.conj().T @ big @ p


def circuit_unitary(circuit):
    n = circuit.n_qubits
    if n > 8:
        raise ValueError("brute force is for n <= 8")
    u = np.eye(1 << n, dtype=np.complex128)
    for g in circuit.gates:
        u = full_gate(n, g.qubits, g.matrix) @ u
    return u


def state(circuit):
    return circuit_unitary(circuit)[:, 0].copy()
