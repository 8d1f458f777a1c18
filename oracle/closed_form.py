"""Closed-form amplitudes of product (non-entangling) circuits (oracle).

When every two-qubit gate is a tensor product G_a (x) G_b, the state stays a
product state, and

    A[s2] = prod_{closed q} <s1_q| M_q |0>  x  (x)_{open q} M_q |0>,

with M_q the ordered product of all single-qubit factors that act on qubit q.
Slicing edge (q, t) inserts the projector |b><b| on qubit q's wire right after
its t-th two-qubit gate (before any single-qubit gate that follows, which the
canonical network absorbs forward into the next two-qubit gate).  This gives
per-slice values A_j for networks of any size -- the check that holds at the
full 53-qubit shape, where no state vector fits.

The factors of each 4x4 product gate are recovered with a rank-1 operator
Schmidt (SVD) decomposition, so nothing about how the circuit was drawn is
assumed.
"""

import numpy as np


def factor_product_gate(m, tol=1e-10):
    """m = kron(a, b) -> (a, b).  Raises if m is not a product operator."""
    t = m.reshape(2, 2, 2, 2)                  # a_out, b_out, a_in, b_in
    r = t.transpose(0, 2, 1, 3).reshape(4, 4)  # (a_out a_in), (b_out b_in)
    u, s, vh = np.linalg.svd(r)
    if s[1] > tol * s[0]:
        raise ValueError("two-qubit gate is entangling")
    a = (u[:, 0] * s[0]).reshape(2, 2)
    b = vh[0, :].reshape(2, 2)
    return a, b


def product_amplitudes(circuit, open_q, fixed_q, bits, sliced=(), slice_id=0):
    """A_j[s2] (or A when nothing is sliced) of a product circuit."""
    n = circuit.n_qubits
    proj = {}
    for i, e in enumerate(sliced):
        proj[(int(e[0]), int(e[1]))] = (int(slice_id) >> i) & 1
    state = [np.array([1.0, 0.0], dtype=np.complex128) for _ in range(n)]
    count = [0] * n
    for g in circuit.gates:
        if len(g.qubits) == 1:
            q = g.qubits[0]
            state[q] = g.matrix @ state[q]
            continue
        a, b = factor_product_gate(g.matrix)
        for q, f in zip(g.qubits, (a, b)):
            state[q] = f @ state[q]
            key = (q, count[q])
            if key in proj:
                keep = proj[key]
                v = np.zeros(2, dtype=np.complex128)
                v[keep] = state[q][keep]
                state[q] = v
            count[q] += 1
    scalar = np.complex128(1.0)
    for q, s in zip(fixed_q, bits):
        scalar *= state[q][int(s)]
    out = np.array([scalar], dtype=np.complex128)
    for q in sorted(open_q):
        out = np.kron(out, state[q])
    return out
