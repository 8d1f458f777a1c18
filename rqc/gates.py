"""Gate matrices of the random-circuit family.

The paper names the single-qubit set {sqrt(X), sqrt(Y), sqrt(W)} and the
two-qubit fSim(theta, phi) gate without writing the matrices (section
"Simulation of the Sycamore circuits").  The readings used here:

* sqrt(P) = (I - i P) / sqrt(2) for P in {X, Y, W}, W = (X + Y) / sqrt(2).
  These square to -i P (a global phase away from P); probabilities do not
  depend on the phase, and both sides of every comparison use exactly these
  matrices.
* fSim(theta, phi) in the basis |q0 q1> (q0 the more significant bit):
  [[1, 0, 0, 0], [0, cos t, -i sin t, 0], [0, -i sin t, cos t, 0],
   [0, 0, 0, exp(-i phi)]].

All matrices are complex128, row index = output basis state, column index =
input basis state.
"""

import numpy as np

_I = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_W = (_X + _Y) / np.sqrt(2.0)


def _sqrt_pauli(p):
    return (_I - 1j * p) / np.sqrt(2.0)


def sqrt_x():
    return _sqrt_pauli(_X)


def sqrt_y():
    return _sqrt_pauli(_Y)


def sqrt_w():
    return _sqrt_pauli(_W)


def pauli(name):
    return {"I": _I, "X": _X, "Y": _Y, "W": _W}[name].copy()


SINGLE_QUBIT_GATES = ("sqrt_x", "sqrt_y", "sqrt_w")

_SQ = {"sqrt_x": sqrt_x, "sqrt_y": sqrt_y, "sqrt_w": sqrt_w}


def single_qubit(name):
    return _SQ[name]()


def fsim(theta, phi):
    c, s = np.cos(theta), np.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1.0
    m[1, 1] = c
    m[1, 2] = -1j * s
    m[2, 1] = -1j * s
    m[2, 2] = c
    m[3, 3] = np.exp(-1j * phi)
    return m


def random_su2(rng):
    """A Haar-like random 2x2 unitary drawn from a seeded numpy Generator.

    Used only to build product (non-entangling) two-qubit gates for the
    closed-form test circuits."""
    z = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return (q * (d / np.abs(d))).astype(np.complex128)
