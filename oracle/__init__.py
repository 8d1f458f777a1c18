"""CPU oracle for the sliced big-head contraction -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check of the package entry point and the
benchmark's CPU-baseline leg may import, call, link or run anything in this
directory.  The GPU library never does, and this package never imports the
GPU library: the two share no code.  The only common dependency is the seeded
input generator `rqc`, which holds no arithmetic of the method.

Everything here is plain and slow on purpose, in complex128 / float64:

* statevector   -- Schroedinger simulation, gate by gate (the method the
                   paper contrasts with, introduction); numpy for small n and
                   a plain C/OpenMP version for up to ~28 qubits.
* unitary       -- brute-force Kronecker-product unitary for n <= 8.
* network       -- the circuit's tensor network with single-qubit gates
                   absorbed into two-qubit gates, slicing of edges, and a
                   naive pairwise contraction ("Computing bitstring
                   probabilities"; appendix A "Dynamic slicing").
* closed_form   -- amplitudes and per-slice values of product
                   (non-entangling) circuits, written as per-qubit products.
* stats         -- linear XEB (Eq. 1), Porter-Thomas checks (Eq. 2),
                   post-selection curve, marginal and conditional
                   probabilities (appendix C), GPU efficiency (Eq. 3).
* mlp           -- float64 reference MLP (forward, backward, Adam) for the
                   learned step-time model's gradient check.

Parity status per function is listed in each module's header.
"""
