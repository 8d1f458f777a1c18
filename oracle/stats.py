"""Probability statistics of the amplitude tensor (oracle, float64).

* Linear XEB, Eq. (1): F = 2^n / L * sum_i P(s_i) - 1 over the L computed
  bitstrings (section "Fidelity").  With s1 fixed and all L = 2^n2 values of
  s2 weighted equally this is F_unif = 2^n1 * sum P - 1.
* F_self = 2^n * sum P^2 / sum P - 1: the XEB of bitstrings drawn from P
  itself; about 1 when the probabilities follow Porter-Thomas, Eq. (2).
* Post-selection curve: probabilities sorted in decreasing order, the XEB of
  the top k (section "Fidelity", right panel of Fig. 2).
* Marginal P(s1) = sum_s2 P(s1; s2) and conditional P(s2 | s1) = P / P(s1)
  (appendix C): P(s1) = (F_unif + 1) 2^-n1, and the conditional
  distribution's own XEB is exactly 0.
* Sampling from P(s2 | s1) (appendix C; the conclusion notes the method can
  sample from it) by inverse transform: a uniform u picks the smallest s2
  whose cumulative probability exceeds u times the total.
* Porter-Thomas checks: Kolmogorov-Smirnov distance of N p against Exp(1)
  and the second moment E[(N p)^2] = 2.
* GPU efficiency, Eq. (3): E = 8 * (complex multiply-adds) / (peak * time).
"""

import numpy as np


def probabilities(amps):
    a = np.asarray(amps, dtype=np.complex128)
    return a.real ** 2 + a.imag ** 2


def xeb(p, n_qubits):
    """Eq. (1) over all given probabilities, equal weights."""
    p = np.asarray(p, dtype=np.float64)
    return (2.0 ** n_qubits) / p.size * p.sum() - 1.0


def xeb_self(p, n_qubits):
    p = np.asarray(p, dtype=np.float64)
    return (2.0 ** n_qubits) * (p * p).sum() / p.sum() - 1.0


def topk_curve(p, n_qubits, ks):
    s = np.sort(np.asarray(p, dtype=np.float64))[::-1]
    c = np.cumsum(s)
    return np.array([(2.0 ** n_qubits) / k * c[k - 1] - 1.0 for k in ks])


def marginal(p):
    return float(np.sum(p))


def conditional(p):
    p = np.asarray(p, dtype=np.float64)
    return p / p.sum()


def conditional_samples(p, u):
    """Inverse-transform samples of the distribution p / sum(p): for each u in
    [0, 1) the smallest index j with cdf[j] > u * cdf[-1] (cdf the inclusive
    cumulative sum), clamped to the last index."""
    p = np.asarray(p, dtype=np.float64)
    cdf = np.cumsum(p)
    j = np.searchsorted(cdf, np.asarray(u, dtype=np.float64) * cdf[-1], side="right")
    return np.minimum(j, p.size - 1).astype(np.int64), cdf


def pt_ks_distance(p, n_qubits):
    """sup |F_emp(x) - (1 - e^-x)| for x = 2^n p."""
    x = np.sort(np.asarray(p, dtype=np.float64) * 2.0 ** n_qubits)
    m = x.size
    cdf = 1.0 - np.exp(-x)
    hi = np.arange(1, m + 1) / m
    lo = np.arange(0, m) / m
    return float(max(np.max(np.abs(hi - cdf)), np.max(np.abs(cdf - lo))))


def pt_second_moment(p, n_qubits):
    x = np.asarray(p, dtype=np.float64) * 2.0 ** n_qubits
    return float(np.mean(x * x))


def efficiency(complex_macs, peak_flops, seconds):
    """Eq. (3): 8 real flops per complex multiply-add."""
    return 8.0 * complex_macs / (peak_flops * seconds)


def norm_rel_error(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def max_err_over_rms(x, ref):
    """max_i |x_i - ref_i| / sqrt(mean_i |ref_i|^2): the largest single error
    measured against the typical amplitude (elementwise relative error is
    ill-posed where Porter-Thomas amplitudes come close to zero)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    return float(np.max(np.abs(x - ref)) / rms)


def full_bitstrings(s2_indices, n_qubits, open_q, fixed_q, fixed_bits):
    """Whole n-bit strings (as integers, qubit q at bit n-1-q) of open-qubit
    indices s2 (first open qubit the most significant bit of s2) with the
    closed qubits at s1."""
    n2 = len(open_q)
    base = 0
    for q, b in zip(fixed_q, fixed_bits):
        base |= int(b) << (n_qubits - 1 - int(q))
    out = []
    for s2 in s2_indices:
        v = base
        for j, q in enumerate(open_q):
            v |= ((int(s2) >> (n2 - 1 - j)) & 1) << (n_qubits - 1 - int(q))
        out.append(v)
    return out


def mix_top_with_random(p, k, n_qubits, random_strings):
    """Mixing the k most probable computed bitstrings with random ones
    (section "Discussions", footnote on relaxing the correlation of the
    samples): the top k indices of p (ties broken towards the lower index),
    returned in increasing index order, the XEB of those k alone
    F_top = 2^n / k * sum_top p - 1, and the expected XEB of the whole set of
    N = k + R bitstrings when the R random bitstrings are uniform over all
    2^n strings (their expected 2^n p is 1):
    F_mix = (2^n * sum_top p + R) / N - 1 = k / N * F_top."""
    p = np.asarray(p, dtype=np.float64)
    order = np.lexsort((np.arange(p.size), -p))     # probability descending, then index ascending
    top = np.sort(order[:k])
    s = float(np.sum(p[top]))
    r = len(random_strings)
    n_all = k + r
    f_top = (2.0 ** n_qubits) / k * s - 1.0 if k else 0.0
    f_mix = ((2.0 ** n_qubits) * s + r) / n_all - 1.0 if n_all else 0.0
    return top, s, f_top, f_mix
