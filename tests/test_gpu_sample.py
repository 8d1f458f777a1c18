"""Sampling from P(s2 | s1) on the device (tn_sample) against the oracle's
inverse transform.  Cumulative sums are taken in different orders on the two
sides, so a uniform that falls within rounding of an interval boundary may
pick either neighbour: every draw must be a valid inverse-transform draw
under the oracle's cumulative sums (to 1e-12 of the total), and almost all
must equal the oracle's."""

import sys

import numpy as np
import pytest

import rqc
from oracle import statevector as sv
from oracle import stats

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _draw(amps_np, n_open, u_np):
    import torch
    from paper_2103_03074_amd import tn
    assert torch.cuda.is_available()
    a = torch.from_numpy(np.ascontiguousarray(amps_np, dtype=np.complex128).view(np.float64)).cuda()
    u = torch.from_numpy(np.asarray(u_np, dtype=np.float64)).cuda()
    out = torch.empty(u.numel(), dtype=torch.int64, device="cuda")
    ws = torch.empty(tn.sample_workspace_bytes(n_open), dtype=torch.uint8, device="cuda")
    tn.sample(a, n_open, u, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check_valid(p, u, got):
    ref, cdf = stats.conditional_samples(p, u)
    tot = cdf[-1]
    t = u * tot
    tol = 1e-12 * tot
    above = cdf[got] > t - tol
    below = np.where(got > 0, cdf[np.maximum(got - 1, 0)] <= t + tol, True)
    assert np.all(above & below)
    assert np.all(p[got] > 0)
    return np.mean(got == ref)


def test_sample_c2_amplitudes(c2_state):
    w, psi = c2_state
    amps = sv.amplitudes_from_state(psi, 25, w["open_q"], w["fixed_q"], w["bits"])   # 2^10 amplitudes
    u = np.random.default_rng(7).random(100_000)
    _say("sample: c2 amplitudes, 1e5 draws")
    got = _draw(amps, 10, u)
    assert _check_valid(stats.probabilities(amps), u, got) > 0.999
    # bitwise repeatable
    assert np.array_equal(got, _draw(amps, 10, u))


@pytest.mark.parametrize("n_open", [11, 21])
def test_sample_multi_level_scan(n_open):
    """2^11 and 2^21 probabilities: two and three levels of block sums."""
    rng = np.random.default_rng(n_open)
    a = rng.normal(size=1 << n_open) + 1j * rng.normal(size=1 << n_open)
    a[rng.integers(0, a.size, 64)] = 0.0
    u = rng.random(50_000)
    _say("sample: synthetic", n_open, "open qubits")
    got = _draw(a, n_open, u)
    assert _check_valid(stats.probabilities(a), u, got) > 0.999


def test_sample_degenerate_cases():
    from paper_2103_03074_amd import tn
    import torch
    _say("sample: one amplitude, all-zero amplitudes, no draws")
    assert _draw(np.array([0.3 - 0.1j]), 0, [0.0, 0.5, 0.999]).tolist() == [0, 0, 0]
    assert _draw(np.zeros(16, dtype=np.complex128), 4, [0.0, 0.9]).tolist() == [15, 15]
    assert _draw(np.ones(8, dtype=np.complex128), 3, []).tolist() == []
    # a workspace that is too small is refused before any launch
    a = torch.zeros(2 * 16, dtype=torch.float64, device="cuda")
    u = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(tn.TnError) as ei:
        tn.sample(a, 4, u, out, ws)
    assert ei.value.status == -1


def test_sample_bench_shape_uniform_grid():
    """2^16 Porter-Thomas-like probabilities (the 40-qubit workload's open
    count), evenly spaced uniforms: the draw counts match the exact
    interval counts of the oracle's cumulative sums."""
    rng = np.random.default_rng(3)
    a = rng.normal(size=1 << 16) + 1j * rng.normal(size=1 << 16)
    n = 1 << 20
    u = (np.arange(n) + 0.5) / n
    _say("sample: 2^16 probabilities, 2^20 grid draws")
    got = _draw(a, 16, u)
    p = stats.probabilities(a)
    assert _check_valid(p, u, got) > 0.9999
    ref, _ = stats.conditional_samples(p, u)
    diff = np.abs(np.bincount(got, minlength=p.size) - np.bincount(ref, minlength=p.size))
    assert diff.max() <= 1 and diff.sum() <= 2 * np.count_nonzero(got != ref)


# --- mixing the most probable bitstrings with random ones -----------------

def _mix(amps_np, n_qubits, open_q, fixed_q, bits, k, words_np):
    import torch
    from paper_2103_03074_amd import tn
    n_open = len(open_q)
    a = torch.from_numpy(np.ascontiguousarray(amps_np, dtype=np.complex128).view(np.float64)).cuda()
    wd = torch.from_numpy(np.asarray(words_np, dtype=np.uint64).view(np.int64)).cuda()
    out = torch.empty(k + len(words_np), dtype=torch.int64, device="cuda")
    ws = torch.empty(tn.mix_workspace_bytes(n_open), dtype=torch.uint8, device="cuda")
    r = tn.mix_topk(a, n_qubits, open_q, fixed_q, bits, k, wd, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64), r


def _check_mix(amps, n_qubits, open_q, fixed_q, bits, k, words):
    got, r = _mix(amps, n_qubits, open_q, fixed_q, bits, k, words)
    p = stats.probabilities(amps)
    top, s, f_top, f_mix = stats.mix_top_with_random(p, k, n_qubits, words)
    ref_top = stats.full_bitstrings(top, n_qubits, open_q, fixed_q, bits)
    mask = (1 << n_qubits) - 1 if n_qubits < 64 else (1 << 64) - 1
    assert [int(x) for x in got[:k]] == ref_top                       # bit-exact selection
    assert [int(x) for x in got[k:]] == [int(w) & mask for w in words]
    assert r["P_top"] == pytest.approx(s, rel=1e-12, abs=1e-300)
    assert r["F_top"] == pytest.approx(f_top, rel=1e-10, abs=1e-10)
    assert r["F_mix_expected"] == pytest.approx(f_mix, rel=1e-10, abs=1e-10)
    return r


def test_mix_topk_c2_amplitudes(c2_state):
    """25-qubit state, 10 open qubits: the 20 most probable bitstrings mixed
    with 1000 random ones, against the oracle's selection and estimate."""
    w, psi = c2_state
    amps = sv.amplitudes_from_state(psi, 25, w["open_q"], w["fixed_q"], w["bits"])
    words = np.random.default_rng(7).integers(0, 2 ** 63, size=1000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    _say("mix top-k c2, k 20, random 1000")
    r = _check_mix(amps, 25, w["open_q"], w["fixed_q"], w["bits"], 20, words)
    _say("mix top-k c2", r)
    assert r["F_top"] > 1.0                      # the top of a Porter-Thomas sample lies far above the mean


@pytest.mark.parametrize("n_open,k", [(20, 220), (20, 0), (12, 4096), (12, 1000)])
def test_mix_topk_many_blocks_and_ties(n_open, k):
    """Multi-block selection (2^20 amplitudes), k = 0 and k = all, and many
    ties (a quarter of the amplitudes zero, one value repeated across
    blocks) with the threshold inside the tie: the lower indices win."""
    rng = np.random.default_rng(n_open * 7 + k)
    L = 1 << n_open
    a = (rng.normal(size=L) + 1j * rng.normal(size=L)) * 2.0 ** (-n_open / 2)
    a[rng.choice(L, size=L // 4, replace=False)] = 0.0
    if 0 < k < L:   # 300 copies of the k-th largest amplitude: the threshold falls inside the tie
        kth = int(np.argsort(-np.abs(a), kind="stable")[k - 1])
        a[rng.choice(L, size=300, replace=False)] = a[kth]
    n_fixed = 5
    n = n_open + n_fixed
    open_q = sorted(rng.choice(n, size=n_open, replace=False).tolist())
    fixed_q = [q for q in range(n) if q not in open_q]
    bits = rng.integers(0, 2, size=n_fixed).tolist()
    words = rng.integers(0, 2 ** 63, size=257, dtype=np.uint64)
    _say("mix top-k, n_open", n_open, "k", k)
    _check_mix(a, n, open_q, fixed_q, bits, k, words)
