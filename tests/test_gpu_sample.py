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
