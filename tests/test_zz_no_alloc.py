"""The allocation-free sampling entry point (tn_sample_noalloc, workspace in
a file-scope device array) against tn_sample with a caller-owned workspace:
the same kernels, so the drawn indices must be identical, on two calls in a
row, the second with a smaller input."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _draws(torch, tn, amps, n_open, u, noalloc):
    out = torch.empty(u.numel(), dtype=torch.int64, device="cuda")
    if noalloc:
        tn.sample_noalloc(amps, n_open, u, out)
    else:
        ws = torch.empty(tn.sample_workspace_bytes(n_open), dtype=torch.uint8, device="cuda")
        tn.sample(amps, n_open, u, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_sampling_matches_workspace_sampling():
    import torch
    from paper_2103_03074_amd import tn
    assert torch.cuda.is_available()
    g = torch.Generator(device="cpu").manual_seed(11)
    for n_open, n_samples in ((20, 1 << 16), (12, 1000)):
        _say("noalloc sampling, n_open", n_open, "samples", n_samples)
        a = torch.randn(2 << n_open, generator=g, dtype=torch.float64)
        a[: 2 * 37] = 0.0                    # zero-probability entries are never drawn
        amps = a.cuda()
        u = torch.rand(n_samples, generator=g, dtype=torch.float64).cuda()
        ref = _draws(torch, tn, amps, n_open, u, noalloc=False)
        got = _draws(torch, tn, amps, n_open, u, noalloc=True)
        np.testing.assert_array_equal(got, ref)
        assert got.min() >= 37 and got.max() < (1 << n_open)


def test_noalloc_sampling_rejects_sizes_beyond_its_array():
    import torch
    from paper_2103_03074_amd import tn
    amps = torch.zeros(2, dtype=torch.float64, device="cuda")
    u = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(tn.TnError):
        tn.sample_noalloc(amps, 21, u, out)     # rejected on the host before any launch
