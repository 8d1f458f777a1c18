"""The learned step-time model's kernels (forward, backward, Adam) against
the float64 oracle MLP on the CPU."""

import sys

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _to_dict(flat, d_in, h):
    flat = np.asarray(flat, dtype=np.float64)
    o = 0
    out = {}
    for name, shape in (("w1", (d_in, h)), ("b1", (h,)), ("w2", (h, h)), ("b2", (h,)), ("w3", (h, 1)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape).copy()
        o += n
    assert o == flat.size
    return out


def _from_dict(d):
    return np.concatenate([d[k].ravel() for k in ("w1", "b1", "w2", "b2", "w3", "b3")])


def _data(batch, d_in, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(batch, d_in)).astype(np.float32)
    t = rng.normal(size=batch).astype(np.float32)
    return x, t


@pytest.mark.parametrize("batch", [1, 37, 256])
def test_mlp_forward_and_gradient_match_oracle(batch):
    import torch
    from paper_2103_03074_amd import tn
    d_in, h = tn.STEP_FEATURES, 128
    m = tn.Mlp(d_in, h, seed=3)
    x, t = _data(batch, d_in, batch)
    dx, dt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    _say("mlp forward/gradient, batch", batch)
    y = torch.empty(batch, dtype=torch.float32, device="cuda")
    m.forward(dx, y)
    g, loss = m.gradient(dx, dt)
    p = _to_dict(m.get_params(), d_in, h)
    y_ref, _ = omlp.forward(p, x.astype(np.float64))
    np.testing.assert_allclose(y.cpu().numpy(), y_ref, rtol=1e-4, atol=1e-5)
    assert loss == pytest.approx(omlp.loss(p, x.astype(np.float64), t.astype(np.float64)), rel=1e-4)
    g_ref = _from_dict(omlp.backward(p, x.astype(np.float64), t.astype(np.float64)))
    scale = np.abs(g_ref).max()
    np.testing.assert_allclose(g, g_ref, rtol=0, atol=2e-4 * scale)


def test_mlp_adam_step_matches_oracle():
    import torch
    from paper_2103_03074_amd import tn
    d_in, h = tn.STEP_FEATURES, 32
    m = tn.Mlp(d_in, h, seed=5)
    x, t = _data(64, d_in, 9)
    dx, dt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    p = _to_dict(m.get_params(), d_in, h)
    state = {}
    _say("mlp adam, two steps")
    for _ in range(2):
        g = omlp.backward(p, x.astype(np.float64), t.astype(np.float64))
        omlp.adam_step(p, g, state, lr=1e-3)
        m.train_step(dx, dt, 1e-3)
    np.testing.assert_allclose(m.get_params(), _from_dict(p), rtol=0, atol=2e-5)


def test_mlp_training_reduces_loss():
    import torch
    from paper_2103_03074_amd import tn
    d_in = tn.STEP_FEATURES
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, size=(512, d_in)).astype(np.float32)
    t = (2.0 * x[:, 0] - x[:, 3] + 0.5 * x[:, 7] ** 2).astype(np.float32)
    dx, dt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    m = tn.Mlp(d_in, 64, seed=2)
    _say("mlp training")
    first = m.train_step(dx, dt, 3e-3)
    for _ in range(300):
        last = m.train_step(dx, dt, 3e-3)
    assert last < 0.05 * first
