"""Float64 reference MLP for the learned step-time model (oracle).

Not a passage of the paper: the paper's cost is the FLOP count of each
pairwise step, 2^(nA + nB + nAB) (appendix A, Fig. 3).  The learned model
maps step-shape features to log step time with a 3-layer perceptron
d_in -> H -> H -> 1, ReLU activations, mean squared error, Adam.

Plain numpy in float64: forward, analytic backward, Adam update.  Pinned by
central finite differences of the loss (parity of the analytic gradient) and
by a closed form on a one-layer special case.
"""

import numpy as np


def init_params(d_in, hidden=128, seed=0):
    rng = np.random.default_rng(seed)
    def lin(i, o):
        w = rng.normal(scale=np.sqrt(2.0 / i), size=(i, o))
        b = np.zeros(o)
        return w, b
    w1, b1 = lin(d_in, hidden)
    w2, b2 = lin(hidden, hidden)
    w3, b3 = lin(hidden, 1)
    return {"w1": w1, "b1": b1, "w2": w2, "b2": b2, "w3": w3, "b3": b3}


def forward(params, x):
    z1 = x @ params["w1"] + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ params["w2"] + params["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ params["w3"] + params["b3"])[:, 0]
    return y, (x, z1, h1, z2, h2)


def loss(params, x, t):
    y, _ = forward(params, x)
    return float(np.mean((y - t) ** 2))


def backward(params, x, t):
    """Gradient of mean((y - t)^2) with respect to every parameter."""
    y, (x, z1, h1, z2, h2) = forward(params, x)
    b = x.shape[0]
    dy = 2.0 * (y - t) / b                      # (B,)
    g = {}
    g["w3"] = h2.T @ dy[:, None]
    g["b3"] = np.array([dy.sum()])
    dh2 = dy[:, None] @ params["w3"].T
    dz2 = dh2 * (z2 > 0)
    g["w2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ params["w2"].T
    dz1 = dh1 * (z1 > 0)
    g["w1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015) with bias correction; updates in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1 - beta1) * grads[k]
        v[...] = beta2 * v + (1 - beta2) * grads[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)
    return params


def finite_difference(params, x, t, key, idx, h=1e-6):
    p = {k: v.copy() for k, v in params.items()}
    p[key][idx] += h
    lp = loss(p, x, t)
    p[key][idx] -= 2 * h
    lm = loss(p, x, t)
    return (lp - lm) / (2 * h)
