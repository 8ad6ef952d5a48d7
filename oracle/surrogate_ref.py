"""FP64 numpy reference of the surrogate network's operators and of the network itself.

TEST INFRASTRUCTURE ONLY: the tests import it to check the GPU operators (include/
surrogate.h) and their gradients.  It shares no code with the GPU path.  Every operator is
written from its definition (layout [n][d][h][w][c], convolution weights [27][cout][cin] with
tap = (dz+1)*9 + (dy+1)*3 + (dx+1), zero padding 1); gradients follow from the chain rule.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shifted(x, dz, dy, dx):
    """y[v] = x[v + (dz, dy, dx)] with zeros outside."""
    n, d, h, w, c = x.shape
    p = np.zeros((n, d + 2, h + 2, w + 2, c))
    p[:, 1:-1, 1:-1, 1:-1] = x
    return p[:, 1 + dz:1 + dz + d, 1 + dy:1 + dy + h, 1 + dx:1 + dx + w]


def conv3d(x, w, b=None):
    out = np.zeros(x.shape[:4] + (w.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += _shifted(x, dz, dy, dx) @ w[t].T
    if b is not None:
        out += b
    return out


def conv3d_dgrad(dout, w):
    """d/dx of sum(dout * conv3d(x, w)): x[u] meets w[t] at output u - off(t)."""
    dx = np.zeros(dout.shape[:4] + (w.shape[2],))
    for t, (dz, dy, dxx) in enumerate(TAPS):
        dx += _shifted(dout, -dz, -dy, -dxx) @ w[t]
    return dx


def conv3d_wgrad(x, dout):
    cout, cin = dout.shape[-1], x.shape[-1]
    dw = np.zeros((27, cout, cin))
    D = dout.reshape(-1, cout)
    for t, (dz, dy, dx) in enumerate(TAPS):
        dw[t] = D.T @ _shifted(x, dz, dy, dx).reshape(-1, cin)
    return dw, D.sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def pool(x):
    n, d, h, w, c = x.shape
    return x.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def pool_bwd(dout):
    return np.repeat(np.repeat(np.repeat(dout, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up_bwd(dout):
    n, d, h, w, c = dout.shape
    return dout.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4, 6))


# ---------------------------------------------------------------- the network
# layer name -> (cin, cout); input has 8 channels (4 fields + 4 zero), output uses 4 of 32
LAYERS = [("e1a", 8, 32), ("e1b", 32, 32), ("e2", 32, 64), ("bt", 64, 64), ("d2", 64, 32), ("d1", 32, 32),
          ("out", 32, 32)]
USED = 4


def forward(params, x):
    """Returns (prediction (n, d, h, w, 32) whose first 4 channels are the fields' change,
    cache for backward)."""
    c = {"x": x}
    c["e1a"] = relu(conv3d(x, *params["e1a"]))
    c["e1"] = relu(conv3d(c["e1a"], *params["e1b"]))
    c["p1"] = pool(c["e1"])
    c["e2"] = relu(conv3d(c["p1"], *params["e2"]))
    c["p2"] = pool(c["e2"])
    c["bt"] = relu(conv3d(c["p2"], *params["bt"]))
    c["u2"] = up(c["bt"]) + c["e2"]
    c["d2"] = relu(conv3d(c["u2"], *params["d2"]))
    c["u1"] = up(c["d2"]) + c["e1"]
    c["d1"] = relu(conv3d(c["u1"], *params["d1"]))
    c["y"] = conv3d(c["d1"], *params["out"])
    return c["y"], c


def mse(y, target):
    e = y[..., :USED] - target
    loss = float((e * e).mean())
    g = np.zeros_like(y)
    g[..., :USED] = 2.0 * e / e.size
    return loss, g


def backward(params, c, dy):
    """Gradients of sum(dy * y) with respect to every weight and bias."""
    g = {}
    g["out"] = conv3d_wgrad(c["d1"], dy)
    dd1 = conv3d_dgrad(dy, params["out"][0]) * (c["d1"] > 0)
    g["d1"] = conv3d_wgrad(c["u1"], dd1)
    du1 = conv3d_dgrad(dd1, params["d1"][0])
    dd2 = up_bwd(du1) * (c["d2"] > 0)
    g["d2"] = conv3d_wgrad(c["u2"], dd2)
    du2 = conv3d_dgrad(dd2, params["d2"][0])
    dbt = up_bwd(du2) * (c["bt"] > 0)
    g["bt"] = conv3d_wgrad(c["p2"], dbt)
    dp2 = conv3d_dgrad(dbt, params["bt"][0])
    de2 = (pool_bwd(dp2) + du2) * (c["e2"] > 0)
    g["e2"] = conv3d_wgrad(c["p1"], de2)
    dp1 = conv3d_dgrad(de2, params["e2"][0])
    de1 = (pool_bwd(dp1) + du1) * (c["e1"] > 0)
    g["e1b"] = conv3d_wgrad(c["e1a"], de1)
    de1a = conv3d_dgrad(de1, params["e1b"][0]) * (c["e1a"] > 0)
    g["e1a"] = conv3d_wgrad(c["x"], de1a)
    return g


def init_params(seed: int = 0, scale: float = 1.0):
    """He-style normal initialisation, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, cin, cout in LAYERS:
        std = scale * np.sqrt(2.0 / (27 * cin))
        p[name] = (rng.normal(0.0, std, size=(27, cout, cin)), np.zeros(cout))
    return p
