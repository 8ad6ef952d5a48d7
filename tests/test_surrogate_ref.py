"""Pins of the FP64 surrogate reference (CPU): the convolution against a brute-force sum,
its gradients and the whole network's gradients against central finite differences, and
the pooling / upsampling pairs as adjoints."""
import numpy as np

from oracle import surrogate_ref as R


def _rng(k):
    return np.random.default_rng(k)


def test_conv3d_brute_force():
    rng = _rng(1)
    x = rng.normal(size=(2, 3, 4, 5, 8))
    w = rng.normal(size=(27, 32, 8))
    b = rng.normal(size=32)
    out = R.conv3d(x, w, b)
    n, z, y, xx, co = 1, 0, 3, 2, 7  # a voxel on the boundary (z = 0, y = h - 1)
    s = b[co]
    for t, (dz, dy, dx) in enumerate(R.TAPS):
        zz, yy, xq = z + dz, y + dy, xx + dx
        if 0 <= zz < 3 and 0 <= yy < 4 and 0 <= xq < 5:
            s += sum(x[n, zz, yy, xq, ci] * w[t, co, ci] for ci in range(8))
    assert abs(out[n, z, y, xx, co] - s) < 1e-12


def test_conv3d_gradients_finite_differences():
    rng = _rng(2)
    x = rng.normal(size=(1, 2, 3, 4, 8))
    w = rng.normal(size=(27, 32, 8)) * 0.1
    dout = rng.normal(size=(1, 2, 3, 4, 32))
    f = lambda xx, ww: float((R.conv3d(xx, ww) * dout).sum())
    dx = R.conv3d_dgrad(dout, w)
    dw, db = R.conv3d_wgrad(x, dout)
    h = 1e-6
    for idx in [(0, 0, 0, 0, 0), (0, 1, 2, 3, 7), (0, 1, 1, 2, 4)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (f(x + e, w) - f(x - e, w)) / (2 * h)
        assert abs(fd - dx[idx]) < 1e-6 * max(1.0, abs(fd))
    for idx in [(0, 0, 0), (13, 31, 7), (26, 5, 2)]:
        e = np.zeros_like(w)
        e[idx] = h
        fd = (f(x, w + e) - f(x, w - e)) / (2 * h)
        assert abs(fd - dw[idx]) < 1e-6 * max(1.0, abs(fd))
    assert np.allclose(db, dout.reshape(-1, 32).sum(axis=0))


def test_pool_and_up_are_adjoint_to_their_gradients():
    rng = _rng(3)
    x = rng.normal(size=(2, 4, 6, 8, 3))
    y = rng.normal(size=(2, 2, 3, 4, 3))
    assert abs((R.pool(x) * y).sum() - (x * R.pool_bwd(y)).sum()) < 1e-10
    assert abs((R.up(y) * x).sum() - (y * R.up_bwd(x)).sum()) < 1e-10


def test_network_gradient_finite_differences():
    rng = _rng(4)
    p = R.init_params(seed=5)
    x = rng.normal(size=(1, 4, 4, 8, 8))
    x[..., 4:] = 0.0
    target = rng.normal(size=(1, 4, 4, 8, R.USED))

    def loss(pp):
        y, _ = R.forward(pp, x)
        return R.mse(y, target)[0]

    y, c = R.forward(p, x)
    _, dy = R.mse(y, target)
    g = R.backward(p, c, dy)
    h = 1e-6
    for name, idx in [("e1a", (4, 3, 1)), ("e2", (13, 40, 17)), ("bt", (0, 2, 63)), ("out", (26, 1, 30)),
                      ("d1", (9, 0, 0))]:
        w, b = p[name]
        e = np.zeros_like(w)
        e[idx] = h
        pp = dict(p)
        pp[name] = (w + e, b)
        lp = loss(pp)
        pp[name] = (w - e, b)
        lm = loss(pp)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[name][0][idx]) < 1e-5 * max(1e-3, abs(fd)) + 1e-10, (name, fd, g[name][0][idx])
    # a bias
    w, b = p["d2"]
    e = np.zeros_like(b)
    e[3] = h
    pp = dict(p)
    pp["d2"] = (w, b + e)
    lp = loss(pp)
    pp["d2"] = (w, b - e)
    lm = loss(pp)
    assert abs((lp - lm) / (2 * h) - g["d2"][1][3]) < 1e-8
