"""GPU tests of the learned surrogate (include/surrogate.h, paper_1705_03141_amd/surrogate.py).

* each operator (convolution forward, data gradient, weight and bias gradient) against the
  FP64 reference on BF16-representable inputs;
* the whole network's weight gradients against the FP64 reference;
* training on coarse-grained jet trajectories made by the lattice itself: the loss falls,
  the trained network predicts held-out cases better than persistence and than the
  untrained network, and the lattice as judge keeps it where its interface error is at
  most one coarse cell.
"""
import sys
import time

import numpy as np
import pytest

from oracle import surrogate_ref as R
from paper_1705_03141_amd import lbm
from paper_1705_03141_amd import surrogate as S
from paper_1705_03141_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bf16_round(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def to_dev_bf16(x):
    import torch
    u = np.ascontiguousarray(bf16_round(x).astype(np.float32)).view(np.uint32) >> 16
    return torch.from_numpy(u.astype(np.uint16).view(np.int16)).to("cuda")


def from_dev_bf16(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("cin,cout", [(8, 32), (32, 64), (64, 32)])
def test_conv_operators_against_reference(cin, cout):
    import torch
    rng = np.random.default_rng(cin + cout)
    n, d, h, w = 2, 4, 6, 10
    x = bf16_round(rng.normal(size=(n, d, h, w, cin)))
    wt = bf16_round(rng.normal(size=(27, cout, cin)) * 0.1)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    dout = bf16_round(rng.normal(size=(n, d, h, w, cout)))
    L = S._lib()
    xd, wd, doutd = to_dev_bf16(x), to_dev_bf16(wt), to_dev_bf16(dout)
    bd = torch.from_numpy(b.astype(np.float32)).to("cuda")
    y32 = torch.empty((n, d, h, w, cout), dtype=torch.float32, device="cuda")
    assert L.surr_conv3d_fwd(S._p(xd), S._p(wd), S._p(bd), None, S._p(y32), n, d, h, w, cin, cout, 0, None) == 0
    e_fwd = rel(y32.cpu().numpy(), R.conv3d(x, wt, b))
    # weight and bias gradients (FP32 out)
    gw = torch.empty((27, cout, cin), dtype=torch.float32, device="cuda")
    gb = torch.empty(cout, dtype=torch.float32, device="cuda")
    scratch = torch.empty(L.surr_conv3d_wgrad_scratch_bytes(n, d, h, w, cin, cout) // 4 + 1, dtype=torch.float32,
                          device="cuda")
    assert L.surr_conv3d_wgrad(S._p(xd), S._p(doutd), S._p(gw), S._p(gb), S._p(scratch), n, d, h, w, cin, cout,
                               None) == 0
    rw, rb = R.conv3d_wgrad(x, dout)
    e_wg, e_bg = rel(gw.cpu().numpy(), rw), rel(gb.cpu().numpy(), rb)
    msg = f"[conv {cin}->{cout}] fwd {e_fwd:.2e} wgrad {e_wg:.2e} bgrad {e_bg:.2e}"
    # data gradient (cin multiple of 32 only)
    if cin % 32 == 0:
        w_t = torch.empty((27, cin, cout), dtype=torch.int16, device="cuda")
        assert L.surr_conv3d_flip_weights(S._p(wd), S._p(w_t), cin, cout, None) == 0
        din = torch.empty((n, d, h, w, cin), dtype=torch.int16, device="cuda")
        assert L.surr_conv3d_dgrad(S._p(doutd), S._p(w_t), None, S._p(din), n, d, h, w, cin, cout, None) == 0
        ref_dg = R.conv3d_dgrad(dout, wt)
        e_dg = rel(from_dev_bf16(din), ref_dg)
        # with a ReLU output as mask: zero exactly where it is not positive
        assert L.surr_conv3d_dgrad(S._p(doutd), S._p(w_t), S._p(xd), S._p(din), n, d, h, w, cin, cout, None) == 0
        got_m = from_dev_bf16(din)
        e_dgm = rel(got_m, np.where(x > 0, ref_dg, 0.0))
        msg += f" dgrad {e_dg:.2e} masked {e_dgm:.2e}"
        assert e_dg < 1e-2 and e_dgm < 1e-2 and not got_m[x <= 0].any()
    log(msg)
    assert e_fwd < 1e-5 and e_wg < 1e-5 and e_bg < 1e-5


@pytest.mark.parametrize("cin,cout,d", [(8, 32, 48), (16, 32, 48), (32, 64, 48), (64, 64, 8)])
def test_forward_many_tiles_against_reference(cin, cout, d):
    """Forward convolution where blocks walk several tiles (16 and 32 channels: ranges of 4
    z-planes through the ring of input planes), h is odd (the last tile's second row is
    outside the volume) and w = 70 is ragged against the tile width."""
    import torch
    rng = np.random.default_rng(cin * cout)
    n, h, w = 1, 41, 70
    x = bf16_round(rng.normal(size=(n, d, h, w, cin)))
    wt = bf16_round(rng.normal(size=(27, cout, cin)) * 0.1)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    L = S._lib()
    xd, wd = to_dev_bf16(x), to_dev_bf16(wt)
    bd = torch.from_numpy(b.astype(np.float32)).to("cuda")
    y32 = torch.empty((n, d, h, w, cout), dtype=torch.float32, device="cuda")
    assert L.surr_conv3d_fwd(S._p(xd), S._p(wd), S._p(bd), None, S._p(y32), n, d, h, w, cin, cout, 0, None) == 0
    ref = R.conv3d(x, wt, b)
    e_fwd = rel(y32.cpu().numpy(), ref)
    yb = torch.empty((n, d, h, w, cout), dtype=torch.int16, device="cuda")
    assert L.surr_conv3d_fwd(S._p(xd), S._p(wd), S._p(bd), S._p(yb), None, n, d, h, w, cin, cout, 1, None) == 0
    e_relu = rel(from_dev_bf16(yb), bf16_round(np.maximum(ref, 0.0)))
    log(f"[conv {n}x{d}x{h}x{w} {cin}->{cout}] fwd {e_fwd:.2e} relu/bf16 {e_relu:.2e}")
    assert e_fwd < 1e-5 and e_relu < 1e-2


def test_forward_full_size_sampled():
    """The 32 -> 32 convolution at the surrogate's full resolution (1 x 256 x 64 x 64; each
    block sweeps 16 z-planes) on 300 sampled output voxels, each summed over its 27 taps
    directly in FP64 from the same BF16 operands."""
    import torch
    rng = np.random.default_rng(3)
    n, d, h, w, cin, cout = 1, 256, 64, 64, 32, 32
    L = S._lib()
    x = bf16_round(rng.normal(size=(n, d, h, w, cin)).astype(np.float32))
    wt = bf16_round(rng.normal(size=(27, cout, cin)) * 0.1)
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    xd, wd = to_dev_bf16(x), to_dev_bf16(wt)
    bd = torch.from_numpy(b.astype(np.float32)).to("cuda")
    y32 = torch.empty((n, d, h, w, cout), dtype=torch.float32, device="cuda")
    assert L.surr_conv3d_fwd(S._p(xd), S._p(wd), S._p(bd), None, S._p(y32), n, d, h, w, cin, cout, 0, None) == 0
    y = y32.cpu().numpy()
    idx = np.stack([rng.integers(0, s, 300) for s in (d, h, w)], axis=1)
    idx[:4] = [[0, 0, 0], [d - 1, h - 1, w - 1], [15, 63, 0], [16, 0, 63]]  # faces and z-range ends
    worst = 0.0
    for z, yy, xx in idx:
        ref = b.copy()
        for tap in range(27):
            dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
            zs, ys, xs = z + dz, yy + dy, xx + dx
            if 0 <= zs < d and 0 <= ys < h and 0 <= xs < w:
                ref += wt[tap] @ x[0, zs, ys, xs]
        worst = max(worst, float(np.abs(y[0, z, yy, xx] - ref).max() / max(np.abs(ref).max(), 1e-30)))
    log(f"[conv full size 1x256x64x64 32->32] sampled worst relative error {worst:.2e}")
    assert worst < 1e-5


def test_weight_gradient_long_ranges_against_reference():
    """Weight and bias gradients where each block walks several row segments (the ring of
    source rows carries over between consecutive y), the rows are ragged against the 64-voxel
    segment (w = 70), the input channels fill a partial tile (cin = 40) and cout spans two
    tiles."""
    import torch
    rng = np.random.default_rng(5)
    n, d, h, w, cin, cout = 1, 4, 200, 70, 40, 64
    x = bf16_round(rng.normal(size=(n, d, h, w, cin)))
    dout = bf16_round(rng.normal(size=(n, d, h, w, cout)))
    L = S._lib()
    xd, doutd = to_dev_bf16(x), to_dev_bf16(dout)
    gw = torch.empty((27, cout, cin), dtype=torch.float32, device="cuda")
    gb = torch.empty(cout, dtype=torch.float32, device="cuda")
    scratch = torch.empty(L.surr_conv3d_wgrad_scratch_bytes(n, d, h, w, cin, cout) // 4 + 1, dtype=torch.float32,
                          device="cuda")
    assert L.surr_conv3d_wgrad(S._p(xd), S._p(doutd), S._p(gw), S._p(gb), S._p(scratch), n, d, h, w, cin, cout,
                               None) == 0
    rw, rb = R.conv3d_wgrad(x, dout)
    e_wg, e_bg = rel(gw.cpu().numpy(), rw), rel(gb.cpu().numpy(), rb)
    log(f"[wgrad {n}x{d}x{h}x{w} {cin}->{cout}] wgrad {e_wg:.2e} bgrad {e_bg:.2e}")
    assert e_wg < 1e-5 and e_bg < 1e-5


def test_elementwise_operators_against_reference():
    """Pooling, upsampling, ReLU gradient, addition, input packing and the squared error
    against the FP64 reference: each output is the reference value rounded once to BF16 (the
    sums of BF16 inputs are exact in FP32 here, up to 8 terms of equal exponent range)."""
    import torch
    rng = np.random.default_rng(11)
    L = S._lib()
    n, d, h, w, c = 2, 4, 6, 10, 40
    fine = bf16_round(rng.normal(size=(n, d, h, w, c)))
    coarse = bf16_round(rng.normal(size=(n, d // 2, h // 2, w // 2, c)))
    fd, cd = to_dev_bf16(fine), to_dev_bf16(coarse)
    out_c = torch.empty_like(cd)
    assert L.surr_pool_fwd(S._p(fd), S._p(out_c), n, d, h, w, c, None) == 0
    assert rel(from_dev_bf16(out_c), bf16_round(R.pool(fine))) < 4e-3
    out_f = torch.empty_like(fd)
    assert L.surr_pool_bwd(S._p(cd), S._p(out_f), n, d, h, w, c, None) == 0
    assert np.array_equal(from_dev_bf16(out_f), bf16_round(R.pool_bwd(coarse)))
    assert L.surr_up_add_fwd(S._p(cd), S._p(fd), S._p(out_f), n, d // 2, h // 2, w // 2, c, None) == 0
    assert rel(from_dev_bf16(out_f), bf16_round(R.up(coarse) + fine)) < 4e-3
    assert L.surr_up_bwd(S._p(fd), None, S._p(out_c), n, d // 2, h // 2, w // 2, c, None) == 0
    assert rel(from_dev_bf16(out_c), bf16_round(R.up_bwd(fine))) < 4e-3
    assert L.surr_up_bwd(S._p(fd), S._p(cd), S._p(out_c), n, d // 2, h // 2, w // 2, c, None) == 0
    got = from_dev_bf16(out_c)
    assert rel(got, bf16_round(np.where(coarse > 0, R.up_bwd(fine), 0.0))) < 4e-3 and not got[coarse <= 0].any()
    assert L.surr_pool_fwd(S._p(fd), S._p(out_c), n, d, h, w, 12, None) == -1  # channels not a multiple of 8
    # flat operators: a ragged count, then a pointer off the 16-byte grid (scalar path)
    count = fine.size - 5
    y, g = fine.ravel(), coarse.ravel()
    gd = to_dev_bf16(np.resize(g, fine.size))
    dx = torch.zeros_like(fd)
    assert L.surr_relu_bwd(S._p(fd), S._p(gd), S._p(dx), count, None) == 0
    want = np.where(y > 0, np.resize(g, fine.size), 0.0)
    got = from_dev_bf16(dx).ravel()
    assert np.array_equal(got[:count], want[:count]) and not got[count:].any()
    flat_a, flat_b = fd.view(-1), gd.view(-1)
    o = torch.zeros_like(flat_a)
    assert L.surr_add(S._p(flat_a[1:]), S._p(flat_b[1:]), None, S._p(o[1:]), count, None) == 0
    ref = bf16_round(y[1:count + 1] + np.resize(g, fine.size)[1:count + 1])
    got = from_dev_bf16(o)
    assert rel(got[1:count + 1], ref) < 4e-3 and got[0] == 0 and not got[count + 1:].any()
    # with a mask, on the vector path (aligned, ragged count) and on the scalar path
    mask = np.resize(g, fine.size)
    for off in (0, 1):
        o.zero_()
        assert L.surr_add(S._p(flat_a[off:]), S._p(flat_b[off:]), S._p(flat_b[off:]), S._p(o[off:]), count, None) == 0
        got = from_dev_bf16(o)[off:off + count]
        want = np.where(mask[off:off + count] > 0, y[off:off + count] + mask[off:off + count], 0.0)
        assert rel(got, bf16_round(want)) < 4e-3 and not got[mask[off:off + count] <= 0].any()
    # input packing and the squared error
    nv = n * d * h * w
    x4 = rng.normal(size=(nv, 4)).astype(np.float32)
    packed = torch.empty((nv, 8), dtype=torch.int16, device="cuda")
    assert L.surr_pack_input(S._p(torch.from_numpy(x4).cuda()), S._p(packed), nv, 4, 8, None) == 0
    pk = from_dev_bf16(packed)
    assert np.array_equal(pk[:, :4], bf16_round(x4)) and not pk[:, 4:].any()
    pred = rng.normal(size=(nv, 32)).astype(np.float32)
    tgt = rng.normal(size=(nv, 4)).astype(np.float32)
    dp = torch.empty((nv, 32), dtype=torch.int16, device="cuda")
    part = torch.empty((nv + 255) // 256, dtype=torch.float32, device="cuda")
    assert L.surr_mse(S._p(torch.from_numpy(pred).cuda()), S._p(torch.from_numpy(tgt).cuda()), S._p(dp), S._p(part),
                      nv, 32, 4, None) == 0
    loss_ref, g_ref = R.mse(pred.astype(np.float64), tgt.astype(np.float64))
    loss = float(part.cpu().numpy().astype(np.float64).sum()) / (nv * 4)
    assert abs(loss - loss_ref) / loss_ref < 1e-4
    assert rel(from_dev_bf16(dp), g_ref) < 4e-3 and not from_dev_bf16(dp)[:, 4:].any()
    log(f"[element-wise] pool/up/relu/add/pack/mse match; loss {loss:.6e} ref {loss_ref:.6e}")


def test_network_gradients_against_reference():
    rng = np.random.default_rng(7)
    n, d, h, w = 2, 8, 8, 16
    params = R.init_params(seed=3)
    params = {k: (bf16_round(v[0]), bf16_round(v[1])) for k, v in params.items()}
    x = np.zeros((n, d, h, w, 8))
    x[..., :4] = bf16_round(rng.normal(size=(n, d, h, w, 4)))
    target = rng.normal(size=(n, d, h, w, 4)).astype(np.float32).astype(np.float64)
    net = S.Network(n, d, h, w)
    net.set_params(params)
    net.set_input(x[..., :4])
    net.forward()
    import torch
    loss_gpu, dy = net.loss_and_grad(torch.from_numpy(target.astype(np.float32)).to("cuda"))
    net.backward(dy)
    y, cache = R.forward(params, x)
    loss_ref, dyr = R.mse(y, target)
    g = R.backward(params, cache, dyr)
    log(f"[network] loss gpu {loss_gpu:.6e} ref {loss_ref:.6e}")
    assert abs(loss_gpu - loss_ref) / loss_ref < 2e-2
    for name, _, _ in S.LAYERS:
        a = net.gw[name].cpu().numpy().ravel()
        r = g[name][0].ravel()
        cos = float(a @ r / (np.linalg.norm(a) * np.linalg.norm(r)))
        nerr = float(np.linalg.norm(a - r) / np.linalg.norm(r))
        log(f"  {name}: cosine {cos:.5f} relative norm error {nerr:.3e}")
        assert cos > 0.995 and nerr < 0.08, name


def test_training_on_lattice_trajectories_beats_persistence():
    horizon, snaps = 200, 8
    train = W.regime_sweep(ncases=6, seed=21, sizes=(32,), diameters=(6, 8), fields=True)
    held = W.regime_sweep(ncases=2, seed=99, sizes=(32,), diameters=(6, 8), fields=True)
    t0 = time.perf_counter()
    tr = S.trajectories(train, horizon, snaps)          # (snaps+1, 6, 32, 8, 8, 4)
    te = S.trajectories(held, horizon, snaps)
    t_lbm = time.perf_counter() - t0
    log(f"[surrogate] trajectories: train {tr.shape}, held-out {te.shape}, {t_lbm:.1f} s")
    net = S.Network(tr.shape[1], *tr.shape[2:5], seed=0, lr=2e-3)
    net_te = S.Network(te.shape[1], *te.shape[2:5], seed=0)

    def held_error(params):
        net_te.set_params(params)
        errs = [np.abs(net_te.predict(te[k]) - te[k + 1]).mean() for k in range(snaps)]
        return float(np.mean(errs))

    err_untrained = held_error(net.get_params())
    persistence = float(np.mean([np.abs(te[k] - te[k + 1]).mean() for k in range(snaps)]))
    rng = np.random.default_rng(0)
    losses = []
    for it in range(400):
        k = int(rng.integers(0, snaps))
        losses.append(net.train_step(tr[k], tr[k + 1] - tr[k]))
    err_trained = held_error(net.get_params())
    log(f"[surrogate] loss {np.mean(losses[:20]):.3e} -> {np.mean(losses[-20:]):.3e}; held-out mean |error|: "
        f"persistence {persistence:.4e}, untrained {err_untrained:.4e}, trained {err_trained:.4e}")
    # judge: the lattice checks one window per held-out case
    use, ierr = S.judge(net_te, te[4], te[5])
    t1 = time.perf_counter()
    for _ in range(10):
        net_te.predict(te[4])
    t_net = (time.perf_counter() - t1) / 10
    # the gain: the same horizon on the lattice (both held-out cases in one batch)
    bat = lbm.Batch(held)
    bat.step(1)
    bat.sync()
    t2 = time.perf_counter()
    bat.step(horizon)
    bat.sync()
    t_lbm_h = time.perf_counter() - t2
    bat.close()
    log(f"[surrogate] judge: interface error per held-out case {np.round(ierr, 3).tolist()} coarse cells, "
        f"surrogate kept {use.tolist()}; one prediction {t_net * 1e3:.2f} ms for {horizon} steps of 2 cases "
        f"(host arrays in and out), the lattice {t_lbm_h * 1e3:.2f} ms: {t_lbm_h / t_net:.0f}x")
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:20])
    assert err_trained < persistence and err_trained < err_untrained
    assert use.all()
    assert t_net < t_lbm_h / 5
