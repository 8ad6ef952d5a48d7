"""GPU tests of the learned surrogate (include/surrogate.h, paper_1705_03141_amd/surrogate.py).

* each operator (convolution forward, data gradient, weight and bias gradient) against the
  FP64 reference on BF16-representable inputs;
* the whole network's weight gradients against the FP64 reference, element by element;
* the surrogate at its configured size in a regime-map sweep: trained on the lattice's own
  coarse-grained trajectories of sweep cases, it fast-forwards held-out cases where its
  ensemble's predicted interface error allows and is scored against the FP32 lattice.
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


ELEM_BAR = 24.0  # in units of the BF16 unit roundoff, relative to max|g| of the layer


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
    # Element by element: every weight-gradient element within ELEM_BAR of the layer's
    # largest reference element.  The GPU stores each activation and each activation gradient
    # in BF16 (unit roundoff u = 2^-8, about 20 roundings between the input and the first
    # layer's gradient); the reference does not round.
    u = 2.0 ** -8
    for name, _, _ in S.LAYERS:
        a = net.gw[name].cpu().numpy().ravel()
        r = g[name][0].ravel()
        elem = float(np.abs(a - r).max() / np.abs(r).max())
        nerr = float(np.linalg.norm(a - r) / np.linalg.norm(r))
        ab = net.gb[name].cpu().numpy()
        rb = g[name][1]
        belem = float(np.abs(ab - rb).max() / np.abs(rb).max())
        log(f"  {name}: max element error {elem:.3e} = {elem / u:.2f} u of max|g|; bias {belem / u:.2f} u; "
            f"norm error {nerr:.3e}")
        assert elem < ELEM_BAR * u and belem < ELEM_BAR * u and nerr < 0.08, name


def test_surrogate_fast_forwards_sweep_cases():
    """The surrogate at its configured size in use.  Sixteen jet cases drawn as in the
    regime-map sweep (the smallest width, 96^2 x 384, D 8-16) run 2000 steps in FP16 storage;
    their 4x-coarsened (phi, u/u_in) every 200 steps, padded to 64 x 64 x 256 x 4, train a
    3-member ensemble on 12 cases.  The 4 held-out cases are fast-forwarded from step 800:
    a horizon is taken by the ensemble while the members' interface spread (the predicted
    interface error, no lattice answer needed) stays within one coarse cell, else the case
    falls back to the lattice.  Accepted predictions are scored against plain FP32 lattice
    runs of the same cases."""
    import torch

    horizon, snaps, start, ahead = 200, 10, 4, 5
    cases = W.regime_sweep(ncases=16, seed=31, sizes=(96,), diameters=(8, 16))
    held = cases[12:]
    t0 = time.perf_counter()
    states, t_lbm16, unstable = S.coarse_trajectories(cases, horizon, snaps, storage="f16")
    truth, _, _ = S.coarse_trajectories(held, horizon, snaps, storage="f32")
    log(f"[surrogate] trajectories {tuple(states.shape)} and FP32 truth in {time.perf_counter() - t0:.1f} s; "
        f"unstable {unstable}")
    assert not unstable
    ens = S.Ensemble(batch=4, members=3, seed=0)
    losses = ens.train(states, cases=list(range(12)), steps=800)
    log(f"[surrogate] member losses (first 20, last 20 steps): {losses}")
    assert all(last < 0.5 * first for first, last in losses)
    # one-horizon skill on the held-out cases against persistence, both against FP32
    ext = [S.coarse_extent(pb) for pb in held]
    skill, persist = [], []
    for k, (d, h, w) in enumerate(ext):
        for s in range(start, snaps):
            pred = torch.stack(ens.predict(states[s, 12 + k:13 + k])).mean(0)
            skill.append(float((pred[0, :d, :h, :w] - truth[s + 1, k, :d, :h, :w]).abs().mean()))
            persist.append(float((states[s, 12 + k, :d, :h, :w] - truth[s + 1, k, :d, :h, :w]).abs().mean()))
    log(f"[surrogate] held-out one-horizon mean |error|: ensemble {np.mean(skill):.4e}, persistence {np.mean(persist):.4e}")
    assert np.mean(skill) < np.mean(persist)
    rep = S.fast_forward(ens, states[:, 12:], truth, list(range(4)), ext, start=start, horizons=ahead)
    taken = sum(r["taken"] for r in rep.values())
    acc = [a for r in rep.values() for a in r["actual"]]
    rej = [r["rejected"] for r in rep.values() if r["rejected"]]
    # wall time: one horizon of one case on the lattice (its share of the batched FP16 steps)
    # against one ensemble prediction
    cells = np.array([pb.ncells for pb in cases], dtype=float)
    t_case = t_lbm16 / snaps * cells[12:] / cells.sum()
    x = states[start, 12:13]
    ens.predict(x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        ens.predict(x)
    torch.cuda.synchronize()
    t_pred = (time.perf_counter() - t1) / 5
    saved = sum(r["taken"] * (t_case[k] - t_pred) for k, r in rep.items())
    log(f"[surrogate] fast-forward: {taken}/{4 * ahead} horizons by the surrogate; actual interface error of "
        f"accepted predictions {np.round(acc, 3).tolist()} coarse cells (mean {np.mean(acc) if acc else 0:.3f}); "
        f"rejected {rej}; per horizon: lattice {np.round(t_case * 1e3, 2).tolist()} ms per case, ensemble "
        f"{t_pred * 1e3:.2f} ms; lattice time saved {saved * 1e3:.1f} ms")
    assert taken >= 1
    assert np.mean(acc) <= 1.0
    assert t_pred < t_case.min()
    # the fallback engages where the predicted error exceeds the limit: with a limit of 0.02
    # coarse cells, cases go back to the lattice, and every horizon the surrogate still took
    # had a predicted error within it
    strict = S.fast_forward(ens, states[:, 12:], truth, list(range(4)), ext, start=start, horizons=ahead, limit=0.02)
    rejected = [r["rejected"] for r in strict.values() if r["rejected"]]
    log(f"[surrogate] limit 0.02: {sum(r['taken'] for r in strict.values())} horizons taken, rejections {rejected}")
    assert rejected and all(r["predicted"] > 0.02 for r in rejected)
    assert all(p <= 0.02 for r in strict.values() for p in r["predicted"])
