"""Learned surrogate of the lattice Boltzmann method (argument marshalling for include/
surrogate.h; every operator runs in the HIP library).

A 3-level 3-D convolutional encoder-decoder with 32 base channels maps the coarse-grained
state of a jet, (phi, u / u_in) averaged over 4^3 blocks, to the change of that state over
`horizon` steps of the method.  Weights and activations are BF16 on the matrix cores with
FP32 accumulation and FP32 master weights (Adam).  torch provides device memory only.

Architecture (channels-last, additive skips):
  e1a = relu(conv 8->32)  e1 = relu(conv 32->32)          full resolution R
  e2  = relu(conv 32->64 (pool e1))                        R/2
  bt  = relu(conv 64->64 (pool e2))                        R/4
  d2  = relu(conv 64->32 (up bt + e2))                     R/2
  d1  = relu(conv 32->32 (up d2 + e1))                     R
  y   = conv 32->32, channels 0..3 = change of (phi, ux, uy, uz)
The input's channels 4..7 are zero (the convolution needs multiples of 8).

Use in a regime-map sweep (`fast_forward`): an ensemble of independently initialised and
trained networks advances each case by one horizon; the spread of the members' interface
positions is the predicted interface error, known without running the lattice.  Where it
exceeds one coarse cell the case falls back to the lattice.  The method stays the judge of
what the surrogate delivers: its predictions are scored against the plain FP32 lattice.
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, Optional, Tuple

import numpy as np

from . import lbm as _lbm

LAYERS = [("e1a", 8, 32), ("e1b", 32, 32), ("e2", 32, 64), ("bt", 64, 64), ("d2", 64, 32), ("d1", 32, 32),
          ("out", 32, 32)]
FIELDS = 4
IN_CH = 8
_bound = False


def _lib():
    global _bound
    L = _lbm.library()
    if not _bound:
        vp, i, ll, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_float
        L.surr_conv3d_fwd.argtypes = [vp, vp, vp, vp, vp, i, i, i, i, i, i, i, vp]
        L.surr_conv3d_flip_weights.argtypes = [vp, vp, i, i, vp]
        L.surr_conv3d_dgrad.argtypes = [vp, vp, vp, vp, i, i, i, i, i, i, vp]
        L.surr_conv3d_wgrad_scratch_bytes.argtypes = [i, i, i, i, i, i]
        L.surr_conv3d_wgrad_scratch_bytes.restype = ctypes.c_size_t
        L.surr_conv3d_wgrad.argtypes = [vp, vp, vp, vp, vp, i, i, i, i, i, i, vp]
        L.surr_relu_bwd.argtypes = [vp, vp, vp, ll, vp]
        L.surr_pool_fwd.argtypes = [vp, vp, i, i, i, i, i, vp]
        L.surr_pool_bwd.argtypes = [vp, vp, i, i, i, i, i, vp]
        L.surr_up_add_fwd.argtypes = [vp, vp, vp, i, i, i, i, i, vp]
        L.surr_up_bwd.argtypes = [vp, vp, vp, i, i, i, i, i, vp]
        L.surr_mse.argtypes = [vp, vp, vp, vp, ll, i, i, vp]
        L.surr_adam.argtypes = [vp, vp, vp, vp, vp, ll, f, f, f, f, i, vp]
        L.surr_add.argtypes = [vp, vp, vp, vp, ll, vp]
        L.surr_to_bf16.argtypes = [vp, vp, ll, vp]
        L.surr_to_f32.argtypes = [vp, vp, ll, vp]
        L.surr_pack_input.argtypes = [vp, vp, ll, i, i, vp]
        _bound = True
    return L


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _ok(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed ({rc})")


class Network:
    """The encoder-decoder on the GPU for inputs of shape (n, d, h, w); d, h, w divisible by 4."""

    def __init__(self, n: int, d: int, h: int, w: int, seed: int = 0, lr: float = 1e-3, stream=None,
                 device: str = "cuda"):
        import torch

        if d % 4 or h % 4 or w % 4:
            raise ValueError("d, h and w must be multiples of 4")
        self.torch = torch
        self.shape = (n, d, h, w)
        self.lr = lr
        self.t = 0
        self.stream = stream
        self.device = dev = device
        rng = np.random.default_rng(seed)
        # Every layer's weights [27][cout][cin] and bias [cout] are views into flat buffers
        # (FP32 master copy, BF16 copy, gradient, Adam moments), so one Adam launch updates
        # them all; each segment is a multiple of 8 elements, which keeps the BF16 views
        # 16-byte aligned for the convolution kernels.
        sizes = [(27 * cout * cin, cout) for _, cin, cout in LAYERS]
        self.nparams = total = sum(a + b for a, b in sizes)
        flat = {k: torch.zeros(total, dtype=torch.float32, device=dev) for k in ("w", "g", "m", "v")}
        self._flat = flat
        self._flat_bf16 = torch.empty(total, dtype=torch.int16, device=dev)
        self.w32, self.wbf, self.wt, self.b, self.gw, self.gb, self.m, self.v = {}, {}, {}, {}, {}, {}, {}, {}
        off = 0
        for (name, cin, cout), (nw, nb) in zip(LAYERS, sizes):
            std = math.sqrt(2.0 / (27 * cin))
            w0 = rng.normal(0.0, std, size=(27, cout, cin)).astype(np.float32)
            if name == "out":
                w0 *= 0.1  # start close to "no change"
            wv = lambda k: flat[k][off:off + nw].view(27, cout, cin)
            bv = lambda k: flat[k][off + nw:off + nw + nb]
            self.w32[name], self.b[name] = wv("w"), bv("w")
            self.w32[name].copy_(torch.from_numpy(w0))
            self.gw[name], self.gb[name] = wv("g"), bv("g")
            self.m[name] = (wv("m"), bv("m"))
            self.v[name] = (wv("v"), bv("v"))
            self.wbf[name] = self._flat_bf16[off:off + nw].view(27, cout, cin)
            self.wt[name] = torch.empty((27, cin, cout), dtype=torch.int16, device=dev)
            off += nw + nb
        self._refresh_bf16()
        self.act: Dict[str, "torch.Tensor"] = {}
        self.grad: Dict[str, "torch.Tensor"] = {}

        def buf(key, dims, c, dtype=torch.int16):
            self.act[key] = torch.empty(dims + (c,), dtype=dtype, device=dev)

        full, half, quarter = (n, d, h, w), (n, d // 2, h // 2, w // 2), (n, d // 4, h // 4, w // 4)
        for key, dims, c in [("x", full, 8), ("e1a", full, 32), ("e1", full, 32), ("p1", half, 32), ("e2", half, 64),
                             ("p2", quarter, 64), ("bt", quarter, 64), ("u2", half, 64), ("d2", half, 32),
                             ("u1", full, 32), ("d1", full, 32)]:
            buf(key, dims, c)
        self.y = torch.empty(full + (32,), dtype=torch.float32, device=dev)
        self.g_full32 = [torch.empty(full + (32,), dtype=torch.int16, device=dev) for _ in range(3)]
        self.g_half64 = [torch.empty(half + (64,), dtype=torch.int16, device=dev) for _ in range(2)]
        self.g_half32 = torch.empty(half + (32,), dtype=torch.int16, device=dev)
        self.g_half32b = torch.empty(half + (32,), dtype=torch.int16, device=dev)
        self.g_quarter64 = [torch.empty(quarter + (64,), dtype=torch.int16, device=dev) for _ in range(2)]
        L = _lib()
        sc = max(L.surr_conv3d_wgrad_scratch_bytes(n, d, h, w, cin, cout) for _, cin, cout in LAYERS)
        self.scratch = torch.empty(int(sc) // 4 + 1, dtype=torch.float32, device=dev)
        self.loss_part = torch.empty((n * d * h * w + 255) // 256, dtype=torch.float32, device=dev)

    # ------------------------------------------------------------ parameters
    def _refresh_bf16(self):
        L = _lib()
        for name, cin, cout in LAYERS:
            _ok(L.surr_to_bf16(_p(self.w32[name]), _p(self.wbf[name]), self.w32[name].numel(), self.stream), "to_bf16")
            _ok(L.surr_conv3d_flip_weights(_p(self.wbf[name]), _p(self.wt[name]), cin, cout, self.stream), "flip")

    def set_params(self, params: dict):
        """Load weights [27][cout][cin] and biases from host arrays."""
        for name, _, _ in LAYERS:
            w, b = params[name]
            self.w32[name].copy_(self.torch.from_numpy(np.asarray(w, dtype=np.float32)))
            self.b[name].copy_(self.torch.from_numpy(np.asarray(b, dtype=np.float32)))
        self._refresh_bf16()

    def get_params(self) -> dict:
        return {name: (self.w32[name].cpu().numpy(), self.b[name].cpu().numpy()) for name, _, _ in LAYERS}

    # ------------------------------------------------------------ forward / backward
    def _conv(self, src, name, dst, dims, relu=True, out_f32=None):
        L = _lib()
        _, cin, cout = next(l for l in LAYERS if l[0] == name)
        _ok(L.surr_conv3d_fwd(_p(src), _p(self.wbf[name]), _p(self.b[name]), _p(dst), _p(out_f32), *dims, cin, cout,
                              1 if relu else 0, self.stream), f"conv {name}")

    def _device_f32(self, a):
        """A host array or a device tensor as a contiguous FP32 tensor on the network's device."""
        t = self.torch
        if isinstance(a, t.Tensor):
            if a.device.type != t.device(self.device).type or a.dtype != t.float32:
                raise TypeError("expected an FP32 tensor on the network's device")
            return a.contiguous()
        return t.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(self.device)

    def set_input(self, x):
        """x: (n, d, h, w, 4) host array or FP32 device tensor."""
        xf = self._device_f32(x)
        if tuple(xf.shape) != self.shape + (FIELDS,):
            raise ValueError(f"input of shape {tuple(xf.shape)}, expected {self.shape + (FIELDS,)}")
        nv = self.shape[0] * self.shape[1] * self.shape[2] * self.shape[3]
        _ok(_lib().surr_pack_input(_p(xf), _p(self.act["x"]), nv, FIELDS, IN_CH, self.stream), "input")

    def forward(self):
        L = _lib()
        n, d, h, w = self.shape
        full, half, quarter = (n, d, h, w), (n, d // 2, h // 2, w // 2), (n, d // 4, h // 4, w // 4)
        A = self.act
        self._conv(A["x"], "e1a", A["e1a"], full)
        self._conv(A["e1a"], "e1b", A["e1"], full)
        _ok(L.surr_pool_fwd(_p(A["e1"]), _p(A["p1"]), *full, 32, self.stream), "pool1")
        self._conv(A["p1"], "e2", A["e2"], half)
        _ok(L.surr_pool_fwd(_p(A["e2"]), _p(A["p2"]), *half, 64, self.stream), "pool2")
        self._conv(A["p2"], "bt", A["bt"], quarter)
        _ok(L.surr_up_add_fwd(_p(A["bt"]), _p(A["e2"]), _p(A["u2"]), *quarter, 64, self.stream), "up2")
        self._conv(A["u2"], "d2", A["d2"], half)
        _ok(L.surr_up_add_fwd(_p(A["d2"]), _p(A["e1"]), _p(A["u1"]), *half, 32, self.stream), "up1")
        self._conv(A["u1"], "d1", A["d1"], full)
        self._conv(A["d1"], "out", None, full, relu=False, out_f32=self.y)
        return self.y

    def _dgrad(self, dout, name, din, dims, relu_y=None):
        _, cin, cout = next(l for l in LAYERS if l[0] == name)
        _ok(_lib().surr_conv3d_dgrad(_p(dout), _p(self.wt[name]), _p(relu_y), _p(din), *dims, cin, cout, self.stream),
            f"dgrad {name}")

    def _wgrad(self, inp, dout, name, dims):
        _, cin, cout = next(l for l in LAYERS if l[0] == name)
        _ok(_lib().surr_conv3d_wgrad(_p(inp), _p(dout), _p(self.gw[name]), _p(self.gb[name]), _p(self.scratch), *dims,
                                     cin, cout, self.stream), f"wgrad {name}")

    def _add(self, a, b, out, relu_y=None):
        _ok(_lib().surr_add(_p(a), _p(b), _p(relu_y), _p(out), a.numel(), self.stream), "add")

    def backward(self, dy):
        """dy: BF16 gradient of the loss with respect to the 32-channel output.  Each ReLU's
        gradient is applied by the operator that produces the gradient of its output (data
        gradient, upsampling gradient or the skip addition)."""
        L = _lib()
        n, d, h, w = self.shape
        full, half, quarter = (n, d, h, w), (n, d // 2, h // 2, w // 2), (n, d // 4, h // 4, w // 4)
        A = self.act
        g0, g1, g2 = self.g_full32
        h0, h1 = self.g_half64
        q0, q1 = self.g_quarter64
        self._wgrad(A["d1"], dy, "out", full)
        self._dgrad(dy, "out", g1, full, relu_y=A["d1"])      # g1 = d(d1 pre-activation)
        self._wgrad(A["u1"], g1, "d1", full)
        self._dgrad(g1, "d1", g2, full)                        # g2 = d(u1) = d(e1 skip) + up-part
        _ok(L.surr_up_bwd(_p(g2), _p(A["d2"]), _p(self.g_half32b), *half, 32, self.stream), "up1_bwd")
        self._wgrad(A["u2"], self.g_half32b, "d2", half)       # g_half32b = d(d2 pre-activation)
        self._dgrad(self.g_half32b, "d2", h0, half)            # h0 = d(u2)
        _ok(L.surr_up_bwd(_p(h0), _p(A["bt"]), _p(q1), *quarter, 64, self.stream), "up2_bwd")
        self._wgrad(A["p2"], q1, "bt", quarter)                # q1 = d(bt pre-activation)
        self._dgrad(q1, "bt", q0, quarter)                     # d(p2)
        _ok(L.surr_pool_bwd(_p(q0), _p(h1), *half, 64, self.stream), "pool2_bwd")
        self._add(h1, h0, h1, relu_y=A["e2"])                  # d(e2 pre-activation): pool part + skip part
        self._wgrad(A["p1"], h1, "e2", half)
        self._dgrad(h1, "e2", self.g_half32, half)             # d(p1)
        _ok(L.surr_pool_bwd(_p(self.g_half32), _p(g0), *full, 32, self.stream), "pool1_bwd")
        self._add(g0, g2, g0, relu_y=A["e1"])                  # d(e1 pre-activation)
        self._wgrad(A["e1a"], g0, "e1b", full)
        self._dgrad(g0, "e1b", g1, full, relu_y=A["e1a"])      # d(e1a pre-activation)
        self._wgrad(A["x"], g1, "e1a", full)

    def loss_and_grad(self, target, sync: bool = True):
        """target: (n, d, h, w, 4) FP32 device tensor.  Returns (loss, BF16 gradient); with
        sync=False the loss is left on the device (read it with last_loss) and None returned."""
        dy = self.g_full32[2]
        nv = self.shape[0] * self.shape[1] * self.shape[2] * self.shape[3]
        _ok(_lib().surr_mse(_p(self.y), _p(target), _p(dy), _p(self.loss_part), nv, 32, FIELDS, self.stream), "mse")
        return (self.last_loss() if sync else None), dy

    def last_loss(self) -> float:
        """Loss of the last loss_and_grad call (waits for it)."""
        nv = self.shape[0] * self.shape[1] * self.shape[2] * self.shape[3]
        return float(self.loss_part.cpu().numpy().astype(np.float64).sum()) / (nv * FIELDS)

    def adam_step(self, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step over every weight and bias (one launch over the flat buffers), then
        the mirrored weights of the data gradient."""
        self.t += 1
        L = _lib()
        f = self._flat
        _ok(L.surr_adam(_p(f["w"]), _p(self._flat_bf16), _p(f["g"]), _p(f["m"]), _p(f["v"]), self.nparams, self.lr,
                        beta1, beta2, eps, self.t, self.stream), "adam")
        for name, cin, cout in LAYERS:
            _ok(L.surr_conv3d_flip_weights(_p(self.wbf[name]), _p(self.wt[name]), cin, cout, self.stream), "flip")

    def train_step(self, x, target, sync_loss: bool = True):
        """One forward, backward and Adam step on (x, target): host arrays or FP32 device
        tensors of shape (n, d, h, w, 4).  Returns the loss (None with sync_loss=False)."""
        self.set_input(x)
        self.forward()
        loss, dy = self.loss_and_grad(self._device_f32(target), sync=sync_loss)
        self.backward(dy)
        self.adam_step()
        return loss

    def predict(self, x: np.ndarray) -> np.ndarray:
        """State after the horizon: x + the network's change (host arrays, (n, d, h, w, 4))."""
        self.set_input(x)
        y = self.forward()
        return x + y[..., :FIELDS].cpu().numpy()


# ---------------------------------------------------------------- data from the method
def coarse_state(lat, u_scale: float, factor: int = 4) -> np.ndarray:
    """(phi, u / u_scale) of a lattice averaged over factor^3 blocks: (d, h, w, 4) with
    (d, h, w) = (nz, ny, nx) / factor."""
    nz, ny, nx = lat.shape
    out = []
    for name, s in (("phi", 1.0), ("ux", u_scale), ("uy", u_scale), ("uz", u_scale)):
        f = lat.field(name) / s
        out.append(f.reshape(nz // factor, factor, ny // factor, factor, nx // factor, factor).mean(axis=(1, 3, 5)))
    return np.stack(out, axis=-1)


def trajectories(problems, horizon: int, snapshots: int, storage: str = "f32") -> np.ndarray:
    """Coarse states of every problem every `horizon` steps, run together as one batch:
    array (snapshots + 1, ncases, d, h, w, 4)."""
    b = _lbm.Batch(problems, storage=storage)
    u = problems[0].u_in
    states = [np.stack([coarse_state(c, u) for c in b.cases])]
    for _ in range(snapshots):
        b.step(horizon)
        b.sync()
        states.append(np.stack([coarse_state(c, u) for c in b.cases]))
    b.close()
    return np.stack(states)


def interface_error_coarse(phi_a: np.ndarray, phi_b: np.ndarray) -> float:
    """Mean interface displacement of phi_a against phi_b, in coarse cells."""
    from .metrics import interface_position_error

    return interface_position_error(phi_a, phi_b, periodic=(True, True, False))["mean_lu"]



# ---------------------------------------------------------------- surrogate in a sweep
BOX = (256, 64, 64)  # padded coarse input (d, h, w) = (z, y, x): 4x-coarsened lattices up to 256 x 256 x 1024


def coarse_trajectories(problems, horizon: int, snapshots: int, storage: str = "f16", box=BOX, factor: int = 4,
                        progress=None):
    """Coarse states (phi, u / u_in) of every problem every `horizon` steps, the problems
    advanced together as one batch; kept on the GPU.  Returns (states, lattice seconds,
    unstable cases): states is an FP32 tensor (snapshots + 1, ncases, d, h, w, 4) with each
    case's coarse lattice in the leading corner of the d x h x w box and zeros beyond it.
    `progress(text)`, if given, is called after the set-up and after every snapshot."""
    import time

    import torch

    b = _lbm.Batch(problems, storage=storage, progress=progress)
    out = torch.zeros((snapshots + 1, len(problems)) + tuple(box) + (FIELDS,), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()  # the zeros are in place before the library writes into them
    u = problems[0].u_in

    def grab(s):
        for k, c in enumerate(b.cases):
            c.coarse_state_into(out[s, k], factor, u)

    grab(0)
    if progress:
        progress(f"{len(problems)} cases set up")
    t_lbm = 0.0
    for s in range(1, snapshots + 1):
        b.sync()
        t0 = time.perf_counter()
        b.step(horizon)
        b.sync()
        t_lbm += time.perf_counter() - t0
        grab(s)
        if progress:
            progress(f"snapshot {s}/{snapshots}")
    b.sync()
    unstable = b.unstable_cases()
    b.close()
    return out, t_lbm, unstable


def coarse_extent(pb, factor: int = 4):
    """(d, h, w) of a problem's coarse lattice."""
    return pb.nz // factor, pb.ny // factor, pb.nx // factor


class Ensemble:
    """`members` networks of batch size `batch` on the padded box, initialised from different
    seeds and trained on the same pairs in different orders."""

    def __init__(self, batch: int, box=BOX, members: int = 3, seed: int = 0, lr: float = 2e-3):
        self.batch = batch
        self.box = tuple(box)
        self.nets = [Network(batch, *box, seed=seed + 101 * m, lr=lr) for m in range(members)]
        self.scale = None  # per-field RMS of the change over a horizon (the networks predict change / scale)

    def train(self, states, cases, steps: int, seed: int = 0):
        """`steps` Adam steps per member on pairs (state s, change to s + 1) of the given cases
        (states: tensor (T + 1, C, d, h, w, 4)); the change is learnt in units of its per-field
        RMS over these pairs.  Returns each member's (first, last) mean loss over 20 steps."""
        import torch

        T = states.shape[0] - 1
        idx = torch.as_tensor(np.asarray(cases), device=states.device)
        sq = torch.zeros(FIELDS, dtype=torch.float64, device=states.device)
        for s in range(T):
            dlt = (states[s + 1, idx] - states[s, idx]).double()
            sq += (dlt * dlt).sum(dim=(0, 1, 2, 3))
        nvox = T * len(cases) * int(np.prod(self.box))
        self.scale = torch.clamp((sq / nvox).sqrt(), min=1e-6).float()
        out = []
        for m, net in enumerate(self.nets):
            rng = np.random.default_rng(seed + 7 * m)
            losses = []
            for it in range(steps):
                s_idx = torch.from_numpy(rng.integers(0, T, size=self.batch)).cuda()
                k_idx = torch.from_numpy(rng.choice(np.asarray(cases), size=self.batch)).cuda()
                x = states[s_idx, k_idx].contiguous()
                target = ((states[s_idx + 1, k_idx] - x) / self.scale).contiguous()
                sync = it < 20 or it >= steps - 20
                loss = net.train_step(x, target, sync_loss=sync)
                if sync:
                    losses.append(loss)
            out.append((float(np.mean(losses[:20])), float(np.mean(losses[-20:]))))
        return out

    def predict(self, x):
        """Next coarse states of x ((n, d, h, w, 4) device tensor, n <= batch) by every member:
        a list of (n, d, h, w, 4) device tensors."""
        import torch

        n = x.shape[0]
        xb = torch.zeros((self.batch,) + self.box + (FIELDS,), dtype=torch.float32, device=x.device)
        xb[:n] = x
        preds = []
        for net in self.nets:
            net.set_input(xb)
            y = net.forward()
            preds.append(x + y[:n, ..., :FIELDS] * self.scale)
        return preds


def predicted_interface_error(member_phis, extent) -> float:
    """Spread of the members' interface positions (coarse cells): the largest mean
    displacement between any two members' phi fields, on the case's coarse lattice."""
    d, h, w = extent
    worst = 0.0
    for a in range(len(member_phis)):
        for b in range(a + 1, len(member_phis)):
            pa, pb = member_phis[a][:d, :h, :w], member_phis[b][:d, :h, :w]
            worst = max(worst, interface_error_coarse(pa, pb), interface_error_coarse(pb, pa))
    return worst


def fast_forward(ens: Ensemble, states, truth, cases, extents, start: int, horizons: int, limit: float = 1.0):
    """Advance `cases` from snapshot `start` by up to `horizons` horizons with the ensemble.
    states: the sweep's own lattice trajectories (the fallback), truth: the plain FP32
    lattice's, both (T + 1, C, d, h, w, 4) device tensors.  A case is advanced by the
    ensemble mean while the predicted interface error stays within `limit` coarse cells; from
    the first horizon where it does not, the case falls back to the lattice.  Every accepted
    prediction is scored against the FP32 lattice (interface error in coarse cells).

    Returns dict: per case the horizons taken by the surrogate, their predicted and actual
    errors, and the actual error of the first rejected prediction (if any)."""
    import torch

    report = {}
    for k, ext in zip(cases, extents):
        state = states[start, k:k + 1]
        taken, pred_err, actual_err, rejected = 0, [], [], None
        for r in range(1, horizons + 1):
            members = ens.predict(state)
            phis = [p[0, ..., 0].cpu().numpy() for p in members]
            perr = predicted_interface_error(phis, ext)
            mean = torch.stack(members).mean(0)
            d, h, w = ext
            act = interface_error_coarse(mean[0, :d, :h, :w, 0].cpu().numpy(),
                                         truth[start + r, k, :d, :h, :w, 0].cpu().numpy())
            if perr > limit:
                rejected = {"horizon": r, "predicted": perr, "actual": act}
                break
            taken += 1
            pred_err.append(perr)
            actual_err.append(act)
            state = mean
        report[k] = {"taken": taken, "predicted": pred_err, "actual": actual_err, "rejected": rejected}
    return report
