"""Failure handling of the C ABI on the GPU: the step kernel's instability flag (NaN or
non-positive density) surfaced by lbm_sync and the read-back calls, per-case flags in a
batch, and checkpoint headers that refuse a state of another lattice.

The unstable state is made on the host: a saved state is edited so that one stored
population is NaN, loaded, and stepped.  Every kernel runs to completion as usual.
"""
import struct
import sys

import numpy as np
import pytest

from paper_1705_03141_amd import lbm
from paper_1705_03141_amd import workloads as W

pytestmark = pytest.mark.gpu

HEADER = 64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nan_state(lat: lbm.Lattice, cell: int) -> bytes:
    """The lattice's saved FP32 state with population 3 of `cell` set to NaN (populations
    follow the 64-byte header as [z][i][y][x] words; cell < nx*ny lies in plane z = 0)."""
    blob = lat.save_state()
    plane = lat.pb.nx * lat.pb.ny
    off = HEADER + (3 * plane + cell) * 4
    b = bytearray(blob)
    b[off:off + 4] = struct.pack("<I", 0x7FC00000)
    return bytes(b)


def test_unstable_state_is_reported():
    pb = W.small_configs()["droplet32"]
    lat = lbm.Lattice(pb)
    lat.step(5)
    lat.sync()
    lat.field("rho_r")  # clean state: no error
    bad = nan_state(lat, cell=100)
    lat.load_state(bad)
    lat.sync()  # the NaN is stored but no step has read it yet
    lat.step(2)
    with pytest.raises(lbm.LbmError) as e:
        lat.sync()
    assert e.value.status == lbm.LBM_EUNSTABLE
    with pytest.raises(lbm.LbmError) as e:
        lat.field("rho_r")
    assert e.value.status == lbm.LBM_EUNSTABLE
    assert lat.diagnostics()["unstable"]
    # a new initial state clears the flag
    lat.init_fields(pb.rho_r, pb.rho_b, pb.u)
    lat.step(3)
    lat.sync()
    assert np.isfinite(lat.field("rho_r")).all()


def test_checkpoint_rejects_other_lattices():
    pb = W.small_configs()["jet_small"]
    a = lbm.Lattice(pb)
    a.step(4)
    blob = a.save_state()
    other_size = W.jet(nx=24, ny=24, nz=40, diameter=8.0)
    for other, storage in ((other_size, "f32"), (pb, "f16")):
        b = lbm.Lattice(other, storage=storage)
        b.step(1)
        before = b.populations()
        padded = blob + bytes(max(0, b.save_state().__len__() - len(blob)))
        with pytest.raises(lbm.LbmError) as e:
            b.load_state(padded)
        assert e.value.status == lbm.LBM_EINVAL
        assert b.steps_done == 1 and np.array_equal(b.populations(), before)
    c = lbm.Lattice(pb, init=False)
    c.load_state(blob)
    assert c.steps_done == 4 and np.array_equal(c.populations(), a.populations())


def test_batch_freezes_unstable_case():
    pbs = [W.jet(nx=24, ny=24, nz=48, diameter=8.0, seed=s) for s in (11, 12, 13)]
    batch = lbm.Batch(pbs)
    batch.step(3)
    batch.sync()
    assert batch.unstable_cases() == []
    bad = nan_state(batch.cases[1], cell=30)
    batch.cases[1].load_state(bad)
    batch.step(4)
    assert batch.unstable_cases() == [1]
    batch.step(5)  # the flagged case is left out, the others go on
    assert batch.unstable_cases() == [1]
    steps = [c.steps_done for c in batch.cases]
    log(f"[batch] steps after freeze: {steps}")
    assert steps[0] == steps[2] == 12 and steps[1] < 12
    for k in (0, 2):
        single = lbm.Lattice(pbs[k])
        single.step(12)
        assert np.array_equal(batch.cases[k].populations(), single.populations()), k
        batch.cases[k].sync()
    with pytest.raises(lbm.LbmError) as e:
        batch.cases[1].sync()
    assert e.value.status == lbm.LBM_EUNSTABLE
    batch.close()
