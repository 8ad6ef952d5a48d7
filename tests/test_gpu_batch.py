"""GPU tests of batched stepping (lbm_batch_*): several uneven jet cases of a regime-map
sweep advanced by one launch per step.

* every case of the batch ends bitwise equal to the same case run alone (the batch kernel
  performs the single-lattice step on its share of the grid);
* one case against the FP64 oracle over 300 steps (1e-5 bar);
* the autotuner's tile choice leaves results bitwise unchanged;
* stepping a case of a batch on its own is refused.
"""
import sys

import numpy as np
import pytest

from paper_1705_03141_amd import lbm, metrics
from paper_1705_03141_amd import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def small_sweep(n=5):
    """Uneven jets of the sweep recipe on small lattices (24-40 cells wide, 4x as tall)."""
    return W.regime_sweep(ncases=n, seed=11, sizes=(24, 32, 40), diameters=(4, 8), fields=True)


def test_batch_matches_single_lattices():
    cases = small_sweep()
    log("[batch] " + ", ".join(f"{c.nx}x{c.ny}x{c.nz}" for c in cases))
    b = lbm.Batch(cases)
    b.step(40)
    b.sync()
    for k, pb in enumerate(cases):
        alone = lbm.Lattice(pb)
        alone.step(40)
        same = bool(np.array_equal(b.cases[k].populations(), alone.populations()))
        alone.close()
        assert same, f"case {k} differs from its single-lattice run"
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_with_lateral_walls_matches_single_lattices(storage):
    """Cases with free-slip lateral walls next to periodic ones: a wall case runs its interior
    tiles in a plain group and its frame in reflecting groups of the batch (one per axis, or
    one per wall with FP16 storage), and still ends bitwise equal to its single-lattice run."""
    cases = small_sweep(3)
    walls = [W.jet(nx=200, ny=72, nz=64, diameter=10.0, seed=5, lateral=W.FREESLIP),
             W.jet(nx=40, ny=40, nz=48, diameter=6.0, seed=6, lateral=W.FREESLIP)]
    cases = cases + walls
    log(f"[batch, walls, {storage}] " + ", ".join(f"{c.nx}x{c.ny}x{c.nz}" for c in cases))
    b = lbm.Batch(cases, storage=storage)
    b.step(30)
    b.sync()
    tx, ty, _ = b.cases[len(cases) - 2].tiling()
    assert lbm.selftest_tile_sets_host(walls[0], tx, ty, storage)[1].sum() > 0, "no interior tiles in the wall case"
    for k, pb in enumerate(cases):
        alone = lbm.Lattice(pb, storage=storage, tiling=b.cases[k].tiling())
        alone.step(30)
        same = bool(np.array_equal(b.cases[k].populations(), alone.populations()))
        alone.close()
        assert same, f"case {k} differs from its single-lattice run"
    b.close()


def test_batch_case_against_oracle(oracle_lib):
    cases = small_sweep(3)
    b = lbm.Batch(cases)
    o = oracle_lib.Oracle(cases[1])
    b.step(300)
    o.step(300)
    e = metrics.relative_errors(b.cases[1].fields(), o.fields())
    log(f"[batch] case 1 ({cases[1].name}) vs oracle, 300 steps: " + " ".join(f"{k}={v:.3e}" for k, v in e.items()))
    b.close()
    assert e["rho"] < 1e-5 and e["rho_r"] < 1e-5 and e["rho_b"] < 1e-5 and e["u"] < 1e-5, e


def test_autotune_keeps_results():
    cases = small_sweep(4)
    ref = lbm.Batch(cases)
    ref.step(25)
    tuned = lbm.Batch(cases)
    tuned.autotune(trial_steps=3)
    tuned.step(25)
    for k in range(len(cases)):
        assert np.array_equal(ref.cases[k].populations(), tuned.cases[k].populations()), k
    ref.close()
    tuned.close()


def test_case_of_a_batch_cannot_step_alone():
    cases = small_sweep(2)
    b = lbm.Batch(cases)
    with pytest.raises(lbm.LbmError) as ei:
        b.cases[0].step(1)
    assert ei.value.status == lbm.LBM_ESTATE
    b.close()
