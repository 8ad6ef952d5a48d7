"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

The oracle cannot run the full lattices for long, so it runs a window of the same problem
(Problem.window: the same seeded fields and inflow noise, cut faces turned into walls) and
the comparison is restricted to cells further than 2 (s + 1) cells from every cut face
after s steps: one step reads at most two cells away (the pull one, the density gradient
one more), so those cells have exactly the inputs of the full lattice.

Also here: the reduced jet (64 x 64 x 256, D = 8) over 1000 steps, per-colour mass over
1000 full-size Rayleigh-Taylor steps, and the interface-position error of FP16 and BF16
storage against FP32 storage.
"""
import os
import sys

import numpy as np
import pytest

from paper_1705_03141_amd import lbm
from paper_1705_03141_amd import metrics
from paper_1705_03141_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_box(lat, x0, y0, z0, wx, wy, wz):
    rr = lat.field_box("rho_r", x0, y0, z0, wx, wy, wz)
    rb = lat.field_box("rho_b", x0, y0, z0, wx, wy, wz)
    u = np.stack([lat.field_box(k, x0, y0, z0, wx, wy, wz) for k in ("ux", "uy", "uz")])
    return {"rho_r": rr, "rho_b": rb, "u": u}


def oracle_box(o, z0, wz):
    f = o.fields()
    return {"rho_r": f["rho_r"][z0:z0 + wz], "rho_b": f["rho_b"][z0:z0 + wz], "u": f["u"][:, z0:z0 + wz]}


def window_parity(O, pb, steps, cz0, cwz):
    """Full lattice on the GPU against an oracle window around z in [cz0, cz0 + cwz)."""
    margin = 2 * (steps + 1)
    wz0 = max(0, cz0 - margin)
    wz1 = min(pb.nz, cz0 + cwz + margin)
    win = pb.window(0, 0, wz0, pb.nx, pb.ny, wz1 - wz0)
    log(f"  GPU {pb.nx}x{pb.ny}x{pb.nz}, oracle window z [{wz0}, {wz1}), compare z [{cz0}, {cz0 + cwz}), "
        f"{steps} steps")
    lat = lbm.Lattice(pb)
    lat.step(steps)
    got = gpu_box(lat, 0, 0, cz0, pb.nx, pb.ny, cwz)
    lat.close()
    o = O.Oracle(win)
    o.step(steps)
    ref = oracle_box(o, cz0 - wz0, cwz)
    e = metrics.relative_errors(got, ref)
    log("  " + " ".join(f"{k}={v:.3e}" for k, v in e.items()))
    return e


def test_rayleigh_taylor_fullsize_window(oracle_lib):
    pb = W.cfg_rayleigh_taylor()
    log("[fullsize] Rayleigh-Taylor 128x128x512")
    e = window_parity(oracle_lib, pb, 40, 240, 32)
    assert e["rho"] < TOL and e["rho_r"] < TOL and e["rho_b"] < TOL and e["u"] < TOL, e


def test_rayleigh_taylor_fullsize_1000_steps():
    """The full Rayleigh-Taylor lattice (128 x 128 x 512) over the parity criterion's 1000
    steps, in the launch configuration bench.py times, against the FP64 oracle's fields on
    four planes (the lower wall plane and three through the perturbed interface), element by
    element.  The oracle's planes were written by tests/golden/make_rt_fullsize_golden.py
    (about 1.5 hours of the oracle on 8 host cores) and are normalised, as everywhere, by the
    oracle's maxima over the whole lattice."""
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "rt128x128x512_1000steps_planes.npz"))
    pb = W.cfg_rayleigh_taylor()
    assert int(g["steps"]) == 1000
    lat = lbm.Lattice(pb)
    lat.step(1000)
    planes = [int(z) for z in g["planes"]]
    got = {"rho_r": np.stack([lat.field_box("rho_r", 0, 0, z, pb.nx, pb.ny, 1)[0] for z in planes]),
           "rho_b": np.stack([lat.field_box("rho_b", 0, 0, z, pb.nx, pb.ny, 1)[0] for z in planes]),
           "u": np.stack([np.stack([lat.field_box(k, 0, 0, z, pb.nx, pb.ny, 1)[0] for z in planes])
                          for k in ("ux", "uy", "uz")])}
    lat.close()
    rho_max, u_max = float(g["max_rho"]), float(g["max_u"])
    e = {k: float(np.abs(got[k] - g[k].astype(np.float64)).max() / rho_max) for k in ("rho_r", "rho_b")}
    e["rho"] = float(np.abs(got["rho_r"] + got["rho_b"] - g["rho_r"].astype(np.float64)
                            - g["rho_b"].astype(np.float64)).max() / rho_max)
    e["u"] = float(np.abs(got["u"] - g["u"].astype(np.float64)).max() / u_max)
    log(f"[fullsize] RT 128x128x512, 1000 steps, planes {planes}: " + " ".join(f"{k}={v:.3e}" for k, v in e.items()))
    assert max(e.values()) < TOL, e


def test_jet_fullsize_window(oracle_lib):
    pb = W.cfg_jet()
    log("[fullsize] jet 256x256x1024 (inflow end)")
    e = window_parity(oracle_lib, pb, 40, 0, 8)
    assert e["rho"] < TOL and e["rho_r"] < TOL and e["rho_b"] < TOL and e["u"] < TOL, e


def test_reduced_jet_1000_steps(oracle_lib):
    """The reduced jet of the parity criterion: 64 x 64 x 256, D = 8, the physics of the
    full-size jet (inflow noise, free-slip inlet plane, convective outflow, gravity)."""
    pb = W.jet(nx=64, ny=64, nz=256, diameter=8.0)
    log("[reduced jet] 64x64x256 D=8, 1000 steps")
    lat = lbm.Lattice(pb)
    o = oracle_lib.Oracle(pb)
    lat.step(1000)
    o.step(1000)
    got = lat.fields()
    ref = o.fields()
    e = metrics.relative_errors(got, ref)
    log("  " + " ".join(f"{k}={v:.3e}" for k, v in e.items()))
    assert e["rho"] < TOL and e["rho_r"] < TOL and e["rho_b"] < TOL and e["u"] < TOL, e


def test_rayleigh_taylor_fullsize_mass_1000_steps():
    """Per-colour mass is conserved by the method (walls, periodic sides, no sources); the
    FP32 lattice must keep it to FP32 accumulation over 1000 full-size steps."""
    pb = W.cfg_rayleigh_taylor()
    lat = lbm.Lattice(pb)
    d0 = lat.diagnostics()
    lat.step(1000)
    d1 = lat.diagnostics()
    m0r, m0b = pb.rho_r.sum(), pb.rho_b.sum()
    dr = (d1["mass_r"] - m0r) / m0r
    db = (d1["mass_b"] - m0b) / m0b
    log(f"[mass] RT 128x128x512 1000 steps: red {dr:.2e} blue {db:.2e} (t=0 read-back {d0['mass_r'] / m0r - 1:.2e})")
    assert abs(dr) < 1e-6 and abs(db) < 1e-6
    assert d1["nan_cells"] == 0


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_half_storage_interface_error(storage):
    """FP16 / BF16 storage against FP32 storage on the full Rayleigh-Taylor lattice: the
    interface may move by at most 0.5 lattice units (2000 steps; the full 20000-step figure
    is measured by bench.py --interface-error)."""
    pb = W.cfg_rayleigh_taylor()
    ref = lbm.Lattice(pb, storage="f32")
    ref.step(2000)
    phi_ref = ref.field("phi")
    ref.close()
    lat = lbm.Lattice(pb, storage=storage)
    lat.step(2000)
    phi = lat.field("phi")
    lat.close()
    e = metrics.interface_position_error(phi, phi_ref)
    log(f"[interface] {storage} vs f32, RT 128x128x512, 2000 steps: {e}")
    assert e["cells"] > 0 and e["max_lu"] < 0.5, e
