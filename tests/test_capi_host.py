"""Host-side checks of the HIP library (no GPU needed).

* The library builds, loads and exports every function include/lbm.h declares.
* Parameter validation rejects what the method does not allow, before touching a device.
* The step kernel's per-cell arithmetic (factored moment transform, closed-form source
  moments, 32-value recoloured state), compiled for the host, reproduces the oracle's
  per-colour post-collision populations.
"""
import ctypes
import itertools

import numpy as np
import pytest

from paper_1705_03141_amd import lbm
from paper_1705_03141_amd import workloads as W


@pytest.fixture(scope="module")
def L():
    return lbm.library()


def test_exports_every_declared_symbol(L):
    names = lbm.header_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    # the surrogate's operators (include/surrogate.h) live in the same library
    import os
    import re
    with open(os.path.join(os.path.dirname(lbm.HEADER), "surrogate.h")) as fh:
        surr = set(re.findall(r"^\s*(?:[a-z_0-9]+\s+)+\**\s*(surr_[a-z_0-9]+)\s*\(", fh.read(), re.M))
    assert len(surr) >= 14
    for n in surr:
        assert hasattr(L, n), n


def _expect(status_code, problem, **override):
    p = lbm.params_from_problem(problem)
    for k, v in override.items():
        setattr(p, k, v)
    ctx = ctypes.c_void_p()
    st = lbm.library().lbm_create(ctypes.byref(p), None, ctypes.byref(ctx))
    assert st == status_code, lbm.library().lbm_last_error(None)


def test_parameter_validation(L):
    pb = W.cfg_static_droplet()
    _expect(lbm.LBM_EINVAL, pb, nu_r=0.0)
    _expect(lbm.LBM_EINVAL, pb, beta=1.5)
    _expect(lbm.LBM_EINVAL, pb, A=-1.0)
    _expect(lbm.LBM_EINVAL, pb, nx=0)
    # the largest x-y plane the kernels' 32-bit byte offsets address: nx*ny*108 < 2^31
    _expect(lbm.LBM_EINVAL, pb, nx=4460, ny=4460, nz=3)
    _expect(lbm.LBM_EINVAL, pb, nx=19884108, ny=1, nz=3)
    # gamma < 19/27 gives alpha_r < 0
    _expect(lbm.LBM_EINVAL, pb, rho_r0=0.5, rho_b0=1.0)
    # x and y faces: both periodic or both free-slip (lateral walls); z faces paired
    ctx = ctypes.c_void_p()
    for faces in ((W.BOUNCEBACK, W.BOUNCEBACK), (W.FREESLIP, W.PERIODIC), (W.OUTFLOW, W.OUTFLOW)):
        for d in (0, 1):
            p = lbm.params_from_problem(pb)
            p.face[2 * d], p.face[2 * d + 1] = faces
            assert L.lbm_create(ctypes.byref(p), None, ctypes.byref(ctx)) == lbm.LBM_EINVAL, (d, faces)
    p = lbm.params_from_problem(pb)
    p.face[4] = W.BOUNCEBACK
    assert L.lbm_create(ctypes.byref(p), None, ctypes.byref(ctx)) == lbm.LBM_EINVAL
    # relaxation rates: conserved rows must be zero, groups of K equal, rates in (0, 2)
    s = list(W.UNIT_RATES)
    s[0] = 1.0
    pb2 = W.cfg_static_droplet()
    pb2.s = s
    _expect(lbm.LBM_EINVAL, pb2)
    s = list(W.UNIT_RATES)
    s[11] = 1.2
    pb2.s = s
    _expect(lbm.LBM_EINVAL, pb2)
    s = list(W.UNIT_RATES)
    s[26] = 2.0
    pb2.s = s
    _expect(lbm.LBM_EINVAL, pb2)


def test_create_without_gpu_reports_device_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    _expect(lbm.LBM_EDEVICE, W.cfg_static_droplet())
    # free-slip lateral walls pass validation
    _expect(lbm.LBM_EDEVICE, W.jet(nx=24, ny=24, nz=48, diameter=8.0, lateral=W.FREESLIP))
    # the largest plane passes validation (and only then meets the missing device)
    _expect(lbm.LBM_EDEVICE, W.cfg_static_droplet(), nx=19884107, ny=1, nz=3)


def test_null_context_arguments_are_rejected(L):
    """Calls on a NULL context return LBM_EINVAL without touching a device."""
    i = ctypes.c_int()
    assert L.lbm_autotune(None, 5) == lbm.LBM_EINVAL
    assert L.lbm_get_tiling(None, ctypes.byref(i), ctypes.byref(i), ctypes.byref(i)) == lbm.LBM_EINVAL
    assert L.lbm_set_tiling(None, 32, 8, 0) == lbm.LBM_EINVAL
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_sync(None) == lbm.LBM_EINVAL


@pytest.mark.parametrize("case", ["droplet", "suga_ratio3", "force_rt"])
def test_host_collision_matches_oracle(oracle_lib, case):
    O = oracle_lib
    rng = np.random.default_rng({"droplet": 1, "suga_ratio3": 2, "force_rt": 3}[case])
    if case == "droplet":
        pb = W.cfg_static_droplet()
    elif case == "suga_ratio3":
        pb = W.static_droplet(n=8, radius=2.5, rho_r0=3.0, rho_b0=1.0, nu=2e-2, A=0.01, beta=0.7)
        pb.nu_r, pb.nu_b = 3e-2, 5e-3
    else:
        pb = W.rayleigh_taylor(width=8, height=12, g=1e-4, reynolds=64.0)
    o = O.Oracle(pb)
    ar = o.alpha_r
    worst = 0.0
    for _ in range(100):
        a, rho = rng.uniform(0, 1), rng.uniform(0.5, 3.0)
        u = rng.normal(scale=0.03, size=3)
        fr = O.colour_equilibrium(a * rho, ar, u) * (1 + 0.02 * rng.normal(size=27))
        fb = O.colour_equilibrium((1 - a) * rho, 8 / 27, u) * (1 + 0.02 * rng.normal(size=27))
        gp, gr = rng.normal(size=3) * 0.2, rng.normal(size=3) * 0.1
        F = np.zeros(3)
        if pb.force_model:
            F = (fr.sum() + fb.sum() - pb.rho_ref) * np.array(pb.g)
        want_r, want_b = o.collide_cell(fr, fb, gp, gr, F)
        got_r, got_b = lbm.selftest_collide_host(pb, fr, fb, gp, gr)
        scale = np.abs(want_r + want_b).max()
        worst = max(worst, np.abs(got_r - want_r).max() / scale, np.abs(got_b - want_b).max() / scale)
    # FP32 arithmetic on deviations, values rebuilt around O(1) rest equilibria
    assert worst < 2e-6, worst


def test_sigma_helpers_match_table2(L):
    """The library's Eq. (sigma) helpers reproduce the interfacial tension the paper lists for
    every (nu, A) pair of its oscillating-droplet table (three significant digits), and
    lbm_A_from_sigma inverts lbm_sigma_from_A."""
    import math
    import os
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "table2_oscillating_droplet.txt"))
    for nu, A, sigma, _ in rows:
        s = lbm.sigma_from_A(A, nu)
        assert abs(s - sigma) <= 0.006 * sigma, (nu, A, s, sigma)
        assert abs(lbm.A_from_sigma(s, nu) - A) <= 1e-15 * A
    # the jet workload's surface-tension parameter is the same conversion at the continuous phase
    pb = W.jet(nx=32, ny=32, nz=64, diameter=8.0, u_in=0.04, weber=220.0, fields=False)
    sigma_we = pb.rho_r0 * 0.04 ** 2 * 8.0 / 220.0   # We = rho_j u^2 D / sigma, Eq. (jetWeber)
    assert pb.A is None and abs(pb.sigma - sigma_we) <= 1e-15 * sigma_we
    assert abs(lbm.sigma_from_A(lbm.params_from_problem(pb).A, pb.nu_b) - sigma_we) <= 1e-12 * sigma_we
    assert math.isnan(lbm.sigma_from_A(1e-2, 0.0)) and math.isnan(lbm.A_from_sigma(-1.0, 0.1))


@pytest.mark.parametrize("dims,faces", [((100, 44, 24), "xy"), ((256, 256, 16), "xy"), ((240, 40, 8), "x"),
                                        ((96, 64, 8), "y"), ((70, 36, 20), ""), ((37, 29, 23), "xy")])
def test_tile_sets_cover_every_tile_once(L, dims, faces):
    """With lateral walls the step launches the plain pull over the interior tiles and the
    reflecting instances over the frame (one launch per axis, or per wall with FP16 storage):
    every tile is processed exactly once, a tile is interior exactly when none of its cells or
    ring cells lies on a wall (checked here from the geometry, cell by cell), and no frame tile
    touches a wall its launch does not reflect at (checked by the library)."""
    pb = W.static_droplet(dims=dims, radius=3.0, rho_r0=1.5, rho_b0=1.0, nu=0.05, A=0.01)
    pb.faces = (W.FREESLIP if "x" in faces else W.PERIODIC,) * 2 + (W.FREESLIP if "y" in faces else W.PERIODIC,) * 2 \
        + (W.FREESLIP, W.FREESLIP)
    nx, ny = dims[0], dims[1]
    for (tx, ty), storage in itertools.product(((32, 4), (32, 8), (64, 4), (64, 8), (32, 16)), ("f32", "f16")):
        c = lbm.selftest_tile_sets_host(pb, tx, ty, storage)
        assert np.all(c.sum(axis=0) == 1), (tx, ty)
        if not faces:
            assert np.all(c[0] == 1)
            continue
        assert np.all(c[0] == 0)
        for j in range(c.shape[1]):
            for i in range(c.shape[2]):
                xs = range(i * tx - 1, i * tx + tx + 1)  # own cells and the ring
                ys = range(j * ty - 1, j * ty + ty + 1)
                on_wall = ("x" in faces and any(x % nx in (0, nx - 1) for x in xs)) or \
                          ("y" in faces and any(y % ny in (0, ny - 1) for y in ys))
                assert c[1, j, i] == (0 if on_wall else 1), (tx, ty, i, j)
    with pytest.raises(lbm.LbmError):
        lbm.selftest_tile_sets_host(pb, 16, 16)
