"""Benchmark of the D3Q27 colour-fluid step on one MI355X.

Workload (default): the liquid jet on 256 x 256 x 1024 (D = 16 inflow disk with 1 % noise,
u = 0.04, gamma 1.6, nu 1.8e-4, We 220, Fr 8.5, free-slip inlet plane, convective outflow,
periodic sides), the largest single-GPU configuration the throughput metric is quoted on;
``--workload rt`` runs the Rayleigh-Taylor problem on 128 x 128 x 512 instead, and
``--workload jet_walls`` the same jet between free-slip lateral walls (the paper's set-up, a
step of up to four launches: interior tiles and the frame along the walls).  FP32
populations and arithmetic.  A "step" is one full time step of the method over the whole
lattice (outlet plane, fused step kernel, inflow plane).  Prints one JSON line:

  value       MLUPS = cells x steps / wall time of the timed steps (inputs resident in HBM)
  roofline    the step kernel against HBM: achieved = 432 B per cell update (one read and one
              write of 2 x 27 FP32 populations, the standard two-colour traffic of the
              method) x cells / mean kernel time from HIP events on the library's stream;
              peak 8000 GB/s.  The kernel itself keeps a 32-value state and moves 256 B per
              update; extra.measured_hbm_gbs is what the HBM counters saw over the same time.
  traffic     HBM bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a plain copy
              (null when the kernel sources differ from those the counters were taken on)
  cpu_baseline  the FP64 oracle timed on the host cores on a window of the same workload
              (rank 0, N = 1 only)

Also reported (extra): the FP16- and BF16-storage throughput, the bytes the kernel itself
must move per update (27 stored deviations + 5 FP32 scalars, read and written once) and
that fraction of the roofline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_GBS = 8000.0
# HBM bytes per step-kernel launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
# scaled by what the counters read for a plain 1 GiB copy (fetch x2.000, write x1.000), per
# workload; valid only for the kernel sources and tile shape they were taken on.
COUNTERS = {
    "jet_256x256x1024": {"sources_sha16": "f1aa97277de1a3f4", "storage": "f32", "fetch_kib": 4771980.0, "fetch_scale": 2.0,
                         "write_kib": 8388608.0, "write_scale": 1.0, "tile": [64, 4]},
    "rayleigh_taylor_128x128x512": {"sources_sha16": "f1aa97277de1a3f4", "storage": "f32", "fetch_kib": 559488.3,
                                    "fetch_scale": 2.0, "write_kib": 1048576.0, "write_scale": 1.0, "tile": [64, 4]},
}
KERNEL_SOURCES = ["csrc/lbm_cell.h", "csrc/lbm_device.h", "csrc/lbm_kernels.h", "csrc/lbm_kernels_impl.h",
                  "csrc/lbm_step.h", "csrc/lbm_storage_f32.hip", "build.py"]
STD_BYTES = 432.0  # 2 colours x 27 populations x 4 B, read + write


def state_bytes(storage: str) -> float:
    elem = 4 if storage == "f32" else 2
    return 2.0 * (27 * elem + 5 * 4)


def run_gpu(pb, storage, steps, warmup, autotune=False):
    import torch
    from paper_1705_03141_amd import lbm

    lat = lbm.Lattice(pb, storage=storage)
    if autotune:
        lat.autotune(trial_steps=30)  # tile shape timed on a scratch lattice, outside the timed region
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = lat.last_step_kernel_ms()
    diag = lat.diagnostics()
    diag["tiling"] = lat.tiling()
    lat.close()
    return wall, kernel_ms, diag


def kernel_sources_sha16() -> str:
    import hashlib

    h = hashlib.sha256()
    for fn in KERNEL_SOURCES:
        with open(os.path.join(HERE, "paper_1705_03141_amd", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, tile, workload: str):
    """HBM bytes per launch, or None when no counters were taken on this workload, or they were
    taken on other kernel sources, another storage or another tile shape."""
    c = COUNTERS.get(workload)
    if (c is None or storage != c["storage"] or kernel_sources_sha16() != c["sources_sha16"]
            or list(tile[:2]) != c["tile"]):
        return None
    return (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_baseline(pb_full, steps=150):
    """The FP64 oracle on a window of the workload: the jet's first 16 planes (inflow disk and
    free-slip inlet plane, about 1 M cells), or the 64 planes around the Rayleigh-Taylor
    interface."""
    import numpy as np  # noqa: F401
    import oracle

    if pb_full.inflow:
        win = pb_full.window(0, 0, 0, pb_full.nx, pb_full.ny, 16)
    else:
        win = pb_full.window(0, 0, pb_full.nz // 2 - 32, pb_full.nx, pb_full.ny, 64)
    o = oracle.Oracle(win)
    o.step(1)  # first touch
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    where = "at the inflow end" if pb_full.inflow else "around the interface"
    return {"value": win.ncells * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{win.nx}x{win.ny}x{win.nz} window of the same workload {where}, {steps} steps, {dt:.1f} s"}


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE per dispatch
    against nbytes gives the scale of those counters."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms": ms,
                      "GBps_read_plus_write": 2 * nbytes / ms / 1e6}), flush=True)


def sweep(steps: int, warmup: int, storage: str = "f16"):
    """The regime-map sweep: 64 uneven jet cases (96^2 x 384 to 160^2 x 640, about 0.63 G
    cells) advanced together by lbm_batch_step after the autotuner has chosen tile shapes."""
    import torch
    from paper_1705_03141_amd import lbm
    from paper_1705_03141_amd import workloads as W

    cases = W.regime_sweep()
    ncells = sum(c.ncells for c in cases)
    log(f"sweep: {len(cases)} cases, {ncells / 1e6:.0f} M cells, storage {storage}")
    b = lbm.Batch(cases, storage=storage, progress=lambda m: log(f"sweep: {m}"))
    free, total = torch.cuda.mem_get_info()
    used_gb = (total - free) / 1e9  # device memory in use once every case holds its state
    log(f"sweep: initialised, {used_gb:.1f} GB of {total / 1e9:.0f} GB in use; autotuning")
    b.autotune(trial_steps=5)
    b.step(warmup)
    b.sync()
    torch.cuda.synchronize()
    # long runs go in chunks of 500 steps, after each of which the step the cases the kernel
    # flagged as unstable were found at is noted (a flagged case is no longer stepped)
    found = {}
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(500, steps - done) if steps > 1000 else steps
        b.step(k)
        done += k
        for c in b.unstable_cases():
            found.setdefault(c, warmup + done)
        if steps > 1000:
            log(f"sweep: {done}/{steps} steps, {len(found)} unstable")
    b.sync()
    wall = time.perf_counter() - t0
    unstable = [{"case": k, "name": cases[k].name, "regime": cases[k].regime, "found_by_step": s}
                for k, s in sorted(found.items())]
    mlups = ncells * steps / wall / 1e6
    std_bytes = 432.0 if storage == "f32" else 216.0
    achieved = std_bytes * ncells / (b.last_step_ms() * 1e-3) / 1e9
    print(json.dumps({"metric": "MLUPS, batched regime-map sweep (64 jet cases)", "value": mlups, "unit": "MLUPS",
                      "steps": steps, "warmup": warmup, "ms_per_step": wall * 1e3 / steps, "dtype": f"f32 compute, {storage} storage",
                      "config": {"workload": "regime_sweep_64_jets", "cases": len(cases), "cells": ncells,
                                 "device_memory_gb": used_gb},
                      "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_GBS, "unit": "GB/s",
                                   "frac": achieved / PEAK_GBS, "bytes_per_cell": std_bytes},
                      "unstable_cases": unstable,
                      "regimes": {r: sum(1 for c in cases if c.regime == r) for r in ("I", "II", "III")}}), flush=True)
    b.close()


def slab_bench(steps: int, warmup: int):
    """One GPU's share of the jet 256 x 256 x 1024 split into z-slabs over 8 GPUs: the step
    kernel on a 256 x 256 x 128 slab of jet physics (gamma 1.6, nu 1.8e-4, We 220, a red
    column of D = 16 through it), z periodic in place of the two neighbouring slabs.  Reports
    the step time, and the bytes of the two boundary planes of the 32-value state a slab
    would send per step: they are contiguous in the [z][value][y][x] layout, so they go to
    RCCL without packing."""
    import numpy as np
    from paper_1705_03141_amd import workloads as W

    pb = W.jet(nx=256, ny=256, nz=128, diameter=16.0, u_in=0.04, gamma=1.6, nu_c=1.8e-4, eta=1.0, weber=220.0,
               froude=8.5, noise_rel=0.0, fields=False)
    pb.faces = (W.PERIODIC,) * 6
    pb.inflow = False
    pb.name = "jet_slab_256x256x128"
    y, x = np.mgrid[0:pb.ny, 0:pb.nx]
    inside = ((x - 127.5) ** 2 + (y - 127.5) ** 2 < 64.0)[None].repeat(pb.nz, axis=0)
    pb.rho_r = np.where(inside, pb.rho_r0, 0.0)
    pb.rho_b = np.where(inside, 0.0, pb.rho_b0)
    pb.u = np.zeros((3, pb.nz, pb.ny, pb.nx))
    pb.u[2][inside] = 0.04
    n = pb.ncells
    wall, kernel_ms, diag = run_gpu(pb, "f32", steps, warmup)
    if diag["unstable"]:
        print("bench.py: the slab went unstable", file=sys.stderr)
        sys.exit(1)
    face_bytes = 2 * (27 + 5) * 4 * pb.nx * pb.ny
    line = {"metric": "MLUPS, one z-slab of the jet (8-GPU share)", "value": n * steps / wall / 1e6, "unit": "MLUPS",
            "steps": steps, "warmup": warmup, "ms_per_step": wall * 1e3 / steps, "kernel_ms": kernel_ms,
            "dtype": "f32", "config": {"workload": pb.name, "tile": list(diag["tiling"])},
            "roofline": {"bound": "hbm", "achieved": STD_BYTES * n / (kernel_ms * 1e-3) / 1e9, "peak": PEAK_GBS,
                         "unit": "GB/s", "frac": STD_BYTES * n / (kernel_ms * 1e-3) / 1e9 / PEAK_GBS},
            "halo_bytes_per_step": face_bytes,
            "halo_us_at_153GBps_per_link": face_bytes / 2 / 153e9 * 1e6}
    print(json.dumps(line), flush=True)


def surrogate_bench(steps: int, warmup: int):
    """Training steps (forward, backward, Adam) of the surrogate on one 64 x 64 x 256 coarse
    state; throughput of its convolutions against the dense BF16 MFMA peak (2.5 PFLOP/s)."""
    import numpy as np
    import torch
    from paper_1705_03141_amd import surrogate as S

    n, d, h, w = 1, 256, 64, 64
    net = S.Network(n, d, h, w)
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.normal(size=(n, d, h, w, 4)).astype(np.float32) * 0.5).cuda()
    target = torch.from_numpy(rng.normal(size=(n, d, h, w, 4)).astype(np.float32) * 0.01).cuda()
    for _ in range(warmup):
        net.train_step(x, target)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(x, target, sync_loss=False)  # inputs resident in HBM; loss read once below
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    loss = net.last_loss()
    if not math.isfinite(loss):
        raise SystemExit(f"surrogate training diverged (loss {loss})")
    nv = {"full": n * d * h * w, "half": n * d * h * w // 8, "quarter": n * d * h * w // 64}
    res = {"e1a": "full", "e1b": "full", "e2": "half", "bt": "quarter", "d2": "half", "d1": "full", "out": "full"}
    fwd = sum(2.0 * nv[res[name]] * 27 * cin * cout for name, cin, cout in S.LAYERS)
    flops = 3.0 * fwd - 2.0 * nv["full"] * 27 * 8 * 32  # forward, weight gradient, data gradient (none for e1a)
    tf = flops / dt / 1e12
    print(json.dumps({"metric": "surrogate training step (forward + backward + Adam), 64x64x256x4 input",
                      "value": dt * 1e3, "unit": "ms", "higher_is_better": False, "steps": steps,
                      "conv_tflops": tf, "roofline": {"bound": "mfma", "achieved": tf, "peak": 2500.0,
                                                      "unit": "TFLOP/s", "frac": tf / 2500.0},
                      "dtype": "bf16 MFMA, f32 accumulate"}), flush=True)


def surrogate_sweep(steps: int, train_steps: int = 1500, start: int = 5, ahead: int = 10):
    """The surrogate in the 64-case regime-map sweep (FP16 storage): the lattice runs every
    case for `steps` steps and keeps the 4x-coarsened (phi, u/u_in) every 200 steps in a
    64 x 64 x 256 x 4 box; a 3-member ensemble trains on 48 cases; the other 16 are
    fast-forwarded from snapshot `start` for up to `ahead` horizons while the ensemble's
    predicted interface error stays within one coarse cell, and every accepted prediction is
    scored against plain FP32 lattice runs of those cases.  Reports the surrogate's share of
    the horizons, its interface error against FP32 (and that of the FP16 lattice itself for
    context) and the lattice time it saves."""
    import numpy as np
    import torch
    from paper_1705_03141_amd import metrics
    from paper_1705_03141_amd import surrogate as S
    from paper_1705_03141_amd import workloads as W

    horizon = 200
    snaps = steps // horizon
    cases = W.regime_sweep()
    held = cases[48:]
    log(f"surrogate sweep: {len(cases)} cases, {snaps} snapshots of {horizon} steps (FP16 lattice)")
    states, t16, unstable = S.coarse_trajectories(cases, horizon, snaps, storage="f16",
                                                  progress=lambda m: log(f"surrogate sweep: FP16 lattice: {m}"))
    log(f"surrogate sweep: FP16 lattice {t16:.1f} s; FP32 lattice of the 16 held-out cases")
    truth, t32, _ = S.coarse_trajectories(held, horizon, snaps, storage="f32",
                                          progress=lambda m: log(f"surrogate sweep: FP32 lattice: {m}"))
    train = [k for k in range(48) if k not in unstable]
    ens = S.Ensemble(batch=4, members=3, seed=0)
    t0 = time.perf_counter()
    losses = ens.train(states, cases=train, steps=train_steps)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log(f"surrogate sweep: ensemble trained in {t_train:.1f} s, losses {losses}")
    ext = [S.coarse_extent(pb) for pb in held]
    rep = S.fast_forward(ens, states[:, 48:], truth, list(range(16)), ext, start=start, horizons=ahead)
    cells = np.array([pb.ncells for pb in cases], dtype=float)
    t_case = t16 / snaps * cells[48:] / cells.sum()
    x = states[start, 48:49]
    ens.predict(x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(10):
        ens.predict(x)
    torch.cuda.synchronize()
    t_pred = (time.perf_counter() - t1) / 10
    acc = [a for r in rep.values() for a in r["actual"]]
    taken = sum(r["taken"] for r in rep.values())
    saved = sum(r["taken"] * (t_case[k] - t_pred) for k, r in rep.items())
    lattice_total = float(t_case.sum()) * ahead
    fp16_err = []
    for k, (d, h, w) in enumerate(ext):
        for s_ in range(start + 1, start + ahead + 1):
            fp16_err.append(S.interface_error_coarse(states[s_, 48 + k, :d, :h, :w, 0].cpu().numpy(),
                                                     truth[s_, k, :d, :h, :w, 0].cpu().numpy()))
    print(json.dumps({
        "metric": "surrogate fast-forward of the 64-case regime-map sweep",
        "cases": {"train": len(train), "held_out": 16, "unstable": unstable},
        "input": list(S.BOX) + [4], "horizon_steps": horizon, "snapshots": snaps, "start_step": start * horizon,
        "horizons_by_surrogate": taken, "horizons_offered": 16 * ahead,
        "interface_error_vs_fp32_coarse_cells": {"mean": float(np.mean(acc)) if acc else None,
                                                 "max": float(np.max(acc)) if acc else None},
        "fp16_lattice_interface_error_vs_fp32_coarse_cells": {"mean": float(np.mean(fp16_err)),
                                                              "max": float(np.max(fp16_err))},
        "rejected": [{"case": k, **r["rejected"]} for k, r in rep.items() if r["rejected"]],
        "ms_per_horizon": {"lattice_per_case_mean": float(t_case.mean() * 1e3), "ensemble_prediction": t_pred * 1e3},
        "lattice_seconds_saved": saved, "lattice_seconds_of_the_window": lattice_total,
        "train_seconds": t_train, "member_losses": losses}), flush=True)


def interface_error(workload: str, steps: int):
    """Interface-position error of FP16 / BF16 storage against FP32 storage after `steps`
    steps (metrics.interface_position_error; lattice units).  The control "f32_perturbed" is
    an FP32 run whose initial red density differs by a relative 1e-6 (eight FP32 units in the
    last place) in one cell on the seeded interface (for the jet, which starts without red
    fluid, the blue density of the axis cell above the inlet): what the flow itself makes of
    a rounding-sized difference, the floor any storage format is measured against."""
    import copy

    import numpy as np
    from paper_1705_03141_amd import lbm, metrics
    from paper_1705_03141_amd import workloads as W

    pb = W.cfg_rayleigh_taylor() if workload == "rt" else W.cfg_jet()
    ctrl = copy.copy(pb)
    k = pb.nx // 2
    if pb.rho_r.any():
        # the cell of the column through the middle where the red fraction is nearest 1/2
        ctrl.rho_r = pb.rho_r.copy()
        col = pb.rho_r[:, k, k] / (pb.rho_r[:, k, k] + pb.rho_b[:, k, k])
        ctrl.rho_r[int(np.argmin(np.abs(col - 0.5))), k, k] *= 1.0 + 1e-6
    else:
        # no red fluid at t = 0 (the jet): the blue cell on the axis one plane above the inlet
        ctrl.rho_b = pb.rho_b.copy()
        ctrl.rho_b[1, k, k] *= 1.0 + 1e-6
    phi = {}
    for st, prob in (("f32", pb), ("f32_perturbed", ctrl), ("f16", pb), ("bf16", pb)):
        lat = lbm.Lattice(prob, storage=st.split("_")[0])
        done = 0
        while done < steps:
            k = min(2000, steps - done)
            lat.step(k)
            lat.sync()
            done += k
            log(f"{pb.name} {st}: {done}/{steps} steps")
        phi[st] = lat.field("phi")
        if lat.diagnostics()["unstable"]:
            log(f"{pb.name} {st}: unstable")
        lat.close()
    out = {"workload": pb.name, "steps": steps}
    for st in ("f32_perturbed", "f16", "bf16"):
        out[st] = metrics.interface_position_error(phi[st], phi["f32"])
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--sweep-storage", default="f16", choices=["f32", "f16", "bf16"],
                    help="population storage of --sweep (the sweep is specified in FP16)")
    ap.add_argument("--workload", default="jet", choices=["rt", "jet", "jet_walls"],
                    help="jet: the liquid jet 256 x 256 x 1024 (the default); rt: Rayleigh-Taylor 128 x 128 x 512; "
                         "jet_walls: the jet between free-slip lateral walls")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP16/BF16-storage runs")
    ap.add_argument("--autotune", action="store_true",
                    help="time the tile shapes first (lbm_autotune) instead of using the default 64 x 4")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead: time the 64-case regime-map sweep of uneven jets in one batch (FP16 storage)")
    ap.add_argument("--slab", action="store_true",
                    help="instead: time one GPU's z-slab (256 x 256 x 128) of the jet split over 8 GPUs")
    ap.add_argument("--surrogate", action="store_true",
                    help="instead: time training steps of the surrogate network on the 64 x 64 x 256 x 4 input")
    ap.add_argument("--surrogate-sweep", action="store_true",
                    help="instead: train the surrogate ensemble on the 64-case sweep's trajectories (--steps lattice "
                         "steps) and fast-forward 16 held-out cases with it")
    ap.add_argument("--interface-error", choices=["rt", "jet"],
                    help="instead of timing: run the workload for --steps steps with FP32, FP16 and BF16 "
                         "storage and print the interface-position error of the half-precision runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design only)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.interface_error:
        interface_error(args.interface_error, args.steps)
        return
    if args.sweep:
        sweep(args.steps, args.warmup, args.sweep_storage)
        return
    if args.surrogate:
        surrogate_bench(args.steps, args.warmup)
        return
    if args.surrogate_sweep:
        surrogate_sweep(args.steps)
        return
    if args.slab:
        slab_bench(args.steps, args.warmup)
        return

    from paper_1705_03141_amd import workloads as W

    pb = {"rt": W.cfg_rayleigh_taylor, "jet": W.cfg_jet, "jet_walls": W.cfg_jet_walls}[args.workload]()
    n = pb.ncells
    log(f"{pb.name} {pb.nx}x{pb.ny}x{pb.nz}, storage {args.storage}, {args.warmup}+{args.steps} steps")
    wall, kernel_ms, diag = run_gpu(pb, args.storage, args.steps, args.warmup, args.autotune)
    log(f"{wall * 1e3 / args.steps:.3f} ms/step wall, kernel {kernel_ms:.3f} ms, tiling {diag['tiling']}")
    if diag["unstable"]:
        print("bench.py: the run went unstable", file=sys.stderr)
        sys.exit(1)
    mlups = n * args.steps / wall / 1e6
    # the standard traffic of the method at the storage width: 2 x 27 populations of 4 B
    # (FP32) or 2 B (FP16/BF16), read and written once per update
    std_bytes = STD_BYTES if args.storage == "f32" else STD_BYTES / 2.0
    achieved = std_bytes * n / (kernel_ms * 1e-3) / 1e9
    extra = {"kernel_ms": kernel_ms, "state_bytes_per_update": state_bytes(args.storage),
             "state_traffic_frac": state_bytes(args.storage) * n / (kernel_ms * 1e-3) / 1e9 / PEAK_GBS}
    for st in ("f16", "bf16"):
        if st != args.storage and not args.no_extra:
            w2, k2, _ = run_gpu(pb, st, max(args.steps // 2, 10), args.warmup, args.autotune)
            log(f"storage {st}: kernel {k2:.3f} ms")
            extra[f"{st}_mlups"] = n * max(args.steps // 2, 10) / w2 / 1e6
    traffic = measured_traffic(args.storage, diag["tiling"], pb.name)
    if traffic is not None:  # HBM bytes the counters saw, over the same kernel time
        extra["measured_hbm_gbs"] = traffic / (kernel_ms * 1e-3) / 1e9
        extra["measured_hbm_frac"] = extra["measured_hbm_gbs"] / PEAK_GBS
    line = {
        "metric": "MLUPS (D3Q27 two-component) and % of HBM roofline; FP16-store vs FP32 at fixed error",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"f32 compute, {args.storage} storage",
        "data": "synthetic",
        "config": {"workload": pb.name, "nx": pb.nx, "ny": pb.ny, "nz": pb.nz, "storage": args.storage,
                   "tile": list(diag["tiling"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_GBS, "traffic": traffic,
                     "basis": f"{std_bytes:.0f} B per cell update (2 x 27 "
                              f"{'FP32' if args.storage == 'f32' else '16-bit'} populations read and written) "
                              "x cells / mean step-kernel time"},
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        line["cpu_baseline"] = cpu_baseline(pb)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
