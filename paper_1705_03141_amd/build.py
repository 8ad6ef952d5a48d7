"""Build of the HIP library ``liblbm.so`` (gfx950) from ``csrc/``.

The kernels of each population storage type are compiled as separate translation units in
parallel, then linked with the host side of the C ABI into one shared library placed next
to this file.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblbm.so")
BUILD = os.path.join(HERE, "_build")
UNITS = ["lbm_storage_f32.hip", "lbm_storage_f16.hip", "lbm_storage_bf16.hip", "lbm_dispatch.hip", "lbm_capi.hip",
         "surr_ops.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")
# Packed FP32 instructions are disabled: the compiler still vectorises plain float code.
# FMA contraction is decided per source expression (-ffp-contract=on): every inlined copy of
# a function then rounds identically, which keeps results independent of the tiling.
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-ffp-contract=on", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]


# The step kernels are scheduled for instruction-level parallelism: with two waves per SIMD the
# default occupancy-oriented schedule leaves more of the LDS and memory latency exposed.
UNIT_FLAGS = {u: ["-mllvm", "-amdgpu-sched-strategy=max-ilp"] for u in UNITS if u.startswith("lbm_storage_")}


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return path


def sources():
    return [os.path.join(CSRC, u) for u in UNITS]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc()] + FLAGS + UNIT_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(UNITS), max(1, (os.cpu_count() or 4)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, sources()))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps += [os.path.join(INCLUDE, "lbm.h"), os.path.join(INCLUDE, "surrogate.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    build()
