"""Address and undefined-behaviour sanitizer builds (CPU, no GPU needed).

* the FP64 oracle, built with gcc -fsanitize=address,undefined, runs every code path
  (oracle/sanitize_driver.c: all face rules, inflow with noise, outflow, body force, user and
  default rates, windows, read-back);
* the host side of the HIP library, its host units (the C ABI, the storage dispatch and the
  surrogate's operators) built with the sanitizers applied to the host code only
  (-Xarch_host), linked with tests/sanitize_host_driver.cpp and with the kernel units of the
  library's own build (device code and launch stubs, whose host side holds no logic), runs
  its host-only paths (validation, surface-tension conversions, the host-compiled collision,
  tile sets, NULLs).
Any sanitizer report fails the run (recovery off).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"), "-o", exe,
          os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-lm"])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "jet: inflow disk" in r.stdout and "ERROR" not in r.stderr


def test_host_library_under_address_and_undefined_sanitizers(tmp_path):
    from paper_1705_03141_amd import build as B

    if not shutil.which("hipcc") and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    # the kernel units come from the library's build (compiling their device code again
    # would take most of this test's time and instruments nothing of interest)
    kernel_units = [u for u in B.UNITS if u.startswith("lbm_storage_")]
    kernel_objs = [os.path.join(B.BUILD, u + ".o") for u in kernel_units]
    if B.stale() or not all(os.path.exists(o) for o in kernel_objs):
        B.build(verbose=False)
    objs = list(kernel_objs)
    procs = []
    for src in B.sources():
        if os.path.basename(src) in kernel_units:
            continue
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1"]
        procs.append(subprocess.Popen([B.hipcc()] + flags + san + ["-c", src, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for pr in procs:
        out, err = pr.communicate(timeout=900)
        assert pr.returncode == 0, err[-3000:]
    drv = str(tmp_path / "sanitize_host_driver.o")
    _run([B.hipcc(), f"--offload-arch={B.ARCH}", "-std=c++17", "-O1", f"-I{B.INCLUDE}"] + san +
         ["-c", os.path.join(ROOT, "tests", "sanitize_host_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "host_san")
    _run([B.hipcc(), f"--offload-arch={B.ARCH}"] + san + ["-o", exe, drv] + objs)
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "0 failures" in r.stdout
