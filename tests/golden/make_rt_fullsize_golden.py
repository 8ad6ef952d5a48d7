"""Writes rt128x128x512_1000steps_planes.npz: the FP64 oracle's fields on four z planes of
the full-size Rayleigh-Taylor workload (128 x 128 x 512, At 0.5, g 1e-5, Re 256, seeded
1e-4 density noise; Sec. III C set-up) after 1000 steps.

Planes: the lower wall plane z = 0 and three planes through the perturbed interface
(z = 250, 255, 261; the interface spans z = 243..268).  Fields: rho_r, rho_b, ux, uy, uz,
stored as float32 (rounding 6e-8 relative, far below the 1e-5 parity bar).

Calls only the oracle.  About 20-30 minutes on 8 host cores and 12 GB of memory:
    python tests/golden/make_rt_fullsize_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1705_03141_amd import workloads as W  # noqa: E402

PLANES = (0, 250, 255, 261)
STEPS = 1000
OUT = os.path.join(HERE, "rt128x128x512_1000steps_planes.npz")


def main():
    pb = W.cfg_rayleigh_taylor()
    o = oracle.Oracle(pb)
    t0 = time.time()
    for k in range(0, STEPS, 50):
        o.step(50)
        print(f"step {k + 50}/{STEPS}, {time.time() - t0:.0f} s", flush=True)
    f = o.fields()
    z = np.array(PLANES)
    np.savez(OUT, planes=z, steps=np.array(STEPS), rho_r=f["rho_r"][z].astype(np.float32),
             rho_b=f["rho_b"][z].astype(np.float32), u=f["u"][:, z].astype(np.float32),
             max_rho=np.array(float(f["rho"].max())), max_u=np.array(float(np.abs(f["u"]).max())))
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
