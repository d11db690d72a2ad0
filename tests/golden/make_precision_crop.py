"""Write tests/golden/precision_crop_1000.npz: the FP64 oracle's state after
1000 steps of the 64^3 crop of the 512x256x256 / 1024-droplet workload
(D3Q27, walls y/z, body force, near contact; the crop of
``workloads.big_3d_crop``), for the 16-bit storage bar of
tests/test_gpu_precision.py.  Calls the oracle only; takes about 15 minutes on
one core.  Run from the repository root:

    python tests/golden/make_precision_crop.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.sim import OracleSim, OracleParams  # noqa: E402
from paper_2405_14551_amd import workloads as W  # noqa: E402

STEPS = 1000
OUT = os.path.join(ROOT, "tests", "golden", "precision_crop_1000.npz")


def main():
    w = W.big_3d_crop()
    kw, cen, rad = W.sim_kwargs(w)
    nx, ny, nz = kw["shape"]
    p = OracleParams(lattice="D3Q27", nx=nx, ny=ny, nz=nz, walls=(False, True, True), tau=kw["tau"],
                     A=kw["A"], beta=kw["beta"], body_force=tuple(kw["body_force"]), nc=True,
                     nc_A=kw["nc_A"], nc_hmin=kw["nc_hmin"], nc_hmax=kw["nc_hmax"])
    orc = OracleSim(p).init_droplets(cen, rad)
    t0 = time.time()
    for k in range(STEPS // 50):
        orc.step(50)
        print(f"oracle step {50 * (k + 1)}/{STEPS} ({time.time() - t0:.0f} s)", flush=True)
    f = orc.fields()
    d = orc.diagnostics()
    np.savez_compressed(OUT, steps=STEPS, shape=np.array([nx, ny, nz]), centres=cen, radii=rad,
                        u=f["u"].astype(np.float32), umax=np.sqrt((f["u"] ** 2).sum(0)).max(),
                        count=int(d[6]), laplace_dp=d[7], mass=np.array(orc.mass()))
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
