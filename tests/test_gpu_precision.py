"""Error statement of the storage precisions against the FP64 oracle.

The 64^3 crop of the 512x256x256 / 1024-droplet workload (walls y/z, body
force, near contact) runs with FP32, shifted FP16 and shifted BF16 storage
(FP32 arithmetic in all three) beside the FP64 oracle.  The paper gives no
accuracy bound for 16-bit storage, so these numbers are a measured statement
("parity unpinned"); the test asserts only what must hold at any precision
(finite fields, FP32 close to FP64, per-colour mass to storage rounding) and
records the errors.  LB_PRECISION_STEPS sets the step count (default 200);
LB_PRECISION_OUT names a directory for a JSON copy of the report."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402
from oracle.sim import OracleSim, OracleParams  # noqa: E402

STEPS = int(os.environ.get("LB_PRECISION_STEPS", "200"))


def test_storage_precision_vs_fp64_oracle():
    w = W.big_3d_crop()
    kw, cen, rad = W.sim_kwargs(w)
    nx, ny, nz = kw["shape"]
    print(f"case precision crop {kw['shape']} droplets {len(rad)} steps {STEPS}", flush=True)
    p = OracleParams(lattice="D3Q27", nx=nx, ny=ny, nz=nz, walls=(False, True, True), tau=kw["tau"],
                     A=kw["A"], beta=kw["beta"], body_force=tuple(kw["body_force"]), nc=True,
                     nc_A=kw["nc_A"], nc_hmin=kw["nc_hmin"], nc_hmax=kw["nc_hmax"])
    orc = OracleSim(p).init_droplets(cen, rad)
    done = 0
    while done < STEPS:
        k = min(50, STEPS - done)
        orc.step(k)
        done += k
        print(f"  oracle step {done}/{STEPS}", flush=True)
    of = orc.fields()
    od = orc.diagnostics()
    umax = np.sqrt((of["u"] ** 2).sum(0)).max()
    report = {"steps": STEPS, "shape": [nx, ny, nz], "droplets": int(len(rad)),
              "oracle": {"umax": float(umax), "laplace_dp": float(od[7]), "count": int(od[6])}}
    runs = [(st, st, "nearest") for st in ("f32", "f32s", "f16", "bf16", "f32t", "f16t", "bf16t", "f16ct")]
    runs += [("f16t_sround", "f16t", "stochastic"), ("bf16t_sround", "bf16t", "stochastic")]
    for name, st, rounding in runs:
        kw2 = dict(kw, storage=st, rounding=rounding)
        sim = lb.Simulation(**kw2).init_droplets(cen, rad)
        d0 = sim.diagnostics()
        sim.step(STEPS)
        g = {k: v.double().cpu().numpy() for k, v in sim.fields(("rho_a", "rho_b", "phi", "u")).items()}
        d = sim.diagnostics()
        sim.close()
        for k in g:
            assert np.isfinite(g[k]).all(), (name, k)
        e = {
            "rho_a": float(np.abs(g["rho_a"] - of["rho_a"]).max() / np.abs(of["rho_a"]).max()),
            "rho_b": float(np.abs(g["rho_b"] - of["rho_b"]).max() / np.abs(of["rho_b"]).max()),
            "u": float(np.abs(g["u"] - of["u"]).max() / umax),
            "u_rms": float(np.sqrt(((g["u"] - of["u"]) ** 2).mean()) / np.sqrt((of["u"] ** 2).mean())),
            "phi": float(np.abs(g["phi"] - of["phi"]).max()),
            "laplace_dp_rel": float(abs(d[7] - od[7]) / abs(od[7])),
            "count": int(d[6]),
            "mass_drift_a": float(abs(d[0] - d0[0]) / d0[0]),
            "mass_drift_b": float(abs(d[1] - d0[1]) / d0[1]),
        }
        report[name] = e
        print(f"  {name}: {json.dumps(e)}", flush=True)
    # the moment-based scheme in FP32 against its own FP64 definition
    from oracle.llb import OracleLLB
    lorc = OracleLLB(p).init_droplets(cen, rad)
    done = 0
    while done < STEPS:
        k = min(50, STEPS - done)
        lorc.step(k)
        done += k
        print(f"  moment oracle step {done}/{STEPS}", flush=True)
    lf = lorc.fields()
    lumax = np.sqrt((lf["u"] ** 2).sum(0)).max()
    sim = lb.Simulation(**dict(kw, storage="f32", scheme="moments")).init_droplets(cen, rad)
    d0 = sim.diagnostics()
    sim.step(STEPS)
    g = {k: v.double().cpu().numpy() for k, v in sim.fields(("rho_a", "rho_b", "phi", "u")).items()}
    d = sim.diagnostics()
    sim.close()
    report["moments_f32"] = {
        "rho_a": float(np.abs(g["rho_a"] - lf["rho_a"]).max() / np.abs(lf["rho_a"]).max()),
        "u": float(np.abs(g["u"] - lf["u"]).max() / lumax),
        "u_rms": float(np.sqrt(((g["u"] - lf["u"]) ** 2).mean()) / np.sqrt((lf["u"] ** 2).mean())),
        "laplace_dp_rel": float(abs(d[7] - lorc.diagnostics()[7]) / abs(lorc.diagnostics()[7])),
        "count": int(d[6]),
        "mass_drift_a": float(abs(d[0] - d0[0]) / d0[0]),
    }
    print(f"  moments_f32 (vs the FP64 moment oracle): {json.dumps(report['moments_f32'])}", flush=True)
    assert report["moments_f32"]["rho_a"] < 1e-4 and report["moments_f32"]["u"] < 1e-2
    out = os.environ.get("LB_PRECISION_OUT")
    if out and os.path.isdir(out):
        with open(os.path.join(out, f"precision_crop_{STEPS}.json"), "w") as fh:
            json.dump(report, fh, indent=1)
    assert report["f32"]["rho_a"] < 1e-4 and report["f32"]["u"] < 1e-2
    assert report["f32"]["count"] == report["oracle"]["count"]
    sys.stdout.flush()
