"""Benchmark of the two-component colour-gradient LB step on one MI355X.

Default workload: the D3Q27 channel (256x128x128, no-slip y/z walls, body
force 1e-6 along x, 64 droplets R=10 at seeded random centres, near-contact
range 3 / strength 0.02, tau 1, FP32 storage and arithmetic).  A step is one
pass of the whole hot path (phase-field pass + collision pass) over the
lattice, with the populations already resident in HBM.

Prints ONE JSON line: MLUPS (million lattice-site updates per second), the
roofline of the dominant kernel (the collision pass) from HIP events recorded
on the library's stream around each launch, and the FP64 CPU oracle timed on
a bounded crop of the same physics.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS & % HBM roofline, 2-comp D3Q27; FP16-store/learned vs plain FP32"
ELEM = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "f32t": 4, "f16t": 2, "bf16t": 2, "f16ct": 2, "f32s": 4}
TOTAL = ("f32t", "f16t", "bf16t", "f16ct")
NSC_BYTES = 16  # recolouring scalars of the total layout, per site


def algorithmic_bytes(q, storage):
    """Per lattice update of the layout in use: (step, collision pass, phase
    pass).  Step: the state read once and written once, plus the phase field
    written once (pass 1) and read once (pass 2); the plain per-colour FP32
    D3Q27 step is 440 B.  Phase pass: state read + phase written.  Collision
    pass: populations read + state written + phase read (per-colour: the
    whole state both ways; total layout: the scalars are written, not read,
    since rho_A follows from phi)."""
    s = ELEM[storage]
    r = 8 if storage == "f64" else 4
    if storage in TOTAL:
        state = q * s + NSC_BYTES
        return 2 * state + 2 * r, 2 * q * s + NSC_BYTES + r, state + r
    state = 2 * q * s
    return 2 * state + 2 * r, 2 * state + r, state + r


def plain_state_bytes(q, storage):
    """Algorithmic bytes of the two-colour state at this precision (per-colour
    populations read and written once, phase field once each way): the
    reference definition the step roofline is quoted against."""
    s = ELEM[storage]
    r = 8 if storage == "f64" else 4
    return 2 * q * s * 2 + 2 * r


def kernel_source_hash():
    """Hash of the sources that fix the passes' code and launch shapes (the
    kernels and their launch wrappers): a traffic figure measured for other
    sources is not reported."""
    import hashlib
    h = hashlib.sha256()
    for name in ("step_kernels.hpp", "lattice_ops.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2405_14551_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag, workload_tag):
    """HBM bytes per launch measured with rocprofv3 counters, if a summary for
    this kernel source is committed (profiles/traffic_<kernel>_<workload>.txt
    holds key = value lines incl. the source hash); None otherwise."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}_{workload_tag}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = kernel_source_hash()
    if kv.get("source_hash") != h or "bytes_per_launch" not in kv:
        return None
    return float(kv["bytes_per_launch"])


def cpu_baseline(seconds_target=10.0):
    """The FP64 oracle, single-threaded, on a 64^3 crop of the channel physics
    (walls y/z, body force, near contact, 4 droplets R=10)."""
    from threadpoolctl import threadpool_limits
    from oracle.sim import OracleSim, OracleParams
    from paper_2405_14551_amd import workloads as W
    shape = (64, 64, 64)
    w = W.channel_3d(shape=shape, count=4, radius=10.0)
    p = OracleParams(lattice="D3Q27", nx=64, ny=64, nz=64, walls=(False, True, True), tau=1.0,
                     A=0.01, beta=0.7, body_force=(1e-6, 0, 0), nc=True, nc_A=0.02,
                     nc_hmin=2.0, nc_hmax=3.0)
    with threadpool_limits(1):
        sim = OracleSim(p).init_droplets(w["centres"], w["radii"])
        steps = 0
        t0 = time.perf_counter()
        while True:
            sim.step(1)
            steps += 1
            el = time.perf_counter() - t0
            if el >= seconds_target or steps >= 50:
                break
    n = shape[0] * shape[1] * shape[2]
    return {"value": n * steps / el / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 numpy oracle, 1 thread, 64x64x64 crop of the channel physics "
                      f"(walls y/z, force 1e-6, near contact on, 4 droplets R=10), {steps} steps "
                      f"in {el:.1f} s on {platform.processor() or platform.machine()} "
                      f"(host nproc {os.cpu_count()})"}


def time_storage(kw, cen, rad, storage, steps, warmup, streaming="two_copies", scheme="populations",
                 rounding="nearest"):
    """MLUPS and per-launch pass times of the same workload with another
    storage layout or streaming (HIP events on the library's stream), and the
    device memory the population state takes per site (both copies with
    two-copy streaming)."""
    import torch
    from paper_2405_14551_amd import lb
    sim = lb.Simulation(**dict(kw, storage=storage, streaming=streaming, scheme=scheme,
                               rounding=rounding)).init_droplets(cen, rad)
    copies = 1 if streaming == "in_place" else 2
    state_per_site = copies * sim.state_bytes() / (kw["shape"][0] * kw["shape"][1] * kw["shape"][2])
    sim.step(warmup)
    sim.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sim.profile_begin()
    with torch.cuda.stream(sim.stream):
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
    prof = sim.profile_end()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nx, ny, nz = kw["shape"]
    sim.close()
    return {"MLUPS": round(nx * ny * nz * steps / (ms / 1e3) / 1e6, 1),
            "collide_ms": round(prof["ms_collide"] / max(prof["n_collide"], 1), 5),
            "phase_ms": round(prof["ms_phase"] / max(prof["n_phase"], 1), 5),
            "state_bytes_per_site": round(state_per_site, 1)}


def time_closure(kw, cen, rad, steps, warmup, explicit):
    """The learned near-contact closure on the same workload: rows collected
    after the warm-up with the explicit force, 500 Adam steps, then the step
    with the closure in the collision pass.  Reports its collision-pass time
    beside the explicit one and the share of interface sites the network
    served."""
    import torch
    from paper_2405_14551_amd import lb, workloads as W
    src = lb.Simulation(**dict(kw, nc="explicit")).init_droplets(cen, rad)
    src.step(warmup)
    rows, tg, na, nf = src.nc_collect()
    src.close()
    tr = lb.Simulation(lattice=kw["lattice"], storage="f32", nc="explicit", shape=(16, 16, 16))
    tr.mlp_set_weights(W.closure_init_weights())
    tr.mlp_train(rows, tg, torch.from_numpy(W.closure_batches(na, nf, 500, 256)), lr=2e-3)
    th, ranges = tr.mlp_get_weights(), tr.mlp_get_ranges()
    tr.close()
    sim = lb.Simulation(**dict(kw, nc="mlp"))
    sim.mlp_set_weights(th)
    sim.mlp_set_ranges(*ranges)
    sim.init_droplets(cen, rad)
    sim.step(warmup)
    sim.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sim.profile_begin()
    with torch.cuda.stream(sim.stream):
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
    prof = sim.profile_end()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    fl = sim.fields(("flags",))["flags"]
    n_if = int(((fl & 1) > 0).sum())
    n_net = int(((fl & 2) > 0).sum())
    nx, ny, nz = kw["shape"]
    sim.close()
    col = prof["ms_collide"] / max(prof["n_collide"], 1)
    return {"MLUPS": round(nx * ny * nz * steps / (ms / 1e3) / 1e6, 1), "collide_ms": round(col, 5),
            "explicit_collide_ms": explicit, "collide_time_vs_explicit": round(col / explicit, 3),
            "training_rows": {"active": na, "free": nf}, "interface_sites": n_if,
            "network_share": round(n_net / max(n_if, 1), 4)}


def ensemble_bench(args):
    """Batched ensemble of 96 independent D3Q19 channels (sizes 64..160 x
    64..96 x 64..96, tau 0.6..1.2, 4..40 droplets each; FP32, near contact):
    autotuned launch configuration, aggregate MLUPS, the collision launch's
    roofline, and the same channels run one after another as stand-alone
    simulations."""
    import torch
    from paper_2405_14551_amd import lb, workloads as W
    w = W.ensemble_channels()
    chans = w["channels"]
    N = int(sum(np.prod(c["shape"]) for c in chans))
    plain = [{k: v for k, v in c.items() if k not in ("centres", "radii")} for c in chans]
    ens = lb.Ensemble(plain, lattice=w["lattice"], storage=w["storage"], nc=w["nc"])
    for k, c in enumerate(chans):
        ens.init_droplets(k, c["centres"], c["radii"])
    best, table = ens.autotune(steps=4)
    print(f"# ensemble autotune best {best}", file=sys.stderr, flush=True)
    for k, c in enumerate(chans):      # restart from the initial state after tuning
        ens.init_droplets(k, c["centres"], c["radii"])
    ens.step(args.warmup)
    ens.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(ens.stream):
        e0.record(ens.stream)
        ens.step(args.steps)
        e1.record(ens.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof_steps = 20
    ens.profile_begin()
    ens.step(prof_steps)
    prof = ens.profile_end()
    ens.sync()
    # collision and phase time per step: one launch each in the batched mode,
    # one per channel in the per-channel mode
    col_ms = prof["ms_collide"] / prof_steps
    ph_ms = prof["ms_phase"] / prof_steps
    launches = max(prof["n_collide"], 1) // prof_steps
    ens.close()
    q = 19
    b_step, b_col, b_phase = algorithmic_bytes(q, "f32")
    mlups = N * args.steps / (ms / 1e3) / 1e6
    achieved = b_col * N / (col_ms / 1e3) / 1e9
    # stand-alone runs of the same channels, one after another
    sa_steps = min(args.steps, 50)
    t_sum = 0.0
    for c in chans:
        kw = dict(c)
        cen, rad = kw.pop("centres"), kw.pop("radii")
        sim = lb.Simulation(lattice=w["lattice"], storage=w["storage"], nc=w["nc"], **kw).init_droplets(cen, rad)
        sim.step(5)
        sim.sync()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(sim.stream):
            a0.record(sim.stream)
            sim.step(sa_steps)
            a1.record(sim.stream)
        torch.cuda.synchronize()
        t_sum += a0.elapsed_time(a1)
        sim.close()
    sa_mlups = N * sa_steps / (t_sum / 1e3) / 1e6
    out = {
        "metric": "MLUPS (aggregate over the ensemble)", "value": round(mlups, 2), "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded channel sizes, tau and droplet placement)",
        "config": {"workload": "ensemble_96_d3q19", "channels": len(chans), "sites": N, "lattice": "D3Q19",
                   "storage": "f32", "near_contact": "explicit", "tuning": best},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "ensemble collision launch" if best["mode"] == "batched" else "per-channel collision launches",
                     "bytes_per_site": b_col, "avg_launch_ms": round(col_ms, 5),
                     "launches_per_step": launches},
        "step_roofline": {"bytes_per_site": b_step, "frac": round(mlups * 1e6 * b_step / 1e9 / HBM_PEAK_GBS, 4),
                          "phase_launch_ms": round(ph_ms, 5)},
        "standalone": {"MLUPS": round(sa_mlups, 1), "steps": sa_steps,
                       "note": "the 96 channels as separate simulations, one after another"},
        "autotune_table": table,
    }
    print(json.dumps(out), flush=True)
    return 0


def copy_calibration(nbytes=1 << 30, reps=10):
    """A plain device-to-device copy of known size: rocprofv3 FETCH_SIZE /
    WRITE_SIZE of these launches give the counter scale (ideal: nbytes each)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_bytes_each_way": nbytes, "reps": reps,
                      "GBps_read_plus_write": 2 * nbytes * reps / dt / 1e9}), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--workload", default="channel_3d", choices=["channel_3d", "big_3d", "dense_3d", "ensemble"])
    ap.add_argument("--storage", default=None, help="f32 (default), f16, bf16, f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the 16-bit storage and learned-closure variants")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (to scale HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU slab "
                                   "decomposition is not part of this build", "n_gpus": args.gpus}))
        return 2

    import torch
    from paper_2405_14551_amd import lb, workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    if args.workload == "ensemble":
        return ensemble_bench(args)
    wl = {"channel_3d": W.channel_3d, "big_3d": W.big_3d, "dense_3d": W.dense_3d}[args.workload]
    w = wl(storage=args.storage) if args.storage else wl()
    if args.storage:
        w["storage"] = args.storage
    kw, cen, rad = W.sim_kwargs(w)
    storage = kw["storage"]
    print(f"# workload {args.workload} storage {storage} shape {kw['shape']}", file=sys.stderr, flush=True)
    sim = lb.Simulation(**kw)
    sim.init_droplets(cen, rad)
    nx, ny, nz = kw["shape"]
    N = nx * ny * nz
    q = sim.q
    sim.step(args.warmup)
    sim.sync()
    stream = sim.stream
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    sim.profile_begin()
    with torch.cuda.stream(stream):
        t_start.record(stream)
        sim.step(args.steps)
        t_end.record(stream)
    prof = sim.profile_end()
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    ms_per_step = ms / args.steps
    mlups = N * args.steps / (ms / 1e3) / 1e6
    b_step, b_col, b_phase = algorithmic_bytes(q, storage)
    col_ms = prof["ms_collide"] / max(prof["n_collide"], 1)
    ph_ms = prof["ms_phase"] / max(prof["n_phase"], 1)
    achieved = b_col * N / (col_ms / 1e3) / 1e9
    traffic = traffic_from_profiles("collide", f"{args.workload}_{storage}")
    diag = sim.diagnostics()
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if storage == "f64" else "f32",
        "data": "synthetic (seeded droplet placement)",
        "config": {"workload": args.workload, "lattice": kw["lattice"], "storage": storage,
                   "shape": list(kw["shape"]), "walls": list(kw["walls"]), "droplets": int(len(rad)),
                   "near_contact": kw["nc"], "sites": N},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_vs_algorithmic": (round(traffic / (b_col * N), 3) if traffic else None),
                     "kernel": "k_collide (collision pass)",
                     "bytes_per_site": b_col, "avg_launch_ms": round(col_ms, 5)},
        "step_roofline": {"bytes_per_site": b_step, "frac": round(mlups * 1e6 * b_step / 1e9 / HBM_PEAK_GBS, 4),
                          "plain_state_bytes_per_site": plain_state_bytes(q, storage),
                          "frac_vs_plain_state": round(mlups * 1e6 * plain_state_bytes(q, storage) / 1e9
                                                       / HBM_PEAK_GBS, 4),
                          "phase_pass_ms": round(ph_ms, 5), "phase_pass_GBs": round(b_phase * N / (ph_ms / 1e3) / 1e9, 1)},
        "sanity": {"droplets_end": int(diag[6]), "umax": float(diag[5])},
    }
    sim.close()
    if not args.no_variants and storage == "f32":
        # same workload: total-population layouts (FP32 / FP16 / BF16 storage,
        # FP32 arithmetic), in-place streaming (one copy of the state) and the
        # learned near-contact closure
        vs = min(args.steps, 200)
        var = {}
        for st, mode in (("f32t", "two_copies"), ("f16t", "two_copies"), ("bf16t", "two_copies"),
                         ("f16ct", "two_copies"), ("f32", "in_place"), ("f16t", "in_place")):
            name = st if mode == "two_copies" else f"{st}_in_place"
            var[name] = time_storage(kw, cen, rad, st, vs, args.warmup, mode)
            var[name]["vs_plain_f32"] = round(var[name]["MLUPS"] / mlups, 3)
            print(f"# variant {name}: {var[name]}", file=sys.stderr, flush=True)
        # FP16 total layout with stochastic rounding of the stored totals
        var["f16t_sround"] = time_storage(kw, cen, rad, "f16t", vs, args.warmup, rounding="stochastic")
        var["f16t_sround"]["vs_plain_f32"] = round(var["f16t_sround"]["MLUPS"] / mlups, 3)
        print(f"# variant f16t_sround: {var['f16t_sround']}", file=sys.stderr, flush=True)
        # the moment-based (regularised) scheme: 15 moments per site
        var["moments_f32"] = time_storage(kw, cen, rad, "f32", vs, args.warmup, scheme="moments")
        var["moments_f32"]["vs_plain_f32"] = round(var["moments_f32"]["MLUPS"] / mlups, 3)
        print(f"# variant moments_f32: {var['moments_f32']}", file=sys.stderr, flush=True)
        if kw.get("nc") == "explicit":
            var["closure_f32"] = time_closure(kw, cen, rad, vs, args.warmup, col_ms)
            print(f"# variant closure: {var['closure_f32']}", file=sys.stderr, flush=True)
        out["variants"] = var
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
