"""Benchmark of the two-component colour-gradient LB step on one MI355X.

Headline workload: the D3Q27 channel (256x128x128, no-slip y/z walls, body
force 1e-6 along x, 64 droplets R=10 at seeded random centres, near-contact
range 3 / strength 0.02, tau 1, FP32 storage and arithmetic, the plain
two-colour layout).  A step is one pass of the whole hot path over the
lattice: the read-once collision pass (pull, colour gradient, flags,
near-contact force, BGK + Guo, perturbation, recolouring, store, and the
scatter of the next step's colour densities) and the combine pass that
finishes the next phase field, with the populations resident in HBM.

Prints ONE JSON line: MLUPS (million lattice-site updates per second) of the
headline, timed with HIP events around the steps only; the roofline of the
dominant kernel (the collision pass) from per-launch events in a separate
profiled run; and beside it every other workload the benchmark is stated
for (512x256x256 in 16-bit storage, the 96-channel ensemble, the dense
emulsion with the learned near-contact closure trained on channel rows), and
the FP64 CPU oracle timed on the same inputs as GPU runs quoted next to it.
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


def say(*a):
    print("#", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(q, storage):
    """Per lattice update of the layout in use: (step, collision pass, phase
    pass).  Step: the state read once and written once, plus the phase field
    written once and read once; the plain per-colour FP32 D3Q27 step is 440 B.
    Phase pass: state read + phase written.  Collision pass: populations read
    + state written + phase read (per-colour: the whole state both ways;
    total layout: the scalars are written, not read, since rho_A follows from
    phi).  The read-once step's collision pass has the collision-pass bytes;
    its combine pass writes the phase field (the step's remaining 4 B)."""
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


KERNEL_SOURCES = ("step_kernels.hpp", "lattice_ops.hpp", "collide_launch.hpp", "scatter_geom.hpp", "api.hip")


def kernel_source_hash():
    """Hash of the sources that fix the passes' code and launch shapes (the
    kernels and their launch wrappers): a traffic figure measured for other
    sources is not reported."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2405_14551_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_tag, workload_tag):
    """HBM bytes per launch measured with rocprofv3 counters, if a summary for
    this kernel source is committed (profiles/traffic_<kernel>_<workload>.txt
    holds key = value lines incl. the source hash); None otherwise."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}_{workload_tag}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash() or "bytes_per_launch" not in kv:
        return None
    return float(kv["bytes_per_launch"])


# ------------------------------------------------------------------ GPU runs
def timed(sim, steps, profile=False):
    """ms per step of `steps` steps (HIP events on the library's stream); with
    profile, also the per-launch averages of the passes from a second run of
    the same length with per-launch events."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sim.sync()
    with torch.cuda.stream(sim.stream):
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if not profile:
        return ms, None
    sim.profile_begin()
    sim.step(steps)
    p = sim.profile_end()
    per = {k: (p["ms_" + k] / p["n_" + k] if p["n_" + k] else 0.0) for k in ("collide", "phase", "combine")}
    return ms, per


def run_variant(kw, cen, rad, steps, warmup, **over):
    """MLUPS and per-launch pass times of a workload with other settings."""
    from paper_2405_14551_amd import lb
    k = dict(kw, **over)
    sim = lb.Simulation(**k).init_droplets(cen, rad)
    copies = 1 if k.get("streaming") == "in_place" else 2
    n = int(np.prod(k["shape"]))
    state = copies * sim.state_bytes() / n
    sim.step(warmup)
    ms, per = timed(sim, steps, profile=True)
    d = sim.diagnostics()
    sim.close()
    return {"MLUPS": round(n / ms / 1e3, 1), "ms_per_step": round(ms, 5),
            "collide_ms": round(per["collide"], 5), "phase_ms": round(per["phase"], 5),
            "combine_ms": round(per["combine"], 5), "state_bytes_per_site": round(state, 1),
            "droplets": int(d[6])}


def headline(args):
    from paper_2405_14551_amd import lb, workloads as W
    w = W.channel_3d(storage=args.storage)
    kw, cen, rad = W.sim_kwargs(w)
    if args.phase != "auto":
        kw = dict(kw, phase=args.phase)
    n = int(np.prod(kw["shape"]))
    say(f"headline channel_3d {args.storage} {kw['shape']}")
    sim = lb.Simulation(**kw).init_droplets(cen, rad)
    sim.step(args.warmup)
    ms, _ = timed(sim, args.steps)
    _, per = timed(sim, args.steps, profile=True)
    diag = sim.diagnostics()
    sim.close()
    return kw, cen, rad, n, ms, per, diag


def big_lattice(steps, warmup):
    """The 512 x 256 x 256 lattice (1024 droplets R = 8): plain FP32 against
    the 16-bit storages (paper Sec. IV.A second group; shifted totals)."""
    from paper_2405_14551_amd import workloads as W
    w = W.big_3d(storage="f32")
    kw, cen, rad = W.sim_kwargs(w)
    out = {}
    for name, over in (("f32", {}), ("f16t", dict(storage="f16t")), ("f16t_sround", dict(storage="f16t", rounding="stochastic")),
                       ("bf16t", dict(storage="bf16t")), ("f16ct", dict(storage="f16ct"))):
        say(f"big_3d {name}")
        out[name] = run_variant(kw, cen, rad, steps, warmup, **over)
    for name in out:
        out[name]["vs_f32"] = round(out[name]["MLUPS"] / out["f32"]["MLUPS"], 3)
    return out


def channel_variants(kw, cen, rad, steps, warmup, ref_mlups):
    out = {}
    for name, over in (("f32_phase_pass", dict(phase="pass")), ("f32t", dict(storage="f32t")),
                       ("f16t", dict(storage="f16t")), ("f16t_sround", dict(storage="f16t", rounding="stochastic")),
                       ("bf16t", dict(storage="bf16t")), ("f16ct", dict(storage="f16ct")),
                       ("f32_in_place", dict(streaming="in_place")),
                       ("f16t_in_place", dict(storage="f16t", streaming="in_place")),
                       ("moments_f32", dict(scheme="moments"))):
        say(f"channel variant {name}")
        out[name] = run_variant(kw, cen, rad, steps, warmup, **over)
        out[name]["vs_plain_f32"] = round(out[name]["MLUPS"] / ref_mlups, 3)
    return out


def train_closure_on_channel(target_rows=10_000_000, every=400, max_steps=10_000):
    """The learned near-contact closure trained as the benchmark states it: on
    stencil / force rows the explicit model generates in channel runs (FP32,
    snapshots every `every` steps until `target_rows` rows or `max_steps`
    steps), 20k Adam steps of 256 rows (half force-active), the learning rate
    stepped down; the force error on a held-out snapshot of a second channel
    run (another droplet placement), per near-contact distance class."""
    import torch
    from paper_2405_14551_amd import lb, workloads as W
    w = W.channel_3d()
    kw, cen, rad = W.sim_kwargs(w)
    sim = lb.Simulation(**kw).init_droplets(cen, rad)
    act, free = [], []
    na_tot = nf_tot = 0
    t = 0
    t0 = time.perf_counter()
    while na_tot + nf_tot < target_rows and t < max_steps:
        sim.step(every)
        t += every
        r, g, na, nf = sim.nc_collect()
        act.append((r[:na].clone(), g[:na].clone()))
        free.append((r[na:].clone(), g[na:].clone()))
        na_tot += na
        nf_tot += nf
    sim.close()
    rows = torch.cat([a[0] for a in act] + [f[0] for f in free])
    tgs = torch.cat([a[1] for a in act] + [f[1] for f in free])
    del act, free
    collect_s = time.perf_counter() - t0
    say(f"closure rows: {na_tot} active, {nf_tot} free from {t} channel steps")
    tr = lb.Simulation(lattice="D3Q27", storage="f32", nc="explicit", shape=(16, 16, 16))
    tr.mlp_set_weights(W.closure_init_weights())
    t1 = time.perf_counter()
    losses = []
    for k, (n_steps, lr) in enumerate(((12000, 2e-3), (6000, 5e-4), (2000, 1e-4))):
        order = W.closure_batches(na_tot, nf_tot, n_steps, 256, seed=k + 1)
        losses.append(float(tr.mlp_train(rows, tgs, torch.from_numpy(order), lr=lr)[-200:].mean()))
    train_s = time.perf_counter() - t1
    theta, ranges = tr.mlp_get_weights(), tr.mlp_get_ranges()
    del rows, tgs
    # held-out snapshot: the same channel with another droplet placement
    wh = W.channel_3d(seed=W.SEED + 1)
    kwh, ch, rh = W.sim_kwargs(wh)
    sh = lb.Simulation(**kwh).init_droplets(ch, rh)
    sh.step(2000)
    r, g, na, nf = sh.nc_collect()
    sh.close()
    pred = tr.mlp_infer(r).double()
    tr.close()
    n = r[:, 27:30].double()
    gn = r[:, 30:31].double()
    T = g.double()
    F = gn * torch.clamp((pred * n).sum(1, keepdim=True), min=0.0) * n   # the force the step applies
    Fraw = gn * pred
    Fexp = gn * T
    mag = torch.linalg.norm(T, dim=1)
    act_m = mag > 0

    def err(Fx, m):
        d = torch.linalg.norm(Fexp[m])
        return float(torch.linalg.norm(Fx[m] - Fexp[m]) / d) if m.any() and d > 0 else None
    classes = {"active": act_m, "h<=2": (mag - 0.5).abs() < 1e-3, "h=3": (mag - 0.5 * (2 / 3) ** 3).abs() < 1e-3,
               "all": torch.ones_like(act_m)}
    return theta, ranges, {
        "recipe": f"channel 256x128x128 FP32 explicit force, rows every {every} steps",
        "rows": {"active": na_tot, "free": nf_tot, "total": na_tot + nf_tot, "stated": 10_000_000,
                 "channel_steps": t},
        "adam_steps": 20000, "batch": 256, "loss_end": losses,
        "collect_s": round(collect_s, 2), "train_s": round(train_s, 2),
        "held_out": {"workload": "channel_3d, droplet seed + 1, step 2000", "rows_active": na, "rows_free": nf,
                     "force_error_applied": {k: err(F, m) for k, m in classes.items()},
                     "force_error_raw": {k: err(Fraw, m) for k, m in classes.items()}},
    }


def closure_speed(kw, cen, rad, theta, ranges, steps, warmup):
    """Collision-pass time and MLUPS with the explicit near-contact scan and
    with the learned closure on the same workload; droplets after the run."""
    from paper_2405_14551_amd import lb
    out = {}
    for mode in ("explicit", "mlp"):
        sim = lb.Simulation(**dict(kw, nc=mode))
        if mode == "mlp":
            sim.mlp_set_weights(theta)
            sim.mlp_set_ranges(*ranges)
        sim.init_droplets(cen, rad)
        sim.step(warmup)
        ms, per = timed(sim, steps, profile=True)
        n = int(np.prod(kw["shape"]))
        fl = sim.fields(("flags",))["flags"]
        d = sim.diagnostics()
        out[mode] = {"MLUPS": round(n / ms / 1e3, 1), "collide_ms": round(per["collide"], 5),
                     "combine_ms": round(per["combine"], 5), "droplets": int(d[6]), "umax": round(float(d[5]), 5),
                     "interface_sites": int(((fl & 1) > 0).sum())}
        if mode == "mlp":
            out[mode]["network_share"] = round(int(((fl & 2) > 0).sum()) / max(out[mode]["interface_sites"], 1), 4)
        sim.close()
    out["collide_time_closure_vs_explicit"] = round(out["mlp"]["collide_ms"] / out["explicit"]["collide_ms"], 3)
    return out


def ensemble(steps, warmup, tune=None):
    """96 independent D3Q19 channels (sizes 64..160 x 64..96 x 64..96, tau
    0.6..1.2, 4..40 droplets each; FP32, near contact): autotuned launch
    configuration (or the given (mode, z_per_block, use_graph)) and
    aggregate MLUPS."""
    import torch
    from paper_2405_14551_amd import lb, workloads as W
    w = W.ensemble_channels()
    chans = w["channels"]
    n = int(sum(np.prod(c["shape"]) for c in chans))
    plain = [{k: v for k, v in c.items() if k not in ("centres", "radii")} for c in chans]
    ens = lb.Ensemble(plain, lattice=w["lattice"], storage=w["storage"], nc=w["nc"])
    for k, c in enumerate(chans):
        ens.init_droplets(k, c["centres"], c["radii"])
    if tune is None:
        best, table = ens.autotune(steps=4)
        for k, c in enumerate(chans):
            ens.init_droplets(k, c["centres"], c["radii"])
    else:
        ens.set_tuning(*tune)
        best, table = ens.tuning(), []
    ens.step(warmup)
    ens.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(ens.stream):
        e0.record(ens.stream)
        ens.step(steps)
        e1.record(ens.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ens.profile_begin()
    ens.step(steps)
    p = ens.profile_end()
    ens.close()
    b_step, b_col, _ = algorithmic_bytes(19, "f32")
    col_ms = p["ms_collide"] / steps
    return {"workload": "ensemble_96_d3q19", "channels": len(chans), "sites": n,
            "MLUPS": round(n / ms / 1e3, 1), "ms_per_step": round(ms, 4), "tuning": best,
            "collision_ms_per_step": round(col_ms, 4),
            "collision_frac": round(b_col * n / (col_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "step_frac": round(n / ms / 1e3 * 1e6 * b_step / 1e9 / HBM_PEAK_GBS, 4),
            "autotune": table}


def same_inputs_gpu(steps_c0=1000, steps_crop=50):
    """GPU MLUPS on the inputs the oracle is timed on: the 2D Laplace droplet
    (FP64) and the 64^3 crop of the 512 x 256 x 256 workload (FP64 and FP32)."""
    from paper_2405_14551_amd import lb, workloads as W
    out = {}
    w = W.laplace_2d(on_site=True)
    kw, cen, rad = W.sim_kwargs(w)
    sim = lb.Simulation(**kw).init_droplets(cen, rad)
    sim.step(10)
    ms, _ = timed(sim, steps_c0)
    sim.close()
    out["laplace_2d_f64"] = {"MLUPS": round(128 * 64 / ms / 1e3, 2), "steps": steps_c0}
    for st in ("f64", "f32"):
        w = W.big_3d_crop(storage=st)
        kw, cen, rad = W.sim_kwargs(w)
        sim = lb.Simulation(**kw).init_droplets(cen, rad)
        sim.step(10)
        ms, _ = timed(sim, max(steps_crop, 200))
        sim.close()
        out[f"crop_64_{st}"] = {"MLUPS": round(64 ** 3 / ms / 1e3, 1)}
    return out


def cpu_baseline():
    """The FP64 numpy oracle, single-threaded, on the same inputs as GPU runs
    in this benchmark: the 2D Laplace droplet (D2Q9 128 x 64, 1000 steps) and
    the 64^3 crop of the 512 x 256 x 256 workload (D3Q27, walls y/z, body
    force, near contact, its droplets; 30 steps).  About 20 s of CPU work."""
    from threadpoolctl import threadpool_limits
    from oracle.sim import OracleSim, OracleParams
    from paper_2405_14551_amd import workloads as W
    res = {}
    with threadpool_limits(1):
        w = W.laplace_2d(on_site=True)
        p = OracleParams(lattice="D2Q9", nx=128, ny=64, nz=1, tau=1.0, A=0.01, beta=0.7)
        sim = OracleSim(p).init_droplets(w["centres"], w["radii"])
        t0 = time.perf_counter()
        sim.step(1000)
        el = time.perf_counter() - t0
        res["laplace_2d"] = {"MLUPS": round(128 * 64 * 1000 / el / 1e6, 4), "steps": 1000, "seconds": round(el, 2)}
        w = W.big_3d_crop(storage="f64")
        p = OracleParams(lattice="D3Q27", nx=64, ny=64, nz=64, walls=tuple(bool(v) for v in w["walls"]), tau=1.0,
                         A=0.01, beta=0.7, body_force=tuple(w["body_force"]), nc=True, nc_A=0.02, nc_hmin=2.0,
                         nc_hmax=3.0)
        sim = OracleSim(p).init_droplets(w["centres"], w["radii"])
        steps = 30
        t0 = time.perf_counter()
        sim.step(steps)
        el = time.perf_counter() - t0
        res["crop_64"] = {"MLUPS": round(64 ** 3 * steps / el / 1e6, 4), "steps": steps, "seconds": round(el, 2)}
    host = f"{platform.processor() or platform.machine()}, host nproc {os.cpu_count()}"
    return {"value": res["crop_64"]["MLUPS"], "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"FP64 numpy oracle, 1 thread ({host}): the 64^3 crop of the 512x256x256 workload "
                      f"(D3Q27, walls y/z, body force 1e-6, near contact on, {len(w['radii'])} droplets R=8), "
                      f"{res['crop_64']['steps']} steps in {res['crop_64']['seconds']} s (value); the 2D Laplace "
                      f"droplet (D2Q9 128x64, 1000 steps) in {res['laplace_2d']['seconds']} s",
            "runs": res}


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
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the channel workload (for profiling runs)")
    ap.add_argument("--storage", default="f32", choices=sorted(ELEM),
                    help="storage of the channel workload (profiling runs; the headline is f32)")
    ap.add_argument("--phase", default="auto", choices=("auto", "scatter", "pass"),
                    help="read-once or two-pass step for the channel workload (profiling runs)")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the ensemble workload, batched with 16 planes per march and no autotuning "
                         "(for profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    if args.ensemble_only:
        print(json.dumps({"ensemble": ensemble(args.steps, args.warmup, tune=("batched", 16, 0))}), flush=True)
        return 0

    kw, cen, rad, n, ms, per, diag = headline(args)
    q = 27
    mlups = n / ms / 1e3
    b_step, b_col, _ = algorithmic_bytes(q, args.storage)
    col_ms = per["collide"]
    achieved = b_col * n / (col_ms / 1e3) / 1e9
    traffic = traffic_from_profiles("collide", f"channel_3d_{args.storage}")
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic (seeded droplet placement)",
        "config": {"workload": "channel_3d", "lattice": "D3Q27", "storage": args.storage,
                   "step": "read-once" if per["combine"] > 0 else "phase pass + collision",
                   "shape": list(kw["shape"]), "walls": list(kw["walls"]), "droplets": int(len(rad)),
                   "near_contact": kw["nc"], "sites": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_vs_algorithmic": (round(traffic / (b_col * n), 3) if traffic else None),
                     "kernel": "k_collide (read-once collision pass)" if per["combine"] > 0
                               else "k_collide (collision pass)", "bytes_per_site": b_col,
                     "avg_launch_ms": round(col_ms, 5),
                     "step_frac": round(mlups * 1e6 * b_step / 1e9 / HBM_PEAK_GBS, 4),
                     "step_bytes_per_site": b_step,
                     "combine_launch_ms": round(per["combine"], 5),
                     "phase_launch_ms": round(per["phase"], 5)},
        "sanity": {"droplets_end": int(diag[6]), "umax": float(diag[5])},
    }
    if not args.headline_only:
        vs = min(args.steps, 50)
        wu = min(args.warmup, 10)
        out["variants"] = channel_variants(kw, cen, rad, vs, wu, mlups)
        out["big_3d"] = big_lattice(min(args.steps, 20), 3)
        theta, ranges, tr = train_closure_on_channel()
        out["closure"] = tr
        out["closure"]["channel_3d"] = closure_speed(kw, cen, rad, theta, ranges, vs, wu)
        from paper_2405_14551_amd import workloads as W
        wd = W.dense_3d()
        kwd, cend, radd = W.sim_kwargs(wd)
        say("dense_3d explicit vs closure")
        out["closure"]["dense_3d"] = closure_speed(kwd, cend, radd, theta, ranges, min(args.steps, 20), 100)
        say("ensemble")
        out["ensemble"] = ensemble(min(args.steps, 20), 5)
        out["same_inputs_gpu"] = same_inputs_gpu()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
