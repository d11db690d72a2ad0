"""Host-side logic on the CPU: the benchmark's byte definitions and guards, and
the seeded workload recipes the parity tests and the benchmark share."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2405_14551_amd import workloads as W  # noqa: E402


def test_algorithmic_bytes_per_update():
    """The step's algorithmic bytes: populations read and written once, the
    phase field once each way (440 B for D3Q27 FP32, 304 B for D2Q9 FP64,
    312 B for D3Q19 FP32); the collision pass of the plain layout reads and
    writes the state and reads phi (436 B), the phase pass reads the state
    and writes phi (220 B); the total layout moves Q values + 16 B of scalars."""
    assert bench.plain_state_bytes(27, "f32") == 440
    assert bench.plain_state_bytes(9, "f64") == 304
    assert bench.plain_state_bytes(19, "f32") == 312
    assert bench.plain_state_bytes(27, "f16t") == 224
    step, coll, phase = bench.algorithmic_bytes(27, "f32")
    assert (step, coll, phase) == (440, 436, 220)
    step, coll, phase = bench.algorithmic_bytes(27, "f16t")
    assert (step, coll, phase) == (2 * (27 * 2 + 16) + 8, 2 * 27 * 2 + 16 + 4, 27 * 2 + 16 + 4)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    line = [l for l in r.stdout.splitlines() if l.startswith("{")][-1]
    assert json.loads(line)["n_gpus"] == 2


def _min_gap(cen, rad, shape, walls):
    n = np.asarray(shape, float)
    worst = np.inf
    for i in range(len(cen)):
        d = cen - cen[i]
        for a in range(3):
            if not walls[a]:
                d[:, a] -= n[a] * np.round(d[:, a] / n[a])
        r = np.sqrt((d * d).sum(1))
        r[i] = np.inf
        worst = min(worst, (r - rad - rad[i]).min())
    return worst


def test_channel_recipe():
    """64 droplets of radius 10 in the 256 x 128 x 128 channel, seeded: at
    least 3 sites between surfaces (minimum image along x) and 2 sites of
    clearance from the walls; the same list on every call."""
    w = W.channel_3d()
    cen, rad = w["centres"], w["radii"]
    assert cen.shape == (64, 3) and np.all(rad == 10.0)
    assert _min_gap(cen, rad, w["shape"], w["walls"]) >= 3.0 - 1e-12
    for a in (1, 2):
        assert np.all(cen[:, a] - rad >= 2.0) and np.all(cen[:, a] + rad <= w["shape"][a] - 1 - 2.0)
    assert np.array_equal(cen, W.channel_3d()["centres"])


def test_ensemble_recipe():
    """96 D3Q19 channels: nx in 64..160, ny and nz in 64..96, tau in
    [0.6, 1.2], each channel's droplets separated by at least 3 sites."""
    w = W.ensemble_channels()
    ch = w["channels"]
    assert len(ch) == 96 and w["lattice"] == "D3Q19"
    for c in ch:
        nx, ny, nz = c["shape"]
        assert 64 <= nx <= 160 and 64 <= ny <= 96 and 64 <= nz <= 96
        assert 0.6 <= c["tau"] <= 1.2
        if len(c["radii"]) > 1:
            assert _min_gap(np.asarray(c["centres"]), np.asarray(c["radii"]), c["shape"], c["walls"]) >= 3.0 - 1e-9


@pytest.mark.parametrize("kind", ["big", "dense"])
def test_large_recipes(kind):
    if kind == "big":
        w = W.big_3d()
        assert w["shape"] == (512, 256, 256) and len(w["radii"]) == 1024
    else:
        w = W.dense_3d()
        assert w["shape"] == (384, 384, 192) and len(w["radii"]) == 2000
        # every film starts beyond the near-contact range h_max = 3
        assert _min_gap(w["centres"], w["radii"], w["shape"], w["walls"]) > 3.0
        assert np.all(w["centres"][:, 2] - 8.0 >= 2.0)
        assert np.all(w["centres"][:, 2] + 8.0 <= w["shape"][2] - 1 - 2.0)
    assert np.all(np.isfinite(w["centres"]))


@pytest.mark.parametrize("workload", ["channel_3d_f32", "channel_3d_f16t"])
def test_committed_counter_summary_matches_the_kernel_sources(workload):
    """The HBM traffic the benchmark reports comes from rocprofv3 counters
    taken for exactly the committed kernel and launch sources: the summary's
    source hash must match them (a kernel edit needs the counters taken
    again), and the bytes per launch must exceed the algorithmic bytes of one
    collision launch on the 256 x 128 x 128 channel."""
    b = bench.traffic_from_profiles("collide", workload)
    assert b is not None, "profiles/traffic_collide_%s.txt is stale or missing" % workload
    sites = 256 * 128 * 128
    per_site = bench.algorithmic_bytes(27, "f32" if workload.endswith("f32") else "f16t")[1]
    assert 1.0 <= b / (per_site * sites) < 1.5
