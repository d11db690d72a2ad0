"""The largest lattice the library accepts in 16-bit storage, held in place
on one MI355X: 1024 x 1024 x 1023 sites (1.07e9; a velocity pair's two FP16
planes take 4.29 GB, one 1024 x 1024 plane short of the 4 GiB a 32-bit byte
offset reaches), D3Q27, FP16 total layout,
in-place (AA) streaming, the channel physics (walls y/z, body force, near
contact) with 256 droplets R = 10.  About 119 GB of device memory for the
handle and 75 GB for one canonical copy of the state.  One odd-kind step
(each site's own slots) from a developed state against the oracle's windowed step at
sampled sites, many in the far planes of the lattice."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402
from oracle.lattice import make_lattice  # noqa: E402
from oracle.sim import step_window  # noqa: E402

from test_gpu_parity import _total_window_gatherer, oparams  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_billion_site_fp16_total_in_place_sampled_sites():
    shape = (1024, 1024, 1023)
    nx, ny, nz = shape
    n = nx * ny * nz
    assert 2 * 2 * n < 2 ** 32 <= 2 * 2 * (n + nx * ny)
    w = W.channel_3d(shape=shape, count=256, radius=10.0, storage="f16t")
    kw, cen, rad = W.sim_kwargs(w)
    kw["streaming"] = "in_place"
    say(f"case largest FP16 total lattice in place {shape} ({n / 1e9:.3f}e9 sites, {len(rad)} droplets)")
    # the library allocates its ~120 GB itself: hand back what torch holds cached
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < 210e9:
        pytest.skip(f"needs about 200 GB of free device memory, {free / 1e9:.0f} GB free")
    try:
        sim = lb.Simulation(**kw)
    except lb.LBError as e:
        if e.code == lb.LB_ENOMEM:
            pytest.skip(f"device memory: {e}")
        raise
    sim.init_droplets(cen, rad)
    sim.step(5)
    sim.sync()
    # throughput at this size (20 steps, HIP events on the library's stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(sim.stream):
        e0.record(sim.stream)
        sim.step(20)
        e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    say(f"  {ms:.2f} ms per step, {n / (ms / 1e3) / 1e6:.0f} MLUPS; state {sim.state_bytes() / 1e9:.1f} GB")
    # 25 steps so far: the state is gathered from the streamed slots, and the
    # next step is of the odd kind (reads and writes each site's own slots)
    rng = np.random.default_rng(11)
    sites = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz - 2), (1, ny - 2, nz - 1), (511, 512, 1022)]
    for _ in range(8):
        sites.append((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz - 64, nz))))
    for _ in range(4):
        sites.append((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    p = oparams(kw, np.float32)
    pre = sim.get_state()
    gA, gB = _total_window_gatherer(sim, pre, 0), _total_window_gatherer(sim, pre, 1)
    want = {s: step_window(p, gA, gB, s) for s in sites}
    del pre, gA, gB
    torch.cuda.empty_cache()
    sim.step(1)
    post = sim.get_state()
    T, sc = sim.split_total_state(post)
    wq = make_lattice("D3Q27").w
    worst = 0.0
    for (x, y, z) in sites:
        a, b, _ = want[(x, y, z)]
        T_orc = a + b - wq
        T_gpu = T[:, z, y, x].double().cpu().numpy()
        half_step = np.maximum(np.abs(T_orc) * 2.0 ** -11, 2.0 ** -25)
        excess = (np.abs(T_gpu - T_orc) - half_step) / np.abs(a + b).max()
        worst = max(worst, float(excess.max()))
        assert np.all(excess < 2e-6), ((x, y, z), excess.max())
        frac = float(sc[0, z, y, x])
        assert abs(frac - a.sum() / (a + b).sum()) < 1e-5, (x, y, z)
    say(f"  sampled {len(sites)} sites, worst excess over half an FP16 step {worst:.2e}")
    del post, T, sc
    sim.close()
    torch.cuda.empty_cache()
