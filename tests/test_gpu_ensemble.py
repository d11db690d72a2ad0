"""GPU tests of the batched ensemble (independent channels of different
sizes, walls, tau and forces advanced together): each channel against the
FP64 oracle in both launch modes, with and without the captured graph; graph
replays against eager stepping; the read-once step's launch modes, store
policies, restart and stand-alone channels bit for bit; and the autotuner."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402
from oracle.sim import OracleSim, OracleParams  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# three uneven channels; off-site droplet centres (no site at a symmetry point)
CHANNELS = [
    dict(shape=(70, 20, 13), walls=(0, 1, 1), tau=0.9, A=0.02, body_force=(2e-5, 0.0, 0.0),
         centres=[[21.17, 9.77, 6.81], [33.17, 10.11, 6.37]], radii=[4.0, 4.0]),
    dict(shape=(64, 16, 12), walls=(0, 0, 0), tau=0.7, A=0.01, body_force=(0.0, 1e-5, 0.0),
         centres=[[20.3, 7.9, 5.6]], radii=[4.5]),
    dict(shape=(40, 24, 20), walls=(0, 0, 1), tau=1.1, tau_b=0.6, A=0.015, body_force=(1e-5, 0.0, 2e-6),
         centres=[[12.3, 11.7, 10.2], [26.8, 12.1, 9.9]], radii=[5.5, 5.5]),
]


def make(storage="f64", lattice="D3Q19"):
    chans = [{k: v for k, v in c.items() if k not in ("centres", "radii")} for c in CHANNELS]
    ens = lb.Ensemble(chans, lattice=lattice, storage=storage, nc="explicit")
    for k, c in enumerate(CHANNELS):
        ens.init_droplets(k, c["centres"], c["radii"])
    return ens


def oracle(c, lattice, steps):
    nx, ny, nz = c["shape"]
    p = OracleParams(lattice=lattice, nx=nx, ny=ny, nz=nz, walls=tuple(bool(w) for w in c["walls"]),
                     tau=c["tau"], tau_b=c.get("tau_b", 0.0), A=c["A"], beta=0.7,
                     body_force=tuple(c["body_force"]), nc=True)
    return OracleSim(p).init_droplets(c["centres"], c["radii"]).step(steps)


@pytest.mark.parametrize("mode,graph", [("batched", 0), ("batched", 1), ("per_channel", 0), ("per_channel", 1)])
@pytest.mark.parametrize("lattice", ["D3Q19", "D3Q27"])
def test_ensemble_fp64_matches_oracle_per_channel(mode, graph, lattice):
    steps = 30
    say(f"case ensemble fp64 {lattice} mode={mode} graph={graph}")
    ens = make("f64", lattice)
    ens.set_tuning(mode, z_per_block=4, use_graph=graph)
    for k in range(0, steps, 10):
        ens.step(10)      # with the graph: four replays and two eager steps
        ens.sync()
        say(f"  step {k + 10} done")
    raw = ens.get_state()
    for k, c in enumerate(CHANNELS):
        st = ens.channel_state(raw, k).cpu().numpy()
        o = oracle(c, lattice, steps)
        e = max(np.abs(st[0] - o.fA).max(), np.abs(st[1] - o.fB).max()) / np.abs(o.fA).max()
        say(f"  channel {k} {c['shape']}: rel err {e:.2e}")
        assert e < 1e-12, (k, e)
        f = {n: v.cpu().numpy() for n, v in ens.fields(k, ("rho_a", "f_nc")).items()}
        of = o.fields()
        assert np.abs(f["rho_a"] - of["rho_a"]).max() < 1e-12
        assert np.abs(f["f_nc"] - of["f_nc"]).max() < 1e-12
    assert any(np.abs(oracle(c, lattice, steps).fields()["f_nc"]).max() > 0 for c in CHANNELS)
    ens.close()


@pytest.mark.parametrize("storage", ["f32", "f16t", "f16ct"])
def test_graph_replays_match_eager(storage):
    """Several graph replays, with eager work and synchronisations between
    them, give bit-identical states to eager single launches."""
    say(f"case ensemble graph replays {storage}")
    a = make(storage)
    b = make(storage)
    a.set_tuning("batched", z_per_block=4, use_graph=1)
    b.set_tuning("batched", z_per_block=4, use_graph=0)
    for chunk in (5, 8, 7, 6):
        a.step(chunk)
        a.sync()
        a.fields(0, ("rho_a",))          # eager work between replays
        b.step(chunk)
        b.sync()
        assert torch.equal(a.get_state(), b.get_state()), chunk
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f32t"])
def test_read_once_modes_restart_and_single_lattice_agree_bitwise(storage):
    """Read-once ensembles (the default step for these storages): the batched
    launches and the per-channel launches give the same state bit for bit; a
    restart from a saved state (the bootstrap scatter) continues bit for bit;
    and each channel equals the same lattice stepped on its own as a single
    handle with the same march depth (the same tile code and sums)."""
    say(f"case ensemble read-once bitwise {storage}")
    a = make(storage)
    b = make(storage)
    a.set_tuning("batched", z_per_block=4, use_graph=1)
    b.set_tuning("per_channel", z_per_block=4, use_graph=0)
    a.step(9)
    b.step(9)
    a.sync()
    b.sync()
    assert torch.equal(a.get_state(), b.get_state())
    # restart: save after 9 steps, run 6 more, restore, run 6 again
    saved = a.get_state().clone()
    a.step(6)
    a.sync()
    ref = a.get_state().clone()
    a.set_state(saved)
    a.step(6)
    a.sync()
    assert torch.equal(a.get_state(), ref)
    # each channel alone (the ensemble's state is the channels' states in order)
    raw = ref.view(torch.uint8).reshape(-1)
    off = 0
    for k, c in enumerate(CHANNELS):
        kw = {n: v for n, v in c.items() if n not in ("centres", "radii")}
        sim = lb.Simulation(lattice="D3Q19", storage=storage, nc="explicit", **kw)
        sim.set_z_per_block(4)
        sim.init_droplets(c["centres"], c["radii"])
        sim.step(15)
        sim.sync()
        alone = sim.get_state().contiguous().view(torch.uint8).reshape(-1)
        nb = alone.numel()
        assert torch.equal(raw[off:off + nb], alone), k
        off += nb
        sim.close()
    assert off == raw.numel()
    a.close()
    b.close()


@pytest.mark.parametrize("stores", ["nt", "cached"])
def test_read_once_store_policies_agree_bitwise(stores, monkeypatch):
    """The batched read-once collision stores the populations non-temporally
    or through L2 (chosen from the channels' row alignment, forced here both
    ways): the state equals the per-channel launches' bit for bit."""
    say(f"case ensemble read-once stores={stores}")
    monkeypatch.setenv("LB_ENSEMBLE_STORES", stores)
    a = make("f32")
    b = make("f32")
    a.set_tuning("batched", z_per_block=4, use_graph=0)
    b.set_tuning("per_channel", z_per_block=4, use_graph=0)
    a.step(7)
    b.step(7)
    a.sync()
    b.sync()
    assert torch.equal(a.get_state(), b.get_state())
    a.close()
    b.close()


def test_autotune_picks_a_measured_config(tmp_path):
    say("case ensemble autotune")
    ens = make("f32")
    cache = str(tmp_path / "tune.json")
    best, table = ens.autotune(steps=2, cache=cache)
    assert len(table) >= 2
    assert best["ms_per_step"] == min(r["ms_per_step"] for r in table)
    # each candidate measured once: the per-channel mode has no graph variant
    assert not any(r["mode"] == "per_channel" and r["use_graph"] for r in table)
    assert len({(r["mode"], r["z_per_block"], r["use_graph"]) for r in table}) == len(table)
    best2, _ = ens.autotune(steps=2, cache=cache)   # cached
    assert best2["z_per_block"] == best["z_per_block"] and best2["mode"] == best["mode"]
    assert best2["use_graph"] == best["use_graph"]
    ens.sync()
    ens.close()


def _window(t, colour):
    """step_window gatherer over one colour of a channel's device state view."""
    def take(iz, iy, ix):
        dev = t.device
        w = t[colour][:, torch.as_tensor(iz, device=dev)][:, :, torch.as_tensor(iy, device=dev)]
        return w[:, :, :, torch.as_tensor(ix, device=dev)].double().cpu().numpy()
    return take


def test_ensemble_full_size_sampled_sites():
    """The 96-channel D3Q19 ensemble (67.5M sites, FP32, near contact) in the
    benchmark's batched configuration: one step from a developed state
    against the oracle's windowed step at sampled sites of several channels
    (near-contact sites, walls, corners, the channel's last site)."""
    from oracle.sim import step_window
    w = W.ensemble_channels()
    chans = w["channels"]
    plain = [{k: v for k, v in c.items() if k not in ("centres", "radii")} for c in chans]
    say(f"case ensemble full size: {len(chans)} channels")
    ens = lb.Ensemble(plain, lattice="D3Q19", storage="f32", nc="explicit")
    ens.set_tuning("batched", z_per_block=2, use_graph=1)
    for k, c in enumerate(chans):
        ens.init_droplets(k, c["centres"], c["radii"])
    ens.step(6)
    ens.sync()
    pre = ens.get_state().clone()
    ens.step(1)
    ens.sync()
    post = ens.get_state()
    sizes = [np.prod(c["shape"]) for c in chans]
    picks = sorted({0, len(chans) - 1, int(np.argmin(sizes)), int(np.argmax(sizes)), 37, 58})
    rng = np.random.default_rng(11)
    worst = 0.0
    for k in picks:
        c = chans[k]
        nx, ny, nz = c["shape"]
        fnc = ens.fields(k, ("f_nc",))["f_nc"].cpu().numpy()
        act = np.argwhere(np.abs(fnc).sum(0) > 0)
        sites = [(nx - 1, ny - 1, nz - 1), (0, 0, 0), (int(rng.integers(nx)), 0, int(rng.integers(nz)))]
        for j in rng.choice(len(act), size=min(3, len(act)), replace=False):
            z, y, x = act[j]
            sites.append((int(x), int(y), int(z)))
        p = OracleParams(lattice="D3Q19", nx=nx, ny=ny, nz=nz, walls=tuple(bool(v) for v in c["walls"]), tau=c["tau"],
                         A=c["A"], beta=c["beta"], body_force=tuple(c["body_force"]), nc=True, nc_A=c["nc_A"],
                         nc_hmin=c["nc_hmin"], nc_hmax=c["nc_hmax"], decision_dtype=np.float32)
        sv, pv = ens.channel_state(pre, k), ens.channel_state(post, k)
        for (x, y, z) in sites:
            a, b, _ = step_window(p, _window(sv, 0), _window(sv, 1), (x, y, z))
            na = pv[0, :, z, y, x].double().cpu().numpy()
            nb = pv[1, :, z, y, x].double().cpu().numpy()
            e = max(np.abs(na - a).max(), np.abs(nb - b).max()) / np.abs(a + b).max()
            worst = max(worst, e)
            assert e < 2e-6, (k, (x, y, z), e)
    say(f"  channels {picks}: worst rel err {worst:.2e}")
    del pre
    ens.close()
