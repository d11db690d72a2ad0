"""GPU: single-lattice steps replayed from a captured hipGraph (pairs of
non-field steps at the buffer parities of the capture) give the state of
direct launches bit for bit, in every step structure: the read-once step
(two copies and in place), the two-pass step (two copies and in place), the
moment scheme, the learned closure and a D2Q9 lattice.  Replays alternate
with direct steps, field reads, restores and a change of march depth, and
every replay is compared with the direct run.  Also the single-lattice
autotuner over march depths and graph replays."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


BASE = dict(lattice="D3Q27", nc="explicit", shape=(70, 20, 18), walls=(0, 1, 1), body_force=(1e-5, 0, 0),
            u0=(0.02, 0.0, 0.0), tau=0.9, A=0.02)
CEN = np.array([[20.3, 9.7, 8.6], [44.9, 10.2, 9.1]])
RAD = np.array([6.0, 6.0])

CASES = {
    "f32_read_once": dict(storage="f32"),
    "f32_read_once_in_place": dict(storage="f32", streaming="in_place"),
    "f16t_two_pass": dict(storage="f16t"),
    "f16t_two_pass_in_place": dict(storage="f16t", streaming="in_place"),
    "f64_two_pass": dict(storage="f64", phase="pass"),
    "f32_moments": dict(storage="f32", scheme="moments"),
    "f32_closure": dict(storage="f32", nc="mlp"),
    "d2q9_f64": dict(lattice="D2Q9", storage="f64", shape=(128, 64, 1), walls=(0, 0, 0), body_force=(0, 0, 0),
                     u0=(0, 0, 0), tau=1.0, A=0.01, nc="off"),
}


def make(name, graph):
    kw = dict(BASE, **CASES[name])
    sim = lb.Simulation(**kw)
    if kw["nc"] == "mlp":
        sim.mlp_set_weights(W.closure_init_weights())
        sim.mlp_set_ranges(np.full(30, -2.0, np.float32), np.full(30, 2.0, np.float32), 0.0)
    if kw["lattice"] == "D2Q9":
        sim.init_droplets(np.array([[64.0, 32.0, 0.0]]), np.array([16.0]))
    else:
        sim.init_droplets(CEN, RAD)
    sim.set_graph(graph)
    return sim


def same(a, b):
    return torch.equal(a.get_state().contiguous().view(torch.uint8), b.get_state().contiguous().view(torch.uint8))


@pytest.mark.parametrize("name", list(CASES))
def test_graph_replays_match_direct_launches_bitwise(name):
    say(f"case single-lattice graph {name}")
    a = make(name, True)
    b = make(name, False)
    # odd and even chunk lengths: replays start at either parity
    for k, chunk in enumerate((5, 8, 7, 6, 1, 9)):
        a.step(chunk)
        b.step(chunk)
        a.sync()
        b.sync()
        assert same(a, b), (name, k, chunk)
        fa = a.fields(("phi", "u"))
        fb = b.fields(("phi", "u"))
        assert torch.equal(fa["phi"], fb["phi"]) and torch.equal(fa["u"], fb["u"]), (name, k)
    # a restore (the read-once step scatters the restored state first) and a
    # new march depth (new halo blocks: the captured graph is dropped)
    saved = b.get_state().clone()
    a.set_state(saved)
    b.set_state(saved)
    a.step(6)
    b.step(6)
    a.sync()
    b.sync()
    assert same(a, b), (name, "restore")
    # a new initialisation after an odd number of steps: the buffer parities
    # pair up differently, and the graph is captured again
    a.step(1)
    b.step(1)
    for sim in (a, b):
        if CASES[name].get("lattice", "D3Q27") == "D2Q9":
            sim.init_droplets(np.array([[64.0, 32.0, 0.0]]), np.array([16.0]))
        else:
            sim.init_droplets(CEN, RAD)
    a.step(9)
    b.step(9)
    a.sync()
    b.sync()
    assert same(a, b), (name, "re-initialised")
    if CASES[name].get("lattice", "D3Q27") != "D2Q9":
        a.set_z_per_block(4)
        b.set_z_per_block(4)
        a.step(7)
        b.step(7)
        a.sync()
        b.sync()
        assert same(a, b), (name, "z_per_block")
    a.close()
    b.close()


def test_single_lattice_autotune_covers_depths_and_graphs():
    """lb_autotune on a single lattice times every march depth up to nz with
    and without graph replays, keeps the fastest and leaves it set."""
    say("case single-lattice autotune")
    sim = make("f32_read_once", False)
    best, table = sim.autotune(steps=3)
    cands = {(r["z_per_block"], r["use_graph"]) for r in table}
    assert cands == {(zb, g) for zb in (1, 2, 4, 8, 16) for g in (0, 1)}, cands
    assert len(table) == len(cands)
    assert best["ms_per_step"] == min(r["ms_per_step"] for r in table)
    assert sim.tuning() == {"z_per_block": best["z_per_block"], "use_graph": best["use_graph"]}
    sim.step(5)
    sim.sync()
    assert torch.isfinite(sim.fields(("rho_a",))["rho_a"]).all()
    sim.close()
