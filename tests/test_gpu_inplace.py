"""In-place (AA-pattern) streaming against two-copy streaming and the oracle.

An in-place step reads the same operands as a two-copy step and does the same
arithmetic on them; only the addresses differ.  The bar between the two is
therefore bitwise equality of every field and of the state (which the library
hands out in the canonical layout whatever the streaming), after odd and even
step counts.  FP64 in place is also held to the oracle at 1e-12 relative."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402
from oracle.sim import OracleSim, OracleParams  # noqa: E402

FIELDS = ("rho_a", "rho_b", "phi", "u", "f_nc", "flags")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _drops(shape, d3):
    nx, ny, nz = shape
    R = min(6.0, ny * 0.3, (nz * 0.3 if d3 else 99))
    cen = np.array([[nx * 0.3 + 0.17, ny * 0.5 - 0.23, nz * 0.5 + 0.31 if d3 else 0.0],
                    [nx * 0.3 + 2 * R + 3.17, ny * 0.5 + 0.11, nz * 0.5 - 0.13 if d3 else 0.0]])
    return cen, [R, R]


def _same(a, b):
    """Bitwise equality of two simulations' fields and states."""
    fa, fb = a.fields(FIELDS), b.fields(FIELDS)
    for k in FIELDS:
        assert torch.equal(fa[k], fb[k]), k
    sa, sb = a.get_state(), b.get_state()
    assert torch.equal(sa.view(torch.uint8), sb.view(torch.uint8)), "state"


CASES = [
    ("D2Q9", (70, 37, 1), (0, 1, 0), "explicit"),
    ("D3Q19", (67, 21, 14), (0, 1, 1), "explicit"),
    ("D3Q27", (70, 20, 13), (0, 1, 1), "explicit"),
    ("D3Q27", (64, 8, 24), (1, 0, 0), "off"),
    ("D3Q27", (33, 17, 9), (1, 1, 1), "explicit"),
]
STORAGES = ["f64", "f32", "f32s", "f16", "bf16", "f32t", "f16t", "bf16t", "f16ct"]


@pytest.mark.parametrize("lat,shape,walls,nc", CASES)
@pytest.mark.parametrize("storage", STORAGES)
def test_in_place_equals_two_copies(lat, shape, walls, nc, storage):
    say(f"case in place vs two copies {lat} {storage} {shape} walls={walls} nc={nc}")
    cen, rad = _drops(shape, lat != "D2Q9")
    kw = dict(lattice=lat, storage=storage, nc=nc, shape=shape, walls=walls, tau=0.9, tau_b=1.3,
              A=0.02, body_force=(2e-5, 1e-6, 0), u0=(0.01, -0.005, 0.0), nc_A=0.03)
    ab = lb.Simulation(**kw).init_droplets(cen, rad)
    ip = lb.Simulation(streaming="in_place", **kw).init_droplets(cen, rad)
    _same(ab, ip)
    for n in (5, 1, 3):               # 5 (odd), 6 (even), 9 (odd) steps
        ab.step(n)
        ip.step(n)
        _same(ab, ip)
    # the host copy of an odd-count state goes through the staging plane
    assert np.array_equal(ip.get_state(host=True), ab.get_state(host=True))


@pytest.mark.parametrize("lat,shape,walls,nc", CASES[1:])
@pytest.mark.parametrize("storage", ["f16t", "bf16t"])
def test_in_place_equals_two_copies_stochastic_rounding(lat, shape, walls, nc, storage):
    """Stochastic rounding keys its random words on site, direction and step,
    not on where a value is stored: pushed slots (in place) and the site's own
    (two copies) receive the same bits, and a second run repeats them."""
    say(f"case in place vs two copies, stochastic rounding {lat} {storage} {shape}")
    cen, rad = _drops(shape, True)
    kw = dict(lattice=lat, storage=storage, nc=nc, shape=shape, walls=walls, tau=0.9, A=0.02,
              body_force=(2e-5, 1e-6, 0), u0=(0.01, -0.005, 0.0), nc_A=0.03, rounding="stochastic")
    ab = lb.Simulation(**kw).init_droplets(cen, rad)
    ip = lb.Simulation(streaming="in_place", **kw).init_droplets(cen, rad)
    again = lb.Simulation(**kw).init_droplets(cen, rad)
    for n in (5, 1):
        ab.step(n)
        ip.step(n)
        again.step(n)
        _same(ab, ip)
        _same(ab, again)
    # the rounding differs from round-to-nearest
    rne = lb.Simulation(**dict(kw, rounding="nearest")).init_droplets(cen, rad)
    rne.step(6)
    assert not torch.equal(rne.get_state(), ab.get_state())
    ab.close()
    ip.close()


@pytest.mark.parametrize("storage", ["f32", "f16t"])
def test_in_place_set_state_resumes(storage):
    """A state taken after an odd number of in-place steps and set into a new
    in-place handle continues exactly as the handle it came from."""
    say(f"case in place set_state {storage}")
    shape = (48, 24, 20)
    cen, rad = _drops(shape, True)
    kw = dict(lattice="D3Q27", storage=storage, nc="explicit", shape=shape, walls=(0, 1, 1), tau=0.8)
    a = lb.Simulation(streaming="in_place", **kw).init_droplets(cen, rad)
    a.step(7)
    b = lb.Simulation(streaming="in_place", **kw).init_droplets(cen, rad)
    b.set_state(a.get_state())
    a.step(4)
    b.step(4)
    _same(a, b)
    a.close()
    b.close()


def test_in_place_fp64_matches_oracle():
    say("case in place fp64 vs oracle D3Q27 walls nc 61 steps")
    shape = (70, 20, 13)
    cen, rad = _drops(shape, True)
    kw = dict(lattice="D3Q27", storage="f64", nc="explicit", shape=shape, walls=(0, 1, 1), tau=0.9,
              A=0.02, body_force=(2e-5, 0, 0), nc_A=0.03)
    sim = lb.Simulation(streaming="in_place", **kw).init_droplets(cen, rad)
    p = OracleParams(lattice="D3Q27", nx=70, ny=20, nz=13, walls=(False, True, True), tau=0.9, A=0.02,
                     beta=0.7, body_force=(2e-5, 0, 0), nc=True, nc_A=0.03)
    orc = OracleSim(p).init_droplets(cen, rad)
    sim.step(61)
    orc.step(61)
    st = sim.get_state().cpu().numpy()
    den = np.abs(orc.fA).max()
    ea = np.abs(st[0] - orc.fA).max() / den
    eb = np.abs(st[1] - orc.fB).max() / den
    g = {k: v.cpu().numpy() for k, v in sim.fields(("rho_a", "u", "f_nc")).items()}
    o = orc.fields()
    eu = np.abs(g["u"] - o["u"]).max() / np.abs(o["u"]).max()
    say(f"  state rel err A {ea:.2e} B {eb:.2e}, u {eu:.2e}")
    assert ea < 1e-12 and eb < 1e-12 and eu < 1e-12
    assert np.abs(g["f_nc"]).max() > 0
    sim.close()


@pytest.mark.parametrize("storage", ["f32", "f32t"])
def test_in_place_closure_equals_two_copies(storage):
    """The learned closure's collision pass in place: bitwise the two-copy
    result, with ranges that send part of the interface sites to the network
    and the rest to the explicit scan."""
    say(f"case in place closure {storage}")
    shape = (64, 32, 24)
    kw = dict(lattice="D3Q27", storage=storage, nc="mlp", shape=shape, walls=(0, 1, 1), tau=1.0)
    cen = [[22.13, 16.21, 11.87], [41.6, 15.79, 12.09]]
    th = W.closure_init_weights(seed=3)
    lo = np.full(30, -2.0, np.float32)
    hi = np.full(30, 2.0, np.float32)
    hi[13] = 0.0                       # centre phase above 0: explicit scan
    sims = []
    for mode in ("two_copies", "in_place"):
        s = lb.Simulation(streaming=mode, **kw)
        s.mlp_set_weights(th)
        s.mlp_set_ranges(lo, hi, 0.0)
        s.init_droplets(cen, [8.0, 8.0])
        sims.append(s)
    for n in (3, 2):
        for s in sims:
            s.step(n)
        _same(*sims)
    fl = sims[1].fields(("flags",))["flags"]
    n_net, n_exp = int(((fl & 2) > 0).sum()), int(((fl & 4) > 0).sum())
    say(f"  network sites {n_net}, explicit-scan sites {n_exp}")
    assert n_net > 50 and n_exp > 50
    for s in sims:
        s.close()


def test_in_place_full_size_channel():
    """The 256 x 128 x 128 D3Q27 channel with 64 droplets (walls y, z, body
    force, explicit near contact) in FP16 total layout: in place bitwise equal
    to two copies after 3 steps, at the launch configuration of the timing."""
    w = W.channel_3d(storage="f16t")
    kw, cen, rad = W.sim_kwargs(w)
    say(f"case in place full size {kw['shape']} f16t")
    ab = lb.Simulation(**kw).init_droplets(cen, rad)
    ip = lb.Simulation(streaming="in_place", **kw).init_droplets(cen, rad)
    ab.step(3)
    ip.step(3)
    _same(ab, ip)
    ab.close()
    ip.close()

