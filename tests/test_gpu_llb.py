"""The moment-based (regularised) scheme through the C ABI against its FP64
oracle (oracle/llb.py).

The state is 15 moments per site; it is compared through the populations the
oracle rebuilds from it (scale O(w_i)), with the bars of the population
scheme: FP64 1e-12, FP32 1e-5 after 100 steps; flags bit-exact."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402
from oracle.llb import OracleLLB  # noqa: E402
from oracle.sim import OracleParams  # noqa: E402

U_FLOOR = 1e-2   # velocity bars relative to max(max |u|, 0.01), as for the population scheme


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oparams(kw, decision=np.float64):
    nx, ny, nz = kw["shape"]
    return OracleParams(lattice=kw["lattice"], nx=nx, ny=ny, nz=nz,
                        walls=tuple(bool(v) for v in kw.get("walls", (0, 0, 0))),
                        tau=kw.get("tau", 1.0), tau_b=kw.get("tau_b", 0.0), A=kw.get("A", 0.01),
                        beta=kw.get("beta", 0.7), body_force=tuple(kw.get("body_force", (0, 0, 0))),
                        u0=tuple(kw.get("u0", (0, 0, 0))), nc=kw.get("nc", "off") == "explicit",
                        nc_A=kw.get("nc_A", 0.02), decision_dtype=decision)


def gpu_moments(sim, rho0=1.0):
    M = sim.get_state().double().cpu().numpy()
    M[0] += rho0            # the library keeps rho - rho0
    return M


def rel(a, b):
    return np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-300)


def _pair(shape, d3):
    nx, ny, nz = shape
    R = min(6.0, ny * 0.3, (nz * 0.3 if d3 else 99))
    cen = np.array([[nx * 0.3 + 0.17, ny * 0.5 - 0.23, nz * 0.5 + 0.31 if d3 else 0.0],
                    [nx * 0.3 + 2 * R + 3.17, ny * 0.5 + 0.11, nz * 0.5 - 0.13 if d3 else 0.0]])
    return cen, [R, R]


def test_init_matches_oracle():
    kw = dict(lattice="D3Q27", storage="f64", scheme="moments", nc="explicit", shape=(37, 20, 13),
              walls=(0, 1, 1), u0=(0.01, -0.02, 0.005))
    cen, rad = _pair(kw["shape"], True)
    say("case llb init")
    sim = lb.Simulation(**kw).init_droplets(cen, rad)
    orc = OracleLLB(oparams(kw)).init_droplets(cen, rad)
    assert np.abs(gpu_moments(sim) - orc.M).max() < 1e-15
    sim.close()


CASES = [
    ("D2Q9", (70, 37, 1), (0, 1, 0), "explicit", 0.0, 200),
    ("D3Q19", (67, 21, 14), (0, 1, 1), "explicit", 0.0, 60),
    ("D3Q27", (70, 20, 13), (0, 1, 1), "explicit", 1.7, 60),
    ("D3Q27", (64, 8, 24), (1, 0, 0), "off", 0.0, 40),
    ("D3Q27", (33, 17, 9), (1, 1, 1), "explicit", 0.0, 40),
]


@pytest.mark.parametrize("lat,shape,walls,nc,tau_b,steps", CASES)
def test_fp64_parity(lat, shape, walls, nc, tau_b, steps):
    d3 = lat != "D2Q9"
    cen, rad = _pair(shape, d3)
    kw = dict(lattice=lat, storage="f64", scheme="moments", nc=nc, shape=shape, walls=walls, tau=0.9,
              tau_b=tau_b, A=0.02, body_force=(2e-5, 0, 0), nc_A=0.03)
    say(f"case llb fp64 {lat} {shape} walls={walls} nc={nc} tau_b={tau_b} steps={steps}")
    sim = lb.Simulation(**kw).init_droplets(cen, rad)
    orc = OracleLLB(oparams(kw)).init_droplets(cen, rad)
    sim.step(steps)
    orc.step(steps)
    PA, PB = orc.populations(gpu_moments(sim))
    ea, eb = rel(PA, orc.fA), rel(PB, orc.fB)
    g = {k: v.cpu().numpy() for k, v in sim.fields(("rho_a", "rho_b", "phi", "u", "f_nc", "flags")).items()}
    o = orc.fields()
    eu = np.abs(g["u"] - o["u"]).max() / max(np.abs(o["u"]).max(), U_FLOOR)
    say(f"  populations rel err A {ea:.2e} B {eb:.2e}, u {eu:.2e}, nc sites {(np.abs(o['f_nc']).sum(0) > 0).sum()}")
    assert ea < 1e-12 and eb < 1e-12 and eu < 1e-12
    for k in ("rho_a", "rho_b", "phi"):
        assert rel(g[k], o[k]) < 1e-12, k
    assert np.abs(g["f_nc"] - o["f_nc"]).max() <= 1e-12 * max(np.abs(o["f_nc"]).max(), 1e-30)
    assert np.array_equal(g["flags"].astype(bool), o["flags"])
    if nc == "explicit":
        assert np.abs(o["f_nc"]).max() > 0
    sim.close()


def test_fp32_parity_100_steps():
    kw = dict(lattice="D3Q27", storage="f32", scheme="moments", nc="explicit", shape=(40, 32, 32),
              walls=(0, 0, 0), u0=(0.02, 0.0, 0.0), body_force=(1e-6, 0.0, 0.0))
    cen = np.array([[11.13, 15.77, 16.21], [29.61, 16.19, 15.83]])
    say("case llb fp32 100 steps")
    sim = lb.Simulation(**kw).init_droplets(cen, [7.5, 7.5])
    orc = OracleLLB(oparams(kw, np.float32)).init_droplets(cen, [7.5, 7.5])
    sim.step(100)
    orc.step(100)
    g = {k: v.double().cpu().numpy() for k, v in sim.fields(("rho_a", "rho_b", "u")).items()}
    o = orc.fields()
    errs = {k: rel(g[k], o[k]) for k in ("rho_a", "rho_b")}
    errs["u"] = np.abs(g["u"] - o["u"]).max() / np.abs(o["u"]).max()
    PA, PB = orc.populations(gpu_moments(sim))
    errs["PA"], errs["PB"] = rel(PA, orc.fA), rel(PB, orc.fB)
    say(f"  llb fp32 errors {errs}")
    for k, e in errs.items():
        assert e < 1e-5, (k, e)
    sim.close()


def test_full_size_channel_conserves_and_keeps_droplets():
    """The 256 x 128 x 128 channel (walls y/z, body force, near contact) with
    the moment state in FP32: 200 steps keep every droplet, the colour masses
    to FP32 rounding, and finite fields."""
    w = W.channel_3d()
    kw, cen, rad = W.sim_kwargs(w)
    kw.update(scheme="moments")
    say(f"case llb full size {kw['shape']}")
    sim = lb.Simulation(**kw).init_droplets(cen, rad)
    d0 = sim.diagnostics()
    sim.step(200)
    d = sim.diagnostics()
    f = sim.fields(("rho_a", "u"))
    assert all(torch.isfinite(v).all() for v in f.values())
    say(f"  droplets {d0[6]:.0f} -> {d[6]:.0f}, mass drift A {abs(d[0] / d0[0] - 1):.2e}, umax {d[5]:.3e}")
    assert int(d[6]) == int(d0[6]) == len(rad)
    assert abs(d[0] / d0[0] - 1) < 1e-5 and abs(d[1] / d0[1] - 1) < 1e-5
    sim.close()


def test_full_size_sampled_sites():
    """The 256 x 128 x 128 channel with the FP32 moment state, in the launch
    configuration of the timing: one GPU step from a developed state against
    the oracle's windowed step at sampled sites (near-contact sites, the
    walls, tile edges, the periodic seam).  The populations rebuilt from the
    GPU's and the oracle's moments agree within 2e-6 of the population scale;
    flags are equal."""
    from oracle.llb import step_window_moments
    w = W.channel_3d()
    kw, cen, rad = W.sim_kwargs(w)
    kw.update(scheme="moments")
    say("case llb full size sampled sites")
    sim = lb.Simulation(**kw).init_droplets(cen, rad)
    sim.step(30)
    M0 = sim.get_state().clone()
    sim.step(1)
    M1 = sim.get_state()
    g = {k: v.cpu().numpy() for k, v in sim.fields(("f_nc", "flags")).items()}

    def gather(iz, iy, ix):
        dev = M0.device
        t = M0[:, torch.as_tensor(iz, device=dev)][:, :, torch.as_tensor(iy, device=dev)]
        t = t[:, :, :, torch.as_tensor(ix, device=dev)].double().cpu().numpy()
        t[0] += 1.0
        return t

    nx, ny, nz = kw["shape"]
    one = OracleLLB(OracleParams(lattice="D3Q27", nx=1, ny=1, nz=1))
    rng = np.random.default_rng(4)
    fnc_sites = np.argwhere(np.abs(g["f_nc"]).sum(0) > 0)
    assert len(fnc_sites) > 0
    sites = [tuple(int(v) for v in fnc_sites[j][::-1])
             for j in rng.choice(len(fnc_sites), size=min(12, len(fnc_sites)), replace=False)]
    sites += [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (63, 3, 7), (64, 4, 8), (200, 1, 1)]
    for _ in range(6):
        sites.append((int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))))
    p = oparams(kw, np.float32)
    worst = 0.0
    for (x, y, z) in sites:
        m, fl = step_window_moments(p, gather, (x, y, z))
        mg = M1[:, z, y, x].double().cpu().numpy()
        mg[0] += 1.0
        oa, ob = one.populations(m.reshape(-1, 1, 1, 1))
        ga, gb = one.populations(mg.reshape(-1, 1, 1, 1))
        e = max(np.abs(ga - oa).max(), np.abs(gb - ob).max()) / np.abs(oa + ob).max()
        worst = max(worst, e)
        assert e < 2e-6, ((x, y, z), e)
        assert bool(g["flags"][z, y, x]) == bool(fl["flags"]), (x, y, z)
    say(f"  llb: sampled {len(sites)} sites, worst rel err {worst:.2e}")
    sim.close()


@pytest.mark.parametrize("centre", [(64.3, 32.2), (64.0, 32.0)])
def test_laplace_case_fp64_1000_steps(centre):
    """The 128 x 64 D2Q9 single-droplet case (R = 16, tau 1, A 0.01, beta 0.7)
    in the moment scheme, FP64, 1000 steps: the Laplace jump agrees with the
    oracle and lies within 10% of sigma / R.

    Off the lattice's symmetry points the state agrees within 1e-12.  With the
    centre on a site, every site on the mirror axes far from the droplet has a
    colour gradient that is zero by symmetry and made of rounding only; the
    GPU's shifted sums (rho_A - rho0/2, about 1e-16 absolute per step on a
    colour-A density near 1e-10 there) and the oracle's unshifted ones drift
    apart at 1e-14, and at a few such sites one side's |g|^2 crosses the
    1e-24 no-gradient threshold and the other's does not, which sets or
    clears the recolouring vector b (about 1e-10 there).  That case is held
    to the Laplace jump only."""
    from oracle.sim import surface_tension
    kw = dict(lattice="D2Q9", storage="f64", scheme="moments", nc="off", shape=(128, 64, 1), walls=(0, 0, 0),
              tau=1.0, A=0.01, beta=0.7)
    cen = [[centre[0], centre[1], 0.0]]
    say(f"case llb laplace d2q9 1000 steps centre {centre}")
    sim = lb.Simulation(**kw).init_droplets(cen, [16.0])
    orc = OracleLLB(oparams(kw)).init_droplets(cen, [16.0])
    sim.step(1000)
    orc.step(1000)
    PA, PB = orc.populations(gpu_moments(sim))
    e = max(rel(PA, orc.fA), rel(PB, orc.fB))
    dp_g, dp_o = sim.diagnostics()[7], orc.diagnostics()[7]
    sigma = surface_tension(0.01, 1.0)
    say(f"  populations rel err {e:.2e}; Laplace jump {dp_g:.9e} (oracle {dp_o:.9e}, sigma/R {sigma / 16:.6e})")
    on_site = centre[0] == int(centre[0]) and centre[1] == int(centre[1])
    if not on_site:
        assert e < 1e-12
        assert abs(dp_g - dp_o) <= 1e-12 * abs(dp_o)
    else:
        assert abs(dp_g - dp_o) <= 1e-6 * abs(dp_o)
    assert abs(dp_g / (sigma / 16) - 1) < 0.10
    sim.close()
