"""Pins of the moment-based (regularised) colour-gradient oracle (oracle/llb.py).

- the populations rebuilt from a moment set carry exactly its moments
  (Hermite orthogonality of the lattices: sum P = rho, sum P c = J,
  sum P c c = rho c_s^2 I + S - (2/9) s I, sum P^A = a rho);
- on states whose pulled populations already lie in the second-order Hermite
  subspace (uniform states), the regularised step is the standard step;
- per-colour mass is conserved to rounding with walls and near contact;
- shear waves decay at nu = c_s^2 (tau - 1/2), and the Laplace law holds with
  the surface tension of the standard scheme."""
import numpy as np
import pytest

from oracle.lattice import make_lattice
from oracle.llb import NM, PAIRS, OracleLLB
from oracle.sim import OracleParams, OracleSim, surface_tension, viscosity


def _random_moments(rng, lat, shape, grad=True):
    d = lat.d
    M = np.zeros((NM,) + shape)
    M[0] = rng.uniform(0.9, 1.1, shape)
    for a in range(d):
        M[1 + a] = rng.uniform(-0.03, 0.03, shape)
    for k, (a, b) in enumerate(PAIRS):
        if a < d and b < d:
            M[4 + k] = rng.uniform(-0.01, 0.01, shape)
    M[11] = rng.uniform(0.0, 1.0, shape)
    if grad:
        M[10] = rng.uniform(0.0, 0.005, shape)
        for a in range(d):
            M[12 + a] = rng.uniform(-0.05, 0.05, shape)
    return M


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19", "D3Q27"])
def test_rebuilt_populations_carry_the_moments(name):
    lat = make_lattice(name)
    d = lat.d
    shape = (3, 4, 5) if d == 3 else (1, 4, 5)
    p = OracleParams(lattice=name, nx=5, ny=4, nz=shape[0])
    sim = OracleLLB(p)
    M = _random_moments(np.random.default_rng(3), lat, shape)
    PA, PB = sim.populations(M)
    P = PA + PB
    c = lat.c.astype(float)
    np.testing.assert_allclose(P.sum(0), M[0], atol=1e-15)
    np.testing.assert_allclose(PA.sum(0), M[11] * M[0], atol=1e-15)
    for a in range(3):
        np.testing.assert_allclose(np.einsum("i,i...->...", c[:, a], P), M[1 + a], atol=1e-15)
    for k, (a, b) in enumerate(PAIRS):
        want = M[4 + k] + ((M[0] / 3.0 - 2.0 / 9.0 * M[10]) if (a == b and a < d) else 0.0)
        np.testing.assert_allclose(np.einsum("i,i...->...", c[:, a] * c[:, b], P), want, atol=1e-15)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q27"])
def test_uniform_state_regularised_step_is_the_standard_step(name):
    """A uniform state (no gradient, so no perturbation and a proportional
    recolouring) pulls populations that are their own Hermite projection:
    one regularised step equals one standard step, forcing included."""
    lat = make_lattice(name)
    nz = 1 if name == "D2Q9" else 3
    shape = (nz, 4, 5)
    p = OracleParams(lattice=name, nx=5, ny=4, nz=nz, tau=0.8, A=0.02, beta=0.7,
                     body_force=(2e-4, -1e-4, 5e-5 if nz > 1 else 0.0))
    rng = np.random.default_rng(9)
    one = _random_moments(rng, lat, (1, 1, 1), grad=False)
    M = np.broadcast_to(one, (NM,) + shape).copy()
    llb = OracleLLB(p).set_moments(M)
    std = OracleSim(p).set_state(*llb.populations(M))
    llb.step()
    std.step()
    np.testing.assert_allclose(llb.fA, std.fA, rtol=0, atol=1e-15)
    np.testing.assert_allclose(llb.fB, std.fB, rtol=0, atol=1e-15)


def test_mass_per_colour_conserved_with_walls_and_near_contact():
    p = OracleParams(lattice="D3Q19", nx=30, ny=20, nz=16, walls=(False, True, True), tau=0.9,
                     tau_b=1.3, A=0.01, beta=0.7, body_force=(1e-5, 0, 0), nc=True)
    sim = OracleLLB(p).init_droplets([[9.3, 10.2, 7.9], [21.1, 9.8, 8.2]], [4.5, 4.5])
    m0 = sim.fA.sum(), sim.fB.sum()
    sim.step(300)
    assert abs(sim.fA.sum() / m0[0] - 1) < 1e-13
    assert abs(sim.fB.sum() / m0[1] - 1) < 1e-13
    assert np.abs(sim.fields()["f_nc"]).max() > 0


@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_shear_wave_viscosity(tau):
    Ly = 64
    p = OracleParams(lattice="D2Q9", nx=2, ny=Ly, nz=1, tau=tau, A=0.0, beta=0.0)
    sim = OracleLLB(p)
    k = 2 * np.pi / Ly
    M = np.zeros((NM, 1, Ly, 2))
    M[0] = 1.0
    M[1] = (1e-3 * np.sin(k * np.arange(Ly))).reshape(1, Ly, 1)
    M[4] = M[1] ** 2
    M[11] = 1.0
    sim.set_moments(M)
    amps = []
    for t in range(400):
        sim.step()
        if t >= 50 and t % 25 == 0:
            ux = sim.fields()["u"][0, 0, :, 0]
            amps.append((t + 1, 2 / Ly * np.sum(ux * np.sin(k * np.arange(Ly)))))
    ts = np.array([a[0] for a in amps], float)
    nu_fit = -np.polyfit(ts, np.log([a[1] for a in amps]), 1)[0] / k ** 2
    assert abs(nu_fit / viscosity(tau) - 1) < 0.01, nu_fit


def test_laplace_law_2d_slope():
    """Delta p = sigma / R with the standard scheme's sigma = (4/9) A tau: the
    perturbation's second moment survives the projection."""
    Rs = np.array([8.0, 10.0, 12.0, 16.0])
    dps = []
    for R in Rs:
        p = OracleParams(lattice="D2Q9", nx=64, ny=64, nz=1, tau=1.0, A=0.01, beta=0.7)
        sim = OracleLLB(p).init_droplets([(32, 32, 0)], [R]).step(1200)
        dps.append(sim.diagnostics()[7])
    slope = np.polyfit(1 / Rs, np.array(dps), 1)[0]
    assert abs(slope / surface_tension(0.01, 1.0) - 1) < 0.05, (slope, dps)


def test_droplet_close_to_the_standard_scheme():
    """Same droplet, 200 steps: the regularised and the standard scheme place
    the interface alike (phase field within 0.01 everywhere)."""
    p = OracleParams(lattice="D2Q9", nx=64, ny=48, nz=1, walls=(False, True, False), tau=0.9, A=0.01,
                     beta=0.7, body_force=(1e-5, 0, 0))
    a = OracleLLB(p).init_droplets([(30.3, 23.8, 0)], [10.0]).step(200)
    b = OracleSim(p).init_droplets([(30.3, 23.8, 0)], [10.0]).step(200)
    assert np.abs(a.fields()["phi"] - b.fields()["phi"]).max() < 0.01


def test_window_step_equals_the_full_step():
    """One step on a radius-6 window reproduces the full lattice's step at
    the window's centre (population and moment schemes), near walls,
    across the periodic seam and at near-contact sites."""
    from oracle.llb import step_window_moments
    from oracle.sim import step_window
    p = OracleParams(lattice="D3Q27", nx=30, ny=20, nz=18, walls=(False, True, True), tau=0.9, A=0.02,
                     beta=0.7, body_force=(1e-5, 0, 0), nc=True, nc_A=0.03)
    cen = [[9.3, 10.2, 8.9], [19.1, 9.8, 9.2]]
    full = OracleLLB(p).init_droplets(cen, [4.5, 4.5]).step(20)
    M0 = full.M.copy()
    fA0, fB0 = full.fA.copy(), full.fB.copy()
    full.step()
    std = OracleSim(p).set_state(fA0, fB0).step()
    fnc = np.argwhere(np.abs(full.fields()["f_nc"]).sum(0) > 0)
    assert len(fnc) > 0
    sites = [(0, 0, 0), (29, 19, 17), (14, 1, 9), tuple(int(v) for v in fnc[0][::-1])]
    for x, y, z in sites:
        m, _ = step_window_moments(p, M0, (x, y, z))
        np.testing.assert_allclose(m, full.M[:, z, y, x], rtol=0, atol=1e-15)
        a, b, _ = step_window(p, fA0, fB0, (x, y, z))
        np.testing.assert_allclose(a, std.fA[:, z, y, x], rtol=0, atol=1e-15)
        np.testing.assert_allclose(b, std.fB[:, z, y, x], rtol=0, atol=1e-15)
