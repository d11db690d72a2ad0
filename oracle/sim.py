"""Vectorised FP64 oracle of one colour-gradient LB time step (test infrastructure).

The state between steps is the post-collision population pair f^A_i, f^B_i,
stored as numpy arrays of shape (q, nz, ny, nx) (x fastest).  One ``step()``
performs, for every fluid site and in this order:

1.  pull streaming  f~^k_i(x) = f^k_i(x - c_i)                 [Eq. lbm, Eq. CGLBE]
    periodic axes wrap (Sec. III.D "Periodic boundary conditions");
    walled axes use halfway bounce-back: if x - c_i is a solid node then
    f~^k_i(x) = f^k_opp(i)(x) (Sec. III.D "No-slip", wall between grid lines)
2.  moments  rho_k = sum_i f~^k_i, rho = rho_A + rho_B,
    phi = (rho_A - rho_B) / rho, j = sum_k sum_i f~^k_i c_i   [Sec. III.C.1; Eq. order_param]
3.  phase-field ghosts at solid nodes: mirror of the fluid node across the
    wall plane (zero normal gradient, cf. the phase-field wall conditions)
4.  colour gradient g = (1/c_s^2) sum_i w_i c_i phi(x + c_i)   [isotropic stencil,
    Taylor expansion in the pseudo-potential section]
5.  interface flags I = |phi| < phi_I
6.  near-contact force F_nc (Eq. near_cont_force, see ``near_contact_force``)
7.  F = F_body + F_nc, u = (j + F/2) / rho                     [Guo forcing]
8.  BGK on the total f = f~^A + f~^B with Guo source           [Eq. disteq]
    at the local relaxation time of the mixture, 1/nu = (rho_A/rho)/nu_A +
    (rho_B/rho)/nu_B, tau = 3 nu + 1/2 (the mixing rule under Eq. sigmaA);
    one viscosity (tau_b = 0) gives tau everywhere
9.  perturbation f* = f + A|g| [w_i (c_i.g)^2/|g|^2 - B_i]     [Omega^(2), A_A = A_B = A]
10. recolouring f^A = (rho_A/rho) f* + beta rho_A rho_B / rho w_i cos(theta_i)
                f^B = (rho_B/rho) f* - beta rho_A rho_B / rho w_i cos(theta_i)
                                                               [Eqs. ome3_1, ome3_2]

Readings where the paper is silent (each listed in the design notes):
Guo forcing for the forcing term the paper leaves open; B_0 = w_0 - 2/3, B_i = w_i;
surface tension sigma = (2/9)(A_A + A_B) tau (the printed omega-bar is read
as 2/(6 nu + 1) = 1/tau); cos(theta) = 0 for the rest direction or g = 0;
the near-contact scan of ``near_contact_force``; halfway bounce-back walls.

Collision on the total is exact: BGK of each colour toward f^eq(rho_k, u) sums
to BGK of the total toward f^eq(rho, u) because f^eq is linear in rho, and the
recolouring only reads the total f*.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
import math

import numpy as np

from .lattice import make_lattice, Lattice
from . import ccl as _ccl


@dataclass
class OracleParams:
    lattice: str = "D3Q27"
    nx: int = 32
    ny: int = 32
    nz: int = 32
    walls: tuple = (False, False, False)   # halfway bounce-back on both faces of that axis
    tau: float = 1.0                       # relaxation time of colour A (of both if tau_b == 0)
    tau_b: float = 0.0                     # relaxation time of colour B; 0: same as tau
    A: float = 0.01                        # perturbation amplitude A = A_A = A_B
    beta: float = 0.7                      # recolouring parameter
    rho0: float = 1.0
    body_force: tuple = (0.0, 0.0, 0.0)    # force density
    u0: tuple = (0.0, 0.0, 0.0)            # uniform initial velocity
    nc: bool = False                       # explicit near-contact force on/off
    nc_A: float = 0.02                     # A_h plateau value
    nc_hmin: float = 2.0
    nc_hmax: float = 3.0
    phi_interface: float = 0.9
    # |g| at or below g_eps counts as no gradient: the normal, cos(theta_i),
    # the perturbation and the near-contact scan are then skipped.  A phase
    # gradient of 1e-12 is rounding noise at symmetric points (a droplet
    # centre on a site), where the direction of g would otherwise be random.
    g_eps: float = 1e-12
    # precision in which integer-valued decisions (flag threshold, rounding of
    # scan offsets, sign tests) are taken; float32 when comparing a float32 run
    decision_dtype: type = np.float64
    # learned closure (oracle.mlp.Closure) replacing the explicit scan at
    # interface sites whose stencil lies in its training range; needs nc=True
    closure: object = None

    def replace(self, **kw):
        return replace(self, **kw)


def round_half_away(v):
    """Round to nearest integer, halves away from zero."""
    return np.sign(v) * np.floor(np.abs(v) + 0.5)


def flags_from_phi(phi, phi_interface, dtype=np.float64):
    """I(x) = |phi(x)| < phi_I, decided in ``dtype``."""
    return np.abs(np.asarray(phi, dtype=dtype)) < dtype(phi_interface)


class OracleSim:
    """Whole-array FP64 colour-gradient LB solver (plain and slow by design)."""

    def __init__(self, params: OracleParams):
        p = params
        self.p = p
        self.lat: Lattice = make_lattice(p.lattice)
        if self.lat.d == 2 and p.nz != 1:
            raise ValueError("D2Q9 needs nz == 1")
        if p.tau <= 0.5:
            raise ValueError("tau must exceed 1/2")
        if p.tau_b and p.tau_b <= 0.5:
            raise ValueError("tau_b must exceed 1/2 (or be 0)")
        self.shape = (p.nz, p.ny, p.nx)
        self.n = (p.nx, p.ny, p.nz)
        self.walls = tuple(bool(b) for b in p.walls)
        if self.lat.d == 2 and self.walls[2]:
            raise ValueError("no z walls in 2D")
        L = self.lat
        self.c = L.c.astype(np.float64)
        self.w = L.w
        self.B = L.B
        self.t = 0
        q = L.q
        self.fA = np.zeros((q,) + self.shape)
        self.fB = np.zeros((q,) + self.shape)
        self._solid_src = self._make_solid_masks()
        self._fields = None

    # ----------------------------------------------------------------- geometry
    def _coords(self):
        z, y, x = np.meshgrid(np.arange(self.p.nz), np.arange(self.p.ny),
                              np.arange(self.p.nx), indexing="ij")
        return x, y, z

    def _make_solid_masks(self):
        """mask[i] is True where the upstream node x - c_i is solid."""
        x, y, z = self._coords()
        pos = (x, y, z)
        masks = []
        for i in range(self.lat.q):
            m = np.zeros(self.shape, dtype=bool)
            for a in range(3):
                if self.walls[a]:
                    src = pos[a] - self.lat.c[i, a]
                    m |= (src < 0) | (src >= self.n[a])
            masks.append(m)
        return masks

    # ---------------------------------------------------------------- equilibrium
    def equilibrium(self, rho, u):
        """f^eq_i = w_i rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)]  (Eq. disteq)."""
        cu = np.einsum("ia,a...->i...", self.c, u)
        uu = (u * u).sum(0)
        w = self.w.reshape((-1,) + (1,) * rho.ndim)
        return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)

    # ------------------------------------------------------------------- init
    def init_droplets(self, centres, radii, width=2.0, phi_in=1.0):
        """phi = phi_in * max_d tanh(2 (R_d - r_d) / width); rho_A = rho0 (1+phi)/2,
        rho_B = rho0 (1-phi)/2; f^k = f^eq(rho_k, u0).  Distances use the minimum
        image on periodic axes (tanh profile: free-energy section)."""
        p = self.p
        x, y, z = self._coords()
        pos = (x.astype(np.float64), y.astype(np.float64), z.astype(np.float64))
        best = np.full(self.shape, -np.inf)
        centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
        radii = np.asarray(radii, dtype=np.float64).reshape(-1)
        dims = 2 if self.lat.d == 2 else 3
        for cen, R in zip(centres, radii):
            r2 = np.zeros(self.shape)
            for a in range(dims):
                d = pos[a] - cen[a]
                if not self.walls[a]:
                    d = d - self.n[a] * np.round(d / self.n[a])
                r2 = r2 + d * d
            best = np.maximum(best, R - np.sqrt(r2))
        phi = phi_in * np.tanh(2.0 * best / width)
        rho_a = p.rho0 * (1.0 + phi) / 2.0
        rho_b = p.rho0 * (1.0 - phi) / 2.0
        u = np.broadcast_to(np.asarray(p.u0, dtype=np.float64).reshape(3, 1, 1, 1),
                            (3,) + self.shape).copy()
        self.fA = self.equilibrium(rho_a, u)
        self.fB = self.equilibrium(rho_b, u)
        self.t = 0
        self._fields = dict(rho_a=rho_a, rho_b=rho_b, phi=phi, u=u,
                            f_nc=np.zeros((3,) + self.shape),
                            flags=flags_from_phi(phi, p.phi_interface, p.decision_dtype),
                            nc_source=np.zeros(self.shape, dtype=np.uint8))
        return self

    def set_state(self, fA, fB, t=0):
        self.fA = np.array(fA, dtype=np.float64).reshape(self.fA.shape)
        self.fB = np.array(fB, dtype=np.float64).reshape(self.fB.shape)
        self.t = t
        self._fields = None
        return self

    # ---------------------------------------------------------------- streaming
    def pull(self, f):
        """f~_i(x) = f_i(x - c_i); periodic wrap; halfway bounce-back at walls."""
        out = np.empty_like(f)
        for i in range(self.lat.q):
            cx, cy, cz = (int(v) for v in self.lat.c[i])
            out[i] = np.roll(f[i], shift=(cz, cy, cx), axis=(0, 1, 2))
            m = self._solid_src[i]
            if m.any():
                out[i][m] = f[self.lat.opp[i]][m]
        return out

    # ------------------------------------------------------------------ gradient
    def pad_phi(self, phi, r):
        """phi with r ghost layers: wrap on periodic axes, mirror across the
        wall plane on walled axes (ghost at -1-k equals fluid node k)."""
        out = phi
        for a in range(3):
            ax = 2 - a   # array axis of spatial axis a (z, y, x order)
            widths = [(0, 0)] * 3
            widths[ax] = (r, r)
            out = np.pad(out, widths, mode="symmetric" if self.walls[a] else "wrap")
        return out

    def gradient(self, phi):
        """g(x) = (1/c_s^2) sum_i w_i c_i phi(x + c_i) over the run's own lattice."""
        P = self.pad_phi(phi, 1)
        nz, ny, nx = self.shape
        g = np.zeros((3,) + self.shape)
        for i in range(self.lat.q):
            cx, cy, cz = (int(v) for v in self.lat.c[i])
            if cx == 0 and cy == 0 and cz == 0:
                continue
            sh = P[1 + cz:1 + cz + nz, 1 + cy:1 + cy + ny, 1 + cx:1 + cx + nx]
            for a in range(3):
                if self.c[i, a] != 0:
                    g[a] += 3.0 * self.w[i] * self.c[i, a] * sh
        return g

    # ------------------------------------------------------------ near contact
    def near_contact_force(self, phi, g, flags):
        """Explicit near-contact repulsion, F_rep = -A_h[h] n delta_I (Eq.
        near_cont_force) with delta_I = |g|/2 and the sign chosen repulsive.

        For an interface site x (flag set, |g| > g_eps): m = -g/|g| points out of
        the phi = +1 region.  For s = 1 .. floor(h_max): y = x + round(s m)
        (halves away from zero).  A solid y ends the scan with no force;
        periodic axes wrap.  The first y that is an interface site whose
        gradient opposes g(x) (g(y).g(x) < 0) gives h = s and
        F_nc = (A_h(h)/2) g(x), A_h = A for h <= h_min, A (h_min/h)^3 above."""
        p = self.p
        F = np.zeros((3,) + self.shape)
        self._nc_source = np.zeros(self.shape, dtype=np.uint8)
        if not p.nc:
            return F
        dt = p.decision_dtype
        gg = (g * g).sum(0)
        cand = flags & (gg > p.g_eps ** 2)
        iz, iy, ix = np.nonzero(cand)
        if iz.size == 0:
            return F
        gx = g[:, iz, iy, ix]
        gn = np.sqrt(gg[iz, iy, ix])
        m = (-gx / gn).astype(dt)
        pos0 = (ix, iy, iz)
        active = np.ones(iz.size, dtype=bool)
        hfound = np.zeros(iz.size)
        for s in range(1, int(math.floor(p.nc_hmax)) + 1):
            off = round_half_away(dt(s) * m).astype(np.int64)
            coords = []
            for a in range(3):
                ca = pos0[a] + off[a]
                if self.walls[a]:
                    solid = (ca < 0) | (ca >= self.n[a])
                    active &= ~solid
                    ca = np.clip(ca, 0, self.n[a] - 1)
                else:
                    ca = np.mod(ca, self.n[a])
                coords.append(ca)
            yx, yy, yz = coords
            gy = g[:, yz, yy, yx]
            dot = (np.asarray(gy, dtype=dt) * np.asarray(gx, dtype=dt)).sum(0)
            hit = active & flags[yz, yy, yx] & (dot < 0)
            hfound[hit] = s
            active &= ~hit
        h = hfound
        got = h > 0
        Ah = np.where(h <= p.nc_hmin, p.nc_A, p.nc_A * (p.nc_hmin / np.where(got, h, 1.0)) ** 3)
        Ah = np.where(got, Ah, 0.0)
        F[:, iz, iy, ix] = 0.5 * Ah * gx
        if p.closure is not None:
            # learned closure where the stencil is inside its training range;
            # the explicit force above stays at the other candidates
            from .mlp import stencil_inputs
            X, gn32 = stencil_inputs(self, phi, g, (iz, iy, ix))
            use = p.closure.in_range(X, gn32)
            src = np.zeros(self.shape, dtype=np.uint8)
            src[iz, iy, ix] = np.where(use, 1, 2)
            self._nc_source = src
            if use.any():
                Fm = p.nc_A * p.closure.force(X[use], gx[:, use])
                F[:, iz[use], iy[use], ix[use]] = Fm.T
        return F

    def relaxation_time(self, rho_a, rho_b):
        """Local relaxation time of the mixture (Sec. III.C.1, the mixing rule
        stated with the surface tension, Eq. sigmaA): the inverse viscosity is
        the density-weighted mean 1/nu = (rho_A/rho)/nu_A + (rho_B/rho)/nu_B
        with nu_k = c_s^2 (tau_k - 1/2), and tau = nu/c_s^2 + 1/2.  With one
        viscosity (tau_b == 0) this is tau at every site."""
        p = self.p
        if not p.tau_b:
            return p.tau
        rho = rho_a + rho_b
        inv_nu = (rho_a / rho) / viscosity(p.tau) + (rho_b / rho) / viscosity(p.tau_b)
        return 3.0 / inv_nu + 0.5

    # -------------------------------------------------------------------- step
    def step(self, n=1):
        for _ in range(n):
            self._step_once()
        return self

    def _step_once(self):
        p = self.p
        q = self.lat.q
        wq = self.w.reshape(q, 1, 1, 1)
        Bq = self.B.reshape(q, 1, 1, 1)
        cnorm = self.lat.cnorm.reshape(q, 1, 1, 1)
        # 1. streaming
        fA = self.pull(self.fA)
        fB = self.pull(self.fB)
        # 2. moments
        rho_a = fA.sum(0)
        rho_b = fB.sum(0)
        rho = rho_a + rho_b
        phi = (rho_a - rho_b) / rho
        f = fA + fB
        j = np.einsum("ia,i...->a...", self.c, f)
        # 3-5. gradient with mirrored ghosts, flags
        g = self.gradient(phi)
        flags = flags_from_phi(phi, p.phi_interface, p.decision_dtype)
        # 6. near contact
        f_nc = self.near_contact_force(phi, g, flags)
        # 7. force and velocity
        F = np.asarray(p.body_force, dtype=np.float64).reshape(3, 1, 1, 1) + f_nc
        u = (j + 0.5 * F) / rho
        # 8. BGK + Guo source on the total, at the mixture's relaxation time
        tau = self.relaxation_time(rho_a, rho_b)
        feq = self.equilibrium(rho, u)
        cu = np.einsum("ia,a...->i...", self.c, u)
        cF = np.einsum("ia,a...->i...", self.c, F)
        uF = (u * F).sum(0)
        S = (1.0 - 0.5 / tau) * wq * (3.0 * (cF - uF) + 9.0 * cu * cF)
        fpost = f - (f - feq) / tau + S
        # 9. perturbation
        gg = (g * g).sum(0)
        gn = np.sqrt(gg)
        cg = np.einsum("ia,a...->i...", self.c, g)
        has = gg > p.g_eps ** 2
        safe_gg = np.where(has, gg, 1.0)
        pert = np.where(has, p.A * gn * (wq * cg * cg / safe_gg - Bq), 0.0)
        fstar = fpost + pert
        # 10. recolouring
        safe_gn = np.where(has, gn, 1.0)
        safe_cn = np.where(cnorm > 0, cnorm, 1.0)
        cos = np.where(has & (cnorm > 0), cg / (safe_cn * safe_gn), 0.0)
        coef = p.beta * rho_a * rho_b / rho
        self.fA = (rho_a / rho) * fstar + coef * wq * cos
        self.fB = (rho_b / rho) * fstar - coef * wq * cos
        self.t += 1
        self._fields = dict(rho_a=rho_a, rho_b=rho_b, phi=phi, u=u, f_nc=f_nc, flags=flags,
                            nc_source=self._nc_source)

    # ------------------------------------------------------------- reporting
    def fields(self):
        """Macroscopic fields of the last step (the moments of the post-streaming
        populations, the force and velocity used by its collision), or of the
        initial state."""
        if self._fields is None:
            raise RuntimeError("no fields yet: call init_droplets() or step()")
        return self._fields

    def labels(self, phi=None):
        if phi is None:
            phi = self.fields()["phi"]
        return _ccl.label(phi > 0, periodic=tuple(not w for w in self.walls),
                          two_d=self.lat.d == 2)

    def diagnostics(self):
        """FP64 global sums: [sum rho_A, sum rho_B, sum j (3), max |u|, droplet
        count, Laplace pressure jump cs2 (<rho>_{phi>0.9} - <rho>_{phi<-0.9})]."""
        fl = self.fields()
        rho = fl["rho_a"] + fl["rho_b"]
        F = np.asarray(self.p.body_force, dtype=np.float64).reshape(3, 1, 1, 1) + fl["f_nc"]
        j = rho * fl["u"] - 0.5 * F
        umax = float(np.sqrt((fl["u"] ** 2).sum(0)).max())
        lab, count = self.labels()
        inside = fl["phi"] > 0.9
        outside = fl["phi"] < -0.9
        dp = float("nan")
        if inside.any() and outside.any():
            dp = (rho[inside].mean() - rho[outside].mean()) / 3.0
        return np.array([fl["rho_a"].sum(), fl["rho_b"].sum(), j[0].sum(), j[1].sum(),
                         j[2].sum(), umax, float(count), dp])

    def mass(self):
        """Per-colour mass of the stored post-collision state."""
        return float(self.fA.sum()), float(self.fB.sum())

    def momentum(self):
        f = self.fA + self.fB
        return np.einsum("ia,ijkl->a", self.c, f)


def surface_tension(A, tau):
    """sigma = (2/9)(A_A + A_B) tau with A_A = A_B = A (Eq. sigmaA, read with
    omega-bar = 1/tau)."""
    return 4.0 / 9.0 * A * tau


def viscosity(tau):
    """nu = c_s^2 (tau - 1/2)."""
    return (tau - 0.5) / 3.0


__all__ = ["OracleParams", "OracleSim", "round_half_away", "flags_from_phi",
           "surface_tension", "viscosity"]


def window_geometry(params: OracleParams, site, radius):
    """Index arrays (ix, iy, iz) of the window of half-width ``radius`` around
    ``site``, the site's position in it and the window's walled axes: walled
    axes are cut at the true walls, periodic axes wrap (whole when shorter
    than the window)."""
    p = params
    n = (p.nx, p.ny, p.nz)
    lat = make_lattice(p.lattice)
    idx = []
    centre = []
    walls = []
    for a in range(3):
        na, xa = n[a], int(site[a])
        if lat.d == 2 and a == 2:
            idx.append(np.array([0]))
            centre.append(0)
            walls.append(False)
            continue
        if p.walls[a]:
            lo, hi = max(0, xa - radius), min(na - 1, xa + radius)
            idx.append(np.arange(lo, hi + 1))
            centre.append(xa - lo)
            walls.append(True)
        elif na <= 2 * radius + 1:
            idx.append(np.arange(na))
            centre.append(xa)
            walls.append(False)
        else:
            idx.append(np.arange(xa - radius, xa + radius + 1) % na)
            centre.append(radius)
            walls.append(False)
    return tuple(idx), tuple(centre), tuple(walls)


def step_window(params: OracleParams, fA, fB, site, radius=6):
    """One step of the site at ``site`` = (x, y, z) from the full post-collision
    state (fA, fB) of shape (q, nz, ny, nx), computed by running the oracle on
    the window of half-width ``radius`` around it.

    The post-collision value at x depends on data within 5 sites only (pull
    radius 1 for the populations of the sites whose phase field enters the
    gradient at the near-contact scan points: 3 + 1 + 1), so with radius >= 6
    the window's own boundary (periodic wrap on periodic axes, a wall on
    walled axes, which coincides with the true wall where the window reaches
    it) cannot influence the centre.  fA and fB may also be callables that
    take the window's index arrays (iz, iy, ix) and return the window
    (q, len(iz), len(iy), len(ix)), for states too large to hold on the host.
    Returns (fA_site (q,), fB_site (q,), fields dict at the site)."""
    p = params
    (ix, iy, iz), centre, walls = window_geometry(p, site, radius)
    if callable(fA):
        wA, wB = fA(iz, iy, ix), fB(iz, iy, ix)
    else:
        sub = np.ix_(np.arange(fA.shape[0]), iz, iy, ix)
        wA, wB = np.asarray(fA)[sub], np.asarray(fB)[sub]
    wp = p.replace(nx=len(ix), ny=len(iy), nz=len(iz), walls=tuple(walls))
    sim = OracleSim(wp).set_state(np.asarray(wA, dtype=np.float64), np.asarray(wB, dtype=np.float64))
    sim.step()
    cx, cy, cz = centre
    fl = sim.fields()
    out = {k: (v[..., cz, cy, cx] if v.ndim == 3 else v[:, cz, cy, cx]) for k, v in fl.items()}
    return sim.fA[:, cz, cy, cx].copy(), sim.fB[:, cz, cy, cx].copy(), out
