"""Moment-based (regularised) colour-gradient step, FP64 (test infrastructure).

The paper's third group of memory strategies (Sec. IV.A) stores hydrodynamic
moments instead of populations and rebuilds the populations from them: the
non-equilibrium part is projected on the second-order Hermite subspace
(Eq. distnoneq), the post-collision populations are f^eq + (1 - omega) f^neq
(Eq. LBpostmom), and streaming moves these rebuilt populations (Eq. llb-pull).

Here that construction is applied to the two-component step of
``oracle.sim.OracleSim``: the pulled total population f~ enters the BGK part
only through its projection on the Hermite subspace of the first three
moments: density, the non-equilibrium momentum j - rho u (which is -F/2 with
the Guo velocity u = (j + F/2)/rho, and zero without forcing, where it drops
out of Eq. distnoneq) and the non-equilibrium momentum flux
    Pi^neq = sum_i f~_i c_i c_i - rho c_s^2 I - rho u u,
    f^neq_i = w_i [ 3 c_i.(j - rho u) + 4.5 (c_i c_i - I/3) : Pi^neq ],
so that the post-collision total is
    P_i = f^eq_i(rho, u) + (1 - omega) f^neq_i + S_i(u, F) + Omega^(2)_i
with the Guo source S, the perturbation Omega^(2) and the recolouring of the
standard step.  Every term is a second-order Hermite expansion plus one fixed
vector, so the post-collision colours are exact functions of a moment set M
of 15 numbers per site (2D: the z entries are zero):
    P_i   = w_i [ rho + 3 c_i.J + 4.5 (c_i c_i - I/3) : S ] + s V_i
    P^A_i = a P_i + (w_i / |c_i|) c_i . b,   P^B_i = P_i - P^A_i
with
    J = rho u + (1 - omega)(j - rho u) + (1 - omega/2) F   (= j + F)
    S = rho u u + (1 - omega) Pi^neq + (1 - omega/2)(u F + F u) + (2A/9) g g / |g|
    s = A |g|,  V_i = (2/3)(delta_i0 - w_i)
    a = rho_A / rho,  b = beta (rho_A rho_B / rho) g / |g|
(c_s^2 = 1/3; with B_0 = w_0 - 2/3 and B_i = w_i the perturbation
A|g|[w_i (c_i.g)^2/|g|^2 - B_i] splits as w_i 4.5 (c c - I/3) : (2A/9) g g/|g|
+ A|g| V_i).  Channel order of M:
    0 rho, 1-3 J, 4-6 S_xx S_yy S_zz, 7-9 S_xy S_xz S_yz, 10 s, 11 a, 12-14 b.
The state at t = 0 (equilibria at u0) is M with J = rho u0, S = rho u0 u0 and
s = b = 0.  A site with |g| <= g_eps has s = 0, b = 0 and no g g term.
"""
from __future__ import annotations

import numpy as np

from .sim import OracleSim

NM = 15
PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))   # S channels 4..9


def v_vector(lat):
    """V_i = (2/3)(delta_i0 - w_i)."""
    v = -(2.0 / 3.0) * lat.w
    v[0] += 2.0 / 3.0
    return v


class OracleLLB(OracleSim):
    """Whole-array FP64 moment-based colour-gradient solver; the state is the
    moment set ``self.M`` of shape (15, nz, ny, nx)."""

    def __init__(self, params):
        super().__init__(params)
        self.M = np.zeros((NM,) + self.shape)

    # --------------------------------------------------------------- state
    def init_droplets(self, centres, radii, width=2.0, phi_in=1.0):
        super().init_droplets(centres, radii, width, phi_in)
        rho_a, rho_b = self.fA.sum(0), self.fB.sum(0)
        rho = rho_a + rho_b
        u0 = np.asarray(self.p.u0, dtype=np.float64)
        M = np.zeros((NM,) + self.shape)
        M[0] = rho
        for a in range(3):
            M[1 + a] = rho * u0[a]
        for k, (a, b) in enumerate(PAIRS):
            M[4 + k] = rho * u0[a] * u0[b]
        M[11] = rho_a / rho
        self.M = M
        self.fA, self.fB = self.populations(M)
        return self

    def set_moments(self, M, t=0):
        self.M = np.array(M, dtype=np.float64)
        self.fA, self.fB = self.populations(self.M)
        self.t = t
        self._fields = None
        return self

    def populations(self, M):
        """Post-collision colours (P^A, P^B) of a moment set."""
        q = self.lat.q
        c = self.c
        w = self.w.reshape(q, 1, 1, 1)
        rho, J, s, a = M[0], M[1:4], M[10], M[11]
        b = M[12:15]
        cJ = np.einsum("ia,a...->i...", c, J)
        ccS = np.zeros((q,) + self.shape)
        for k, (x, y) in enumerate(PAIRS):
            mult = 1.0 if x == y else 2.0
            ccS += mult * np.einsum("i,...->i...", c[:, x] * c[:, y], M[4 + k])
        trS = M[4] + M[5] + M[6]
        P = w * (rho[None] + 3.0 * cJ + 4.5 * (ccS - trS[None] / 3.0)) \
            + v_vector(self.lat).reshape(q, 1, 1, 1) * s[None]
        cn = self.lat.cnorm.reshape(q, 1, 1, 1)
        inv = np.where(cn > 0, 1.0 / np.where(cn > 0, cn, 1.0), 0.0)
        cb = np.einsum("ia,a...->i...", c, b)
        PA = a[None] * P + w * inv * cb
        return PA, P - PA

    # ---------------------------------------------------------------- step
    def _step_once(self):
        p = self.p
        q = self.lat.q
        c = self.c
        # 1. stream the rebuilt post-collision colours
        fA = self.pull(self.fA)
        fB = self.pull(self.fB)
        # 2-7. moments, gradient, flags, near contact, force, velocity (as the
        # standard step)
        rho_a = fA.sum(0)
        rho_b = fB.sum(0)
        rho = rho_a + rho_b
        phi = (rho_a - rho_b) / rho
        f = fA + fB
        j = np.einsum("ia,i...->a...", c, f)
        g = self.gradient(phi)
        from .sim import flags_from_phi
        flags = flags_from_phi(phi, p.phi_interface, p.decision_dtype)
        f_nc = self.near_contact_force(phi, g, flags)
        F = np.asarray(p.body_force, dtype=np.float64).reshape(3, 1, 1, 1) + f_nc
        u = (j + 0.5 * F) / rho
        # 8. regularised BGK: f~ -> f^eq + f^neq(j - rho u, Pi^neq), Guo source
        tau = self.relaxation_time(rho_a, rho_b)
        om = 1.0 / tau
        gu = 1.0 - 0.5 * om
        Pi = np.einsum("ia,ib,i...->ab...", c, c, f)
        # 9-10. perturbation and recolouring enter through s, the g g term and b
        gg = (g * g).sum(0)
        has = gg > p.g_eps ** 2
        gn = np.sqrt(np.where(has, gg, 1.0))
        M = np.zeros((NM,) + self.shape)
        M[0] = rho
        for a in range(3):
            M[1 + a] = rho * u[a] + (1.0 - om) * (j[a] - rho * u[a]) + gu * F[a]
        for k, (a, b) in enumerate(PAIRS):
            # the isotropic pressure rho c_s^2 acts on the lattice's own axes
            iso = rho / 3.0 if (a == b and a < self.lat.d) else 0.0
            pin = Pi[a, b] - rho * u[a] * u[b] - iso
            ggt = np.where(has, g[a] * g[b] / gn, 0.0)
            M[4 + k] = rho * u[a] * u[b] + (1.0 - om) * pin + gu * (u[a] * F[b] + F[a] * u[b]) \
                + (2.0 * p.A / 9.0) * ggt
        M[10] = np.where(has, p.A * gn, 0.0)
        M[11] = rho_a / rho
        coef = p.beta * rho_a * rho_b / rho
        for a in range(3):
            M[12 + a] = np.where(has, coef * g[a] / gn, 0.0)
        self.M = M
        self.fA, self.fB = self.populations(M)
        self.t += 1
        self._fields = dict(rho_a=rho_a, rho_b=rho_b, phi=phi, u=u, f_nc=f_nc, flags=flags,
                            nc_source=self._nc_source)


def step_window_moments(params, M, site, radius=6):
    """One moment-scheme step of the site at ``site`` = (x, y, z) from the full
    moment state M (15, nz, ny, nx), run on the window of half-width
    ``radius`` around it (the new moments at x depend on the moments within 6
    sites: pull radius 1 for the phase field the gradient reads at the
    near-contact scan points, 3 + 1 + 1, as for the population step).  M may be
    a callable taking the window's index arrays (iz, iy, ix).  Returns (moments
    at the site (15,), fields dict at the site)."""
    from .sim import window_geometry
    (ix, iy, iz), centre, walls = window_geometry(params, site, radius)
    if callable(M):
        wM = M(iz, iy, ix)
    else:
        wM = np.asarray(M)[np.ix_(np.arange(NM), iz, iy, ix)]
    wp = params.replace(nx=len(ix), ny=len(iy), nz=len(iz), walls=walls)
    sim = OracleLLB(wp).set_moments(np.asarray(wM, dtype=np.float64))
    sim.step()
    cx, cy, cz = centre
    fl = sim.fields()
    out = {k: (v[..., cz, cy, cx] if v.ndim == 3 else v[:, cz, cy, cx]) for k, v in fl.items()}
    return sim.M[:, cz, cy, cx].copy(), out


__all__ = ["OracleLLB", "NM", "PAIRS", "v_vector", "step_window_moments"]
