"""Per-site Python-loop step for tiny lattices (test infrastructure).

An independent second statement of the step of ``oracle.sim`` (same paper
passages, same readings), written site by site and direction by direction
with plain Python floats and its own velocity tables, so that a slip in the
whole-array bookkeeping of ``sim`` (a wrong roll direction, a transposed
einsum, a mis-padded ghost layer) shows up as a disagreement on 4x4 / 4x4x4
random states.  It shares only the velocity tables' *definition* with ``sim``.
"""
from __future__ import annotations

import math

from .lattice import make_lattice


def _rha(v):
    return math.copysign(math.floor(abs(v) + 0.5), v) if v != 0 else 0.0


class NaiveSim:
    def __init__(self, params):
        self.p = params
        lat = make_lattice(params.lattice)
        self.q = lat.q
        self.d = lat.d
        self.c = [tuple(int(a) for a in row) for row in lat.c.tolist()]
        self.w = [float(x) for x in lat.w_exact]
        self.B = [float(x) for x in lat.b_exact]
        self.opp = [int(o) for o in lat.opp]
        self.n = (params.nx, params.ny, params.nz)
        self.walls = tuple(bool(b) for b in params.walls)

    # site helpers -------------------------------------------------------
    def idx(self, x, y, z):
        nx, ny, _ = self.n
        return x + nx * (y + ny * z)

    def wrap_or_none(self, pos):
        out = []
        for a in range(3):
            v = pos[a]
            if v < 0 or v >= self.n[a]:
                if self.walls[a]:
                    return None
                v %= self.n[a]
            out.append(v)
        return tuple(out)

    def ghost(self, pos):
        """Coordinate used for phi at pos: wrap periodic, mirror across walls."""
        out = []
        for a in range(3):
            v = pos[a]
            n = self.n[a]
            if self.walls[a]:
                if v < 0:
                    v = -1 - v
                elif v >= n:
                    v = 2 * n - 1 - v
            else:
                v %= n
            out.append(v)
        return tuple(out)

    def sites(self):
        nx, ny, nz = self.n
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    yield (x, y, z)

    # one step -------------------------------------------------------------
    def step(self, fA, fB):
        """fA, fB: lists (q) of lists (N) of floats (post-collision).  Returns the
        new post-collision lists and a dict of per-site fields."""
        p = self.p
        q = self.q
        N = self.n[0] * self.n[1] * self.n[2]
        pulled_A = [[0.0] * N for _ in range(q)]
        pulled_B = [[0.0] * N for _ in range(q)]
        for (x, y, z) in self.sites():
            s = self.idx(x, y, z)
            for i in range(q):
                cx, cy, cz = self.c[i]
                src = self.wrap_or_none((x - cx, y - cy, z - cz))
                if src is None:
                    pulled_A[i][s] = fA[self.opp[i]][s]
                    pulled_B[i][s] = fB[self.opp[i]][s]
                else:
                    t = self.idx(*src)
                    pulled_A[i][s] = fA[i][t]
                    pulled_B[i][s] = fB[i][t]
        rhoA = [0.0] * N
        rhoB = [0.0] * N
        phi = [0.0] * N
        for s in range(N):
            ra = sum(pulled_A[i][s] for i in range(q))
            rb = sum(pulled_B[i][s] for i in range(q))
            rhoA[s], rhoB[s] = ra, rb
            phi[s] = (ra - rb) / (ra + rb)
        grad = [None] * N
        flag = [False] * N
        for (x, y, z) in self.sites():
            s = self.idx(x, y, z)
            gv = [0.0, 0.0, 0.0]
            for i in range(q):
                cx, cy, cz = self.c[i]
                t = self.idx(*self.ghost((x + cx, y + cy, z + cz)))
                gv[0] += 3.0 * self.w[i] * cx * phi[t]
                gv[1] += 3.0 * self.w[i] * cy * phi[t]
                gv[2] += 3.0 * self.w[i] * cz * phi[t]
            grad[s] = gv
            flag[s] = abs(phi[s]) < p.phi_interface
        newA = [[0.0] * N for _ in range(q)]
        newB = [[0.0] * N for _ in range(q)]
        fields = dict(phi=phi, rho_a=rhoA, rho_b=rhoB, u=[None] * N, f_nc=[None] * N,
                      flags=flag)
        for (x, y, z) in self.sites():
            s = self.idx(x, y, z)
            g = grad[s]
            gg = g[0] * g[0] + g[1] * g[1] + g[2] * g[2]
            # near-contact scan
            fnc = [0.0, 0.0, 0.0]
            if p.nc and flag[s] and gg > p.g_eps ** 2:
                gn = math.sqrt(gg)
                m = [-g[a] / gn for a in range(3)]
                for step in range(1, int(math.floor(p.nc_hmax)) + 1):
                    off = [int(_rha(step * m[a])) for a in range(3)]
                    tgt = self.wrap_or_none((x + off[0], y + off[1], z + off[2]))
                    if tgt is None:
                        break
                    t = self.idx(*tgt)
                    g2 = grad[t]
                    if flag[t] and (g2[0] * g[0] + g2[1] * g[1] + g2[2] * g[2]) < 0:
                        h = float(step)
                        Ah = p.nc_A if h <= p.nc_hmin else p.nc_A * (p.nc_hmin / h) ** 3
                        fnc = [0.5 * Ah * g[a] for a in range(3)]
                        break
            F = [p.body_force[a] + fnc[a] for a in range(3)]
            rho = rhoA[s] + rhoB[s]
            tau = p.tau
            if p.tau_b:
                # harmonic mean of the colours' viscosities, weighted by density
                nu_a, nu_b = (p.tau - 0.5) / 3.0, (p.tau_b - 0.5) / 3.0
                tau = 3.0 / (rhoA[s] / (rho * nu_a) + rhoB[s] / (rho * nu_b)) + 0.5
            pre = 1.0 - 0.5 / tau
            f = [pulled_A[i][s] + pulled_B[i][s] for i in range(q)]
            j = [sum(f[i] * self.c[i][a] for i in range(q)) for a in range(3)]
            u = [(j[a] + 0.5 * F[a]) / rho for a in range(3)]
            uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
            uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2]
            gn = math.sqrt(gg)
            coef = p.beta * rhoA[s] * rhoB[s] / rho
            for i in range(q):
                ci = self.c[i]
                cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2]
                cF = ci[0] * F[0] + ci[1] * F[1] + ci[2] * F[2]
                cg = ci[0] * g[0] + ci[1] * g[1] + ci[2] * g[2]
                feq = self.w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)
                src = pre * self.w[i] * (3.0 * (cF - uF) + 9.0 * cu * cF)
                val = f[i] - (f[i] - feq) / tau + src
                cnorm = math.sqrt(ci[0] ** 2 + ci[1] ** 2 + ci[2] ** 2)
                cos = 0.0
                if gg > p.g_eps ** 2:
                    val += p.A * gn * (self.w[i] * cg * cg / gg - self.B[i])
                    if cnorm > 0:
                        cos = cg / (cnorm * gn)
                newA[i][s] = rhoA[s] / rho * val + coef * self.w[i] * cos
                newB[i][s] = rhoB[s] / rho * val - coef * self.w[i] * cos
            fields["u"][s] = u
            fields["f_nc"][s] = fnc
        return newA, newB, fields
