"""Velocity sets of the oracle (test infrastructure, see ``oracle/__init__``).

Paper passages: Sec. III.B (Eq. ``lbm`` and the D2Q9 / D3Q27 lattices of the
``lattice_vel`` figure), Eq. ``disteq`` (weights w_i, sound speed c_s^2 = 1/3),
Sec. III.D (the D2Q9 numbering that the periodic copy rules and the Zou-He
wall equations imply), and the B_i isotropy constraints that close the
colour-gradient perturbation operator in Sec. III.C.1.

The weights are not printed in the paper; the standard ones are used and are
pinned by exact rational isotropy identities (tests/test_oracle_lattice.py).
D3Q19 is needed by the batched-ensemble workload; it is the paper's
single-component benchmark lattice (Sec. IV, FluidX3D table).

Everything here is exact (``fractions.Fraction``) and converted to float64 at
the very end.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
import numpy as np

CS2 = Fraction(1, 3)  # lattice sound speed squared, c_s^2


@dataclass(frozen=True)
class Lattice:
    name: str
    d: int                 # spatial dimension
    c: np.ndarray          # (q, 3) int64 velocities; z column is 0 in 2D
    w_exact: tuple         # weights as Fractions
    b_exact: tuple         # B_i coefficients as Fractions
    opp: np.ndarray        # (q,) opposite direction index

    @property
    def q(self) -> int:
        return self.c.shape[0]

    @property
    def w(self) -> np.ndarray:
        return np.array([float(x) for x in self.w_exact], dtype=np.float64)

    @property
    def B(self) -> np.ndarray:
        return np.array([float(x) for x in self.b_exact], dtype=np.float64)

    @property
    def cnorm(self) -> np.ndarray:
        """|c_i| (0 for the rest velocity)."""
        return np.sqrt((self.c.astype(np.float64) ** 2).sum(1))


def _d2q9_velocities():
    # Numbering fixed by the paper's D2Q9 boundary equations (Sec. III.D):
    # 1/3 are +x/-x, 2/4 are +y/-y, 5=(+1,+1), 6=(-1,+1), 7=(-1,-1), 8=(+1,-1).
    return [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
            (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]


def _d3q27_velocities():
    # Free ordering (the paper prints none for 3D): rest, then each shell in
    # (+v, -v) pairs so that opp(2k-1) = 2k.  The first 19 form D3Q19.
    v = [(0, 0, 0)]
    faces = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    for e in faces:
        v.append(e)
        v.append(tuple(-a for a in e))
    edges = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]
    for e in edges:
        v.append(e)
        v.append(tuple(-a for a in e))
    corners = [(1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1)]
    for e in corners:
        v.append(e)
        v.append(tuple(-a for a in e))
    return v


def _weights(vel, shell_weights):
    return tuple(shell_weights[sum(a * a for a in c)] for c in vel)


def _opposites(vel):
    idx = {c: i for i, c in enumerate(vel)}
    return np.array([idx[tuple(-a for a in c)] for c in vel], dtype=np.int64)


def _b_coefficients(w_exact):
    # One admissible solution of the three B_i isotropy constraints:
    # B_i = w_i for moving directions, B_0 = w_0 - 2/3.  Then
    # sum B = 1 - 2/3 = 1/3, sum B c = 0, sum B c c = sum w c c = I/3.
    return tuple([w_exact[0] - Fraction(2, 3)] + list(w_exact[1:]))


def make_lattice(name: str) -> Lattice:
    name = name.upper()
    if name == "D2Q9":
        vel = _d2q9_velocities()
        w = _weights(vel, {0: Fraction(4, 9), 1: Fraction(1, 9), 2: Fraction(1, 36)})
        d = 2
    elif name == "D3Q27":
        vel = _d3q27_velocities()
        w = _weights(vel, {0: Fraction(8, 27), 1: Fraction(2, 27), 2: Fraction(1, 54),
                           3: Fraction(1, 216)})
        d = 3
    elif name == "D3Q19":
        vel = _d3q27_velocities()[:19]
        w = _weights(vel, {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)})
        d = 3
    else:
        raise ValueError(f"unknown lattice {name!r}")
    return Lattice(name=name, d=d, c=np.array(vel, dtype=np.int64), w_exact=w,
                   b_exact=_b_coefficients(w), opp=_opposites(vel))


LATTICES = ("D2Q9", "D3Q19", "D3Q27")


def exact_moment(lat: Lattice, powers) -> Fraction:
    """sum_i w_i prod_a c_{i,a}^{p_a}, exact."""
    tot = Fraction(0)
    for wi, ci in zip(lat.w_exact, lat.c.tolist()):
        term = Fraction(wi)
        for a, p in enumerate(powers):
            term *= Fraction(ci[a]) ** p
        tot += term
    return tot


def all_direction_pairs(lat: Lattice):
    """(i, opp(i)) pairs, for table checks."""
    return [(i, int(lat.opp[i])) for i in range(lat.q)]


__all__ = ["Lattice", "make_lattice", "LATTICES", "CS2", "exact_moment",
           "all_direction_pairs"]
