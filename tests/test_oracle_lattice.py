"""Pins of the oracle's velocity sets: exact isotropy identities, the B_i
constraints of the colour-gradient perturbation operator, and the D2Q9
numbering the paper's boundary-condition equations imply."""
import json
import os
from fractions import Fraction
import itertools

import numpy as np
import pytest

from oracle.lattice import make_lattice, exact_moment, LATTICES

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("name", LATTICES)
def test_isotropy_exact(name):
    L = make_lattice(name)
    d = L.d
    assert sum(L.w_exact) == 1
    for a in range(3):
        pw = [0, 0, 0]
        pw[a] = 1
        assert exact_moment(L, pw) == 0
    # second moment: c_s^2 delta_ab on the d active axes
    for a, b in itertools.product(range(3), repeat=2):
        pw = [0, 0, 0]
        pw[a] += 1
        pw[b] += 1
        want = Fraction(1, 3) if (a == b and a < d) else 0
        assert exact_moment(L, pw) == want, (a, b)
    # odd third moments vanish
    for a, b, c in itertools.product(range(3), repeat=3):
        pw = [0, 0, 0]
        for k in (a, b, c):
            pw[k] += 1
        assert exact_moment(L, pw) == 0
    # fourth moment: c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    for a, b in itertools.product(range(d), repeat=2):
        pw = [0, 0, 0]
        pw[a] += 2
        pw[b] += 2
        want = Fraction(1, 3) if a == b else Fraction(1, 9)
        assert exact_moment(L, pw) == want


@pytest.mark.parametrize("name", LATTICES)
def test_b_constraints_exact(name):
    """sum B = 1/3, sum B c = 0, sum B c c = I/3 (Sec. III.C.1)."""
    L = make_lattice(name)
    B = L.b_exact
    assert sum(B) == Fraction(1, 3)
    for a in range(3):
        assert sum(Bi * int(ci[a]) for Bi, ci in zip(B, L.c.tolist())) == 0
    for a, b in itertools.product(range(L.d), repeat=2):
        s = sum(Bi * int(ci[a]) * int(ci[b]) for Bi, ci in zip(B, L.c.tolist()))
        assert s == (Fraction(1, 3) if a == b else 0)


@pytest.mark.parametrize("name", LATTICES)
def test_opposites_and_counts(name):
    L = make_lattice(name)
    assert L.q == {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}[name]
    assert np.array_equal(L.c[L.opp], -L.c)
    assert len({tuple(r) for r in L.c.tolist()}) == L.q
    assert np.all(L.c[0] == 0)


def test_d2q9_numbering_matches_paper_boundary_equations():
    L = make_lattice("D2Q9")
    fx = json.load(open(os.path.join(GOLD, "d2q9_numbering.json")))
    cx, cy = L.c[:, 0], L.c[:, 1]
    assert sorted(np.nonzero(cx == 1)[0].tolist()) == sorted(fx["cx_plus"]["members"])
    assert sorted(np.nonzero(cx == -1)[0].tolist()) == sorted(fx["cx_minus"]["members"])
    assert sorted(np.nonzero(cy == -1)[0].tolist()) == sorted(fx["cy_minus"]["members"])
    assert sorted(np.nonzero(cy == 1)[0].tolist()) == sorted(fx["cy_plus"]["members"])
    assert sorted(np.nonzero(cy == 0)[0].tolist()) == sorted(fx["rest_or_horizontal"]["members"])
    for i, j in fx["opposite_pairs"]["members"]:
        assert L.opp[i] == j
    bal = fx["x_momentum_balance"]["members"]
    for i, sgn in bal["lhs"] + bal["rhs"]:
        assert cx[i] == sgn
