"""The read-once step's scatter geometry on the CPU.

Each post-collision population belongs to exactly one site of the next step
(the site that pulls it, or the site itself at a wall: halfway bounce-back,
paper Sec. III.D).  tests/scatter_geom_check.cpp routes integer values by
tile-march exactly as the collision kernel's halo layout prescribes
(paper_2405_14551_amd/csrc/scatter_geom.hpp), combines them with the same
neighbour rule as the combine pass, and compares every site with the direct
pull sum; it also checks that every halo index stays inside its block.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "scatter_geom_check.cpp")

CASES = [
    # nx ny nz walls(x y z) dims q TX TY zb
    (40, 24, 20, 0, 1, 1, 3, 27, 64, 4, 8),     # parity case shape, walls y/z, ragged marches
    (65, 9, 7, 1, 0, 0, 3, 27, 64, 4, 3),       # one-site-wide last tile, wall x
    (1, 1, 1, 0, 0, 0, 3, 27, 64, 4, 1),        # every axis one site, periodic: the box wraps on itself
    (130, 10, 33, 1, 1, 1, 3, 19, 64, 4, 32),   # D3Q19, walls everywhere, ragged in x, y and z
    (17, 5, 1, 0, 0, 0, 2, 9, 64, 4, 1),        # D2Q9 periodic
    (17, 5, 1, 1, 1, 0, 2, 9, 64, 4, 1),        # D2Q9 with walls
    (128, 64, 1, 0, 0, 0, 2, 9, 64, 4, 1),      # the 2D Laplace lattice
    (64, 4, 5, 0, 0, 0, 3, 27, 64, 4, 5),       # one tile-march covering the lattice
    (64, 4, 5, 0, 0, 0, 3, 27, 64, 4, 2),       # periodic z with a one-plane last march
    (3, 2, 2, 0, 0, 0, 3, 27, 64, 4, 1),        # tiny periodic lattice
    (70, 13, 16, 1, 0, 1, 3, 27, 32, 8, 5),     # another tile shape
    (256, 16, 12, 0, 1, 1, 3, 27, 64, 4, 32),   # march deeper than the lattice
]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("sg") / "scatter_geom_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-o", exe, SRC], check=True)
    return exe


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:3])) + f"_w{c[3]}{c[4]}{c[5]}_q{c[7]}_zb{c[10]}")
def test_scatter_then_combine_equals_the_pull(checker, case):
    r = subprocess.run([checker, *map(str, case)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
