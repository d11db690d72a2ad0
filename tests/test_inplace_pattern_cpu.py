"""The slot rules of in-place (AA-pattern) streaming, checked on the CPU.

The device path streams in place with three rules per direction i at site x
(walls by halfway bounce-back, other axes periodic):
  pull        slot (i, x - c_i), or (opp(i), x) when x - c_i is solid
  push        slot (opp(i), x + c_i), or (i, x) when x + c_i is solid
              (the pull slot of opp(i))
  own         slot (opp(i), x)
An even step pulls and pushes, an odd step reads `own` and stores at (i, x).
Here a numpy model with these rules runs beside plain two-copy streaming
under the same per-site collision map, and every pass is checked to read and
write each slot exactly once, with every site writing exactly the slots it
read (the property that makes one copy race-free)."""
import numpy as np
import pytest

from oracle.lattice import make_lattice


def _geometry(lat, shape, walls):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([x, y, z])                       # (3, nz, ny, nx)
    n = np.array([nx, ny, nz]).reshape(3, 1, 1, 1)

    def neighbour(i, sign):
        """Linear site index of x + sign c_i and whether it is solid."""
        p = pos + sign * lat.c[i].reshape(3, 1, 1, 1)
        solid = np.zeros(p.shape[1:], bool)
        for a in range(3):
            if walls[a]:
                solid |= (p[a] < 0) | (p[a] >= n[a, 0, 0, 0])
        p = p % n
        return p[0] + nx * (p[1] + ny * p[2]), solid

    site = (x + nx * (y + ny * z))
    return site, neighbour


def _slot_rules(lat, shape, walls):
    """Per direction: flat slot indices (q * N layout) of pull, push, own."""
    N = int(np.prod(shape))
    site, neighbour = _geometry(lat, shape, walls)
    pull, push, own = [], [], []
    for i in range(lat.q):
        o = int(lat.opp[i])
        src, s_solid = neighbour(i, -1)
        dst, d_solid = neighbour(i, +1)
        pull.append(np.where(s_solid, o * N + site, i * N + src).ravel())
        push.append(np.where(d_solid, i * N + site, o * N + dst).ravel())
        own.append((o * N + site).ravel())
    return np.array(pull), np.array(push), np.array(own)


def _collide(rng_mat, v):
    """A fixed per-site linear map mixing all directions (stands in for the
    collision; any map that uses every operand does)."""
    return np.einsum("ij,js->is", rng_mat, v) + 0.01 * np.roll(v, 1, axis=1)


CASES = [("D2Q9", (7, 5, 1), (0, 1, 0)), ("D2Q9", (2, 3, 1), (0, 0, 0)),
         ("D3Q19", (5, 4, 3), (0, 1, 1)), ("D3Q27", (4, 3, 5), (1, 1, 1)),
         ("D3Q27", (3, 2, 2), (0, 0, 0)), ("D3Q27", (6, 1, 4), (1, 0, 1))]


@pytest.mark.parametrize("name,shape,walls", CASES)
def test_aa_pattern_reproduces_two_copy_streaming(name, shape, walls):
    lat = make_lattice(name)
    q, N = lat.q, int(np.prod(shape))
    pull, push, own = _slot_rules(lat, shape, walls)
    local = np.arange(q)[:, None] * N + np.arange(N)[None, :]
    # every pass reads and writes each slot once, and a site writes the slots it read
    for reads, writes in ((pull, push), (own, local)):
        assert np.array_equal(np.sort(reads.ravel()), np.arange(q * N))
        assert np.array_equal(np.sort(writes.ravel()), np.arange(q * N))
        assert np.array_equal(np.sort(reads, axis=0), np.sort(writes, axis=0))
    rng = np.random.default_rng(11)
    M = rng.normal(size=(q, q)) / q
    ab = rng.normal(size=q * N)                     # canonical state, two copies
    aa = ab.copy()                                  # the one copy
    for t in range(7):
        ab = _collide(M, ab[pull]).ravel()
        if t % 2 == 0:
            post = _collide(M, aa[pull])
            aa[push.ravel()] = post.ravel()
            canon = aa[push]                        # f_i(x) sits in its push slot
        else:
            post = _collide(M, aa[own])
            aa[local.ravel()] = post.ravel()
            canon = aa[local]
        assert np.array_equal(canon.ravel(), ab), t
