"""Pins of the oracle's droplet labels: agreement with scipy's connected
components (relabelled to the canonical minimum-index form) where no
component touches a periodic face, periodic joins across faces, and
invariance of the count under periodic shifts."""
import numpy as np
import pytest
from scipy import ndimage

from oracle.ccl import label


def _canonical(lab):
    out = np.full(lab.shape, -1, dtype=np.int64)
    flat = lab.ravel()
    o = out.ravel()
    for k in range(1, flat.max() + 1):
        idx = np.nonzero(flat == k)[0]
        o[idx] = idx.min()
    return out


@pytest.mark.parametrize("shape", [(1, 9, 11), (5, 6, 7)])
def test_matches_scipy_interior(shape):
    rng = np.random.default_rng(4)
    two_d = shape[0] == 1
    for trial in range(5):
        fg = rng.random(shape) < 0.45
        # clear the faces so periodic wrap cannot join anything
        fg[:, 0, :] = fg[:, -1, :] = False
        fg[:, :, 0] = fg[:, :, -1] = False
        if not two_d:
            fg[0] = fg[-1] = False
        st = ndimage.generate_binary_structure(3, 1)
        if two_d:
            st[0] = st[2] = False
        ref, n = ndimage.label(fg, structure=st)
        lab, count = label(fg, periodic=(True, True, True), two_d=two_d)
        assert count == n
        assert np.array_equal(lab, _canonical(ref))


def test_periodic_join_and_walls():
    fg = np.zeros((1, 4, 8), dtype=bool)
    fg[0, 1, 0] = fg[0, 1, 7] = True          # touch across the x face
    lab, count = label(fg, periodic=(True, True, True), two_d=True)
    assert count == 1 and lab[0, 1, 7] == lab[0, 1, 0] == 8
    lab, count = label(fg, periodic=(False, True, True), two_d=True)
    assert count == 2 and lab[0, 1, 7] == 15


def test_count_invariant_under_periodic_shift():
    rng = np.random.default_rng(9)
    fg = rng.random((4, 5, 6)) < 0.3
    _, c0 = label(fg)
    for sh in [(1, 0, 0), (0, 2, 0), (3, 4, 5)]:
        _, c1 = label(np.roll(fg, sh, (0, 1, 2)))
        assert c1 == c0
