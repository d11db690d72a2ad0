"""Droplet labels of the oracle (test infrastructure, see ``oracle/__init__``).

A droplet is a connected component of the dispersed-phase indicator phi > 0
under face connectivity (4 neighbours in 2D, 6 in 3D), with periodic wrap on
periodic axes.  Its label is the smallest linear site index it contains
(x fastest: idx = x + nx (y + ny z)); sites with phi <= 0 get -1.  This
canonical form is unique, so GPU and oracle labels compare bit for bit.
The droplet count is what the coalescence criterion of the near-contact
number (Sec. V, flow-focuser paragraph) is judged by.

Implementation: plain breadth-first search, one component at a time.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def label(fg, periodic=(True, True, True), two_d=False):
    """Return (labels int64 array of fg.shape (nz, ny, nx), count)."""
    fg = np.asarray(fg, dtype=bool)
    nz, ny, nx = fg.shape
    flat = fg.ravel()
    lab = np.full(flat.size, -1, dtype=np.int64)
    n = (nx, ny, nz)
    steps = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0)]
    if not two_d:
        steps += [(0, 0, 1), (0, 0, -1)]
    count = 0
    for start in range(flat.size):
        if not flat[start] or lab[start] >= 0:
            continue
        # BFS collects the whole component; the start is its smallest index
        # because sites are visited in increasing order.
        count += 1
        lab[start] = start
        dq = deque([start])
        while dq:
            s = dq.popleft()
            x = s % nx
            y = (s // nx) % ny
            z = s // (nx * ny)
            for dx, dy, dz in steps:
                c = [x + dx, y + dy, z + dz]
                ok = True
                for a in range(3):
                    if c[a] < 0 or c[a] >= n[a]:
                        if periodic[a]:
                            c[a] %= n[a]
                        else:
                            ok = False
                if not ok:
                    continue
                t = c[0] + nx * (c[1] + ny * c[2])
                if flat[t] and lab[t] < 0:
                    lab[t] = start
                    dq.append(t)
    return lab.reshape(fg.shape), count
