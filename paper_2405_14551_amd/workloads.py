"""Seeded synthetic inputs of the benchmark workloads (no method arithmetic).

Droplet centres are drawn by random sequential addition with numpy's PCG64
generator: a candidate centre is uniform inside the box (keeping a clearance
of R + 2 sites from walled faces) and is accepted when its surface stays at
least ``min_gap`` sites from every accepted droplet (minimum image along
periodic axes).  Both the oracle-based tests and the GPU path receive the
same explicit centre list.

Workloads (sizes as in the benchmark definitions):
  laplace_2d    D2Q9 128x64 periodic, FP64, one droplet R=16 at the box centre
                ((nx-1)/2, (ny-1)/2) = (63.5, 31.5), so that no site is a point
                of exact symmetry (see the note on symmetric points below)
  channel_3d    D3Q27 256x128x128, walls y/z, body force 1e-6 x, 64 droplets R=10,
                near-contact range 3 / strength 0.02, FP32
  big_3d        same physics on 512x256x256 with 1024 droplets R=8
  dense_3d      D3Q27 384x384x192, 2000 droplets R=8 on a jittered FCC slab
                (surface gap 3.5 +- 0.25 per coordinate)
"""
from __future__ import annotations

import numpy as np

SEED = 14551

# Symmetric points: where the phase gradient vanishes by symmetry and a site
# sits exactly there (a droplet centre on a site, the midpoint between
# periodic images), the computed gradient is rounding noise, its direction is
# random, and the recolouring amplifies that noise by a factor of about 3 per
# step.  Two correct implementations then drift apart at those sites (by
# amounts far below any physical scale).  Centres used for parity checks are
# therefore placed off such points.


def rsa_centres(shape, walls, radius, count, seed=SEED, min_gap=3.0, max_tries=200000, dims=3):
    """Random sequential addition of equal droplets; returns (count, 3) float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.asarray(shape, dtype=np.float64)
    lo = np.zeros(3)
    hi = n.copy()
    for a in range(3):
        if walls[a]:
            lo[a] = radius + 2.0
            hi[a] = n[a] - 1 - (radius + 2.0)
    cen = np.zeros((0, 3))
    tries = 0
    while cen.shape[0] < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"placed only {cen.shape[0]} of {count} droplets")
        c = lo + rng.random(3) * (hi - lo)
        if dims == 2:
            c[2] = 0.0
        if cen.shape[0]:
            d = cen - c
            for a in range(dims):
                if not walls[a]:
                    d[:, a] -= n[a] * np.round(d[:, a] / n[a])
            if dims == 2:
                d[:, 2] = 0.0
            if np.min(np.sqrt((d * d).sum(1))) < 2 * radius + min_gap:
                continue
        cen = np.vstack([cen, c])
    return cen


def fcc_slab_centres(shape, radius, count, gap=3.5, jitter=0.25, seed=SEED):
    """Droplets on an FCC lattice with nearest-neighbour surface gap ``gap``
    (+- ``jitter`` uniform displacement per coordinate), filling a slab
    centred in z; periodic x/y, walls z.  With the defaults every surface
    starts just outside the near-contact range (h_max = 3): the force keeps
    the emulsion apart, and without it the films drain and the droplets merge."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = shape
    dnn = 2 * radius + gap                   # nearest-neighbour distance
    a = dnn * np.sqrt(2.0)                   # cubic cell edge
    mx, my = int(nx // a), int(ny // a)
    ax, ay = nx / mx, ny / my                # stretch so the cell tiles the periodic box
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    pts = []
    k = 0
    zlo = radius + 2.0
    while len(pts) < count:
        for i in range(mx):
            for j in range(my):
                for b in basis:
                    z = zlo + (k + b[2]) * a
                    if z > nz - 1 - (radius + 2.0):
                        continue
                    pts.append([(i + b[0]) * ax, (j + b[1]) * ay, z])
        k += 1
        if zlo + k * a > nz:
            break
    pts = np.array(pts[:count], dtype=np.float64)
    pts += rng.uniform(-jitter, jitter, pts.shape)
    # centre the slab in z
    pts[:, 2] += (nz - 1) / 2.0 - 0.5 * (pts[:, 2].min() + pts[:, 2].max())
    return pts


def laplace_2d(on_site=False):
    """The 2D Laplace droplet: D2Q9 128 x 64 periodic, FP64, tau 1, A 0.01,
    beta 0.7, R 16.  on_site=True centres it on the site (64, 32), as the
    workload is stated; the default centre (63.5, 31.5) keeps every symmetry
    point of the periodic lattice off the sites."""
    c = [64.0, 32.0, 0.0] if on_site else [63.5, 31.5, 0.0]
    return dict(lattice="D2Q9", storage="f64", nc="off", shape=(128, 64, 1), walls=(0, 0, 0),
                tau=1.0, A=0.01, beta=0.7, rho0=1.0,
                centres=np.array([c]), radii=np.array([16.0]))


def channel_3d(storage="f32", shape=(256, 128, 128), count=64, radius=10.0, seed=SEED):
    walls = (0, 1, 1)
    cen = rsa_centres(shape, walls, radius, count, seed)
    return dict(lattice="D3Q27", storage=storage, nc="explicit", shape=shape, walls=walls,
                tau=1.0, A=0.01, beta=0.7, rho0=1.0, body_force=(1e-6, 0.0, 0.0),
                nc_A=0.02, nc_hmin=2.0, nc_hmax=3.0,
                centres=cen, radii=np.full(count, radius))


def big_3d(storage="f16"):
    return channel_3d(storage=storage, shape=(512, 256, 256), count=1024, radius=8.0)


def big_3d_crop(storage="f32", crop=64, seed=SEED):
    """The 64^3 crop of big_3d used for precision statements: the same physics
    on a sub-box [x0, x0 + crop) x [0, crop)^2 with walls on the y/z faces (the
    crop's x axis stays periodic), holding the droplets of the big_3d list that
    lie fully inside it with 2 sites of clearance; x0 is the multiple of 8 that
    keeps the most droplets."""
    big = big_3d(storage)
    cen, rad = big["centres"], big["radii"]
    best = None
    for x0 in range(0, big["shape"][0] - crop + 1, 8):   # y0 = z0 = 0 keeps two real walls
        c = cen - np.array([x0, 0.0, 0.0])
        keep = np.all((c - rad[:, None] >= 2.0) & (c + rad[:, None] <= crop - 1 - 2.0), axis=1)
        if best is None or keep.sum() > best[1].sum():
            best = (c, keep)
    c, keep = best
    w = dict(big)
    w.update(shape=(crop, crop, crop), centres=c[keep], radii=rad[keep], storage=storage)
    return w


def dense_3d(storage="f32", count=2000, radius=8.0, shape=(384, 384, 192), seed=SEED):
    cen = fcc_slab_centres(shape, radius, count, seed=seed)
    return dict(lattice="D3Q27", storage=storage, nc="explicit", shape=shape, walls=(0, 0, 1),
                tau=1.0, A=0.01, beta=0.7, rho0=1.0, body_force=(1e-6, 0.0, 0.0),
                nc_A=0.02, nc_hmin=2.0, nc_hmax=3.0,
                centres=cen, radii=np.full(len(cen), radius))


def rsa_centres_radii(shape, walls, radii, seed=SEED, min_gap=3.0, max_tries=4000):
    """Random sequential addition of droplets with given radii (largest
    first); a droplet that finds no free spot in max_tries draws is left out,
    so small boxes may hold fewer droplets than asked for."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.asarray(shape, dtype=np.float64)
    radii = np.sort(np.asarray(radii, dtype=np.float64))[::-1]
    cen = np.zeros((0, 3))
    placed = []
    for R in radii:
        lo = np.zeros(3)
        hi = n.copy()
        for a in range(3):
            if walls[a]:
                lo[a] = R + 2.0
                hi[a] = n[a] - 1 - (R + 2.0)
        for _ in range(max_tries):
            c = lo + rng.random(3) * (hi - lo)
            if cen.shape[0]:
                d = cen - c
                for a in range(3):
                    if not walls[a]:
                        d[:, a] -= n[a] * np.round(d[:, a] / n[a])
                if np.any(np.sqrt((d * d).sum(1)) < np.array(placed) + R + min_gap):
                    continue
            cen = np.vstack([cen, c])
            placed.append(R)
            break
    return cen, np.array(placed)


def ensemble_channels(n=96, seed=SEED, storage="f32"):
    """Batched ensemble: n independent D3Q19 channels, channel c drawn with
    seed + c: nx ~ U{64..160}, ny, nz ~ U{64..96}, tau ~ U[0.6, 1.2],
    4..40 droplets with R ~ U[6, 12] (those that fit); walls y/z, body force
    1e-6 along x, near contact range 3 / strength 0.02."""
    chans = []
    for c in range(n):
        rng = np.random.Generator(np.random.PCG64(seed + c))
        shape = (int(rng.integers(64, 161)), int(rng.integers(64, 97)), int(rng.integers(64, 97)))
        tau = float(rng.uniform(0.6, 1.2))
        count = int(rng.integers(4, 41))
        radii = rng.uniform(6.0, 12.0, count)
        cen, rad = rsa_centres_radii(shape, (0, 1, 1), radii, seed=seed + 1000 + c)
        chans.append(dict(shape=shape, walls=(0, 1, 1), tau=tau, A=0.01, beta=0.7, body_force=(1e-6, 0.0, 0.0),
                          nc_A=0.02, nc_hmin=2.0, nc_hmax=3.0, centres=cen, radii=rad))
    return dict(lattice="D3Q19", storage=storage, nc="explicit", channels=chans)


def sim_kwargs(w):
    """Split a workload dict into Simulation kwargs and the droplet list."""
    kw = {k: v for k, v in w.items() if k not in ("centres", "radii")}
    return kw, w["centres"], w["radii"]


def closure_init_weights(seed=SEED):
    """Initial parameters of the near-contact closure network (30-64-64-3):
    uniform in +-sqrt(6 / (fan_in + fan_out)) (Glorot), zero biases; packed
    as W1, b1, W2, b2, W3, b3 (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in ((30, 64), (64, 64), (64, 3)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def closure_batches(n_active, n_free, n_steps, batch, seed=SEED):
    """Mini-batch row indices for training on collected rows (active rows
    0 .. n_active-1, force-free rows after them): each batch draws half its
    rows from the force-active and half from the force-free rows, uniformly
    with replacement.  int32 array (n_steps, batch)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    half = batch // 2
    if n_active == 0 or n_free == 0:
        return rng.integers(0, n_active + n_free, (n_steps, batch)).astype(np.int32)
    a = rng.integers(0, n_active, (n_steps, half))
    f = n_active + rng.integers(0, n_free, (n_steps, batch - half))
    return np.concatenate([a, f], axis=1).astype(np.int32)
