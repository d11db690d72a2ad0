"""FP64 reference of the learned near-contact closure (test infrastructure).

The paper's outlook proposes learning near-contact interactions from data
instead of fixing them by a hand-written functional (Sec. VI.B.3, learning
near-contact pseudo-potentials).  The closure here learns the explicit model
itself: a perceptron maps the local phase-field stencil of an interface site
to the near-contact force that the explicit scan (Eq. near_cont_force, as
read in ``OracleSim.near_contact_force``) gives there.

Network (a project choice; the paper fixes no architecture):
  input   x (30) = phi(x + d) for the 27 offsets d in {-1, 0, 1}^3 in
          lexicographic order k = (dx+1) + 3 (dy+1) + 9 (dz+1), with the
          mirrored wall ghosts of the gradient stencil, then n = g / |g|
  hidden  h1 = tanh(W1 x + b1) (64), h2 = tanh(W2 h1 + b2) (64)
  output  y = W3 h2 + b3 (3) = F_nc / (A_nc |g|)
The explicit force is (A_h/2) g, so the target is (A_h / (2 A_nc)) g/|g|: the
normal (an input) times a magnitude in {1/2, (h_min/h)^3 / 2, 0}, and the
closure's force is A_nc |g| y.
Parameters are packed as [W1 (64x30 row-major), b1, W2 (64x64), b2,
W3 (3x64), b3], 6339 values.

Training minimises the mean squared error over a mini-batch,
L = 1/(3B) sum_b sum_o (y_bo - t_bo)^2, with Adam (Kingma and Ba, 2015:
bias-corrected first and second moments, beta1 0.9, beta2 0.999, eps 1e-8).

Inference in the device path takes BF16 operands with wide accumulation;
``forward_bf16`` states that arithmetic: inputs, weights and both hidden
layers rounded to BF16 (round to nearest, ties to even), products summed
exactly (FP64 here), biases added unrounded.

At an interface site with |g| > g_eps the closure is used when the input is
inside the training data's range: every one of the 30 inputs within its
[min, max] over the training rows and |g| at least the smallest training
|g| (all compared in FP32).  Otherwise the explicit scan gives the force.
"""
from __future__ import annotations

import numpy as np

N_IN = 30
N_STENCIL = 27
N_H = 64
N_OUT = 3
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_OUT * N_H + N_OUT   # 6339

ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8

# stencil offsets (dx, dy, dz) in input order
OFFSETS = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)],
                   dtype=np.int64)


# ----------------------------------------------------------------- parameters
def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters, got {theta.shape}")
    o = 0

    def take(n, shape):
        nonlocal o
        v = theta[o:o + n].reshape(shape)
        o += n
        return v
    W1 = take(N_H * N_IN, (N_H, N_IN))
    b1 = take(N_H, (N_H,))
    W2 = take(N_H * N_H, (N_H, N_H))
    b2 = take(N_H, (N_H,))
    W3 = take(N_OUT * N_H, (N_OUT, N_H))
    b3 = take(N_OUT, (N_OUT,))
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2),
                           np.ravel(W3), np.ravel(b3)]).astype(np.float64)


# -------------------------------------------------------------- FP64 network
def forward(theta, X):
    """Activations of the network on rows X (m, 30), in FP64."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return dict(h1=h1, h2=h2, y=y)


def loss(theta, X, T):
    y = forward(theta, X)["y"]
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def gradient(theta, X, T):
    """(L, dL/dtheta) by backpropagation through the two tanh layers."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    a = forward(theta, X)
    h1, h2, y = a["h1"], a["h2"], a["y"]
    m = X.shape[0]
    r = y - T
    L = float(np.sum(r * r) / (N_OUT * m))
    dy = 2.0 * r / (N_OUT * m)              # dL/dy
    dW3 = dy.T @ h2
    db3 = dy.sum(0)
    dz2 = (dy @ W3) * (1.0 - h2 * h2)       # tanh' = 1 - tanh^2
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    dW1 = dz1.T @ X
    db1 = dz1.sum(0)
    return L, pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(theta, grad, m, v, t, lr):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = ADAM_BETA1 * m + (1.0 - ADAM_BETA1) * grad
    v = ADAM_BETA2 * v + (1.0 - ADAM_BETA2) * grad * grad
    mh = m / (1.0 - ADAM_BETA1 ** t)
    vh = v / (1.0 - ADAM_BETA2 ** t)
    theta = theta - lr * mh / (np.sqrt(vh) + ADAM_EPS)
    return theta, m, v


def train(theta, X, T, order, lr):
    """Adam over the mini-batches order[s] (row indices into X, T), one
    update per row of ``order``; returns (theta, per-step losses before each
    update)."""
    theta = np.array(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    losses = []
    for s, idx in enumerate(np.asarray(order)):
        L, g = gradient(theta, X[idx], T[idx])
        losses.append(L)
        theta, m, v = adam_step(theta, g, m, v, s + 1, lr)
    return theta, np.array(losses)


# ------------------------------------------------------------ BF16 inference
def bf16_round(x):
    """Nearest BF16 value (8 significant bits, ties to even) of each entry,
    returned as float64.  Normal range only: no value here is near the BF16
    subnormals or overflow."""
    x = np.asarray(x, dtype=np.float64)
    mant, ex = np.frexp(x)                        # x = mant 2^ex, |mant| in [0.5, 1)
    return np.ldexp(np.rint(mant * 256.0) / 256.0, ex)


def forward_bf16(theta, X):
    """Network output with BF16 operands (inputs, weights, hidden values) and
    exact accumulation; biases unrounded."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    xb = bf16_round(np.asarray(X, dtype=np.float64))
    h1 = bf16_round(np.tanh(xb @ bf16_round(W1).T + b1))
    h2 = bf16_round(np.tanh(h1 @ bf16_round(W2).T + b2))
    return h2 @ bf16_round(W3).T + b3


# ------------------------------------------------------------------- inputs
def stencil_inputs(sim, phi, g, sites):
    """Inputs at the given sites (tuple of index arrays iz, iy, ix): phi on the
    3x3x3 neighbourhood with wrap / wall mirroring, then g/|g|; and |g|.
    Both as FP32, the precision in which the range test is taken."""
    iz, iy, ix = sites
    P = sim.pad_phi(phi, 1)
    cols = [P[iz + 1 + dz, iy + 1 + dy, ix + 1 + dx] for dx, dy, dz in OFFSETS]
    gs = g[:, iz, iy, ix]
    gn = np.sqrt((gs * gs).sum(0))
    n = gs / gn
    X = np.stack(cols + [n[0], n[1], n[2]], axis=1).astype(np.float32)
    return X, gn.astype(np.float32)


def collect(sim):
    """Training rows of the last step of ``sim`` (run with the explicit force):
    every interface site with |g| > g_eps, in site order (x fastest), split
    into force-active and force-free ones.  Returns dict with X (m, 30) FP32,
    gnorm (m,) FP32, T (m, 3) = F_nc / (A_nc |g|) (FP64), site (m,) linear
    index, active (m,) bool."""
    p = sim.p
    fl = sim.fields()
    phi, Fnc = fl["phi"], fl["f_nc"]
    g = sim.gradient(phi)
    gg = (g * g).sum(0)
    cand = fl["flags"] & (gg > p.g_eps ** 2)
    iz, iy, ix = np.nonzero(cand)           # lexicographic (z, y, x) = site order
    X, gn = stencil_inputs(sim, phi, g, (iz, iy, ix))
    gs = g[:, iz, iy, ix]
    T = Fnc[:, iz, iy, ix].T / p.nc_A / np.sqrt((gs * gs).sum(0))[:, None]
    site = ix + p.nx * (iy + p.ny * iz)
    active = np.abs(T).sum(1) > 0
    return dict(X=X, gnorm=gn, T=T, site=site, active=active)


def input_ranges(X, gnorm):
    """Per-input [min, max] over the rows and the smallest |g| (FP32, exact)."""
    X = np.asarray(X, dtype=np.float32)
    return X.min(0), X.max(0), np.float32(np.min(gnorm))


class Closure:
    """Trained closure as the step uses it: FP32 parameters (given as the
    FP64 values of FP32 numbers) and the input ranges."""

    def __init__(self, theta, lo, hi, gmin):
        self.theta = np.asarray(theta, dtype=np.float64)
        self.lo = np.asarray(lo, dtype=np.float32)
        self.hi = np.asarray(hi, dtype=np.float32)
        self.gmin = np.float32(gmin)

    def in_range(self, X, gnorm):
        X = np.asarray(X, dtype=np.float32)
        return (np.all((X >= self.lo) & (X <= self.hi), axis=1)
                & (np.asarray(gnorm, dtype=np.float32) >= self.gmin))

    def force(self, X, g):
        """The force the closure gives at rows X: the explicit model (Eq.
        near_cont_force) is a repulsion along the colour gradient, so only the
        output's component along the unit normal is used, and only when it
        pushes along g:  F_nc = A_nc |g| max(0, y . n) n,  n = g/|g|  (g the
        FP64 gradient at the rows, shape (3, m); A_nc is applied by the
        caller)."""
        g = np.asarray(g, dtype=np.float64)
        gn = np.sqrt((g * g).sum(0))
        n = g / gn
        y = forward_bf16(self.theta, X)
        yn = np.maximum(0.0, (y * n.T).sum(1))
        return gn[:, None] * yn[:, None] * n.T
