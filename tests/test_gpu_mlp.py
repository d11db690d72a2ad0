"""GPU tests of the learned near-contact closure through the C ABI, against
the FP64 reference in oracle/mlp.py: the backpropagation and Adam kernels,
the BF16 matrix-core inference, the collection of training rows, one step
with the closure in the collision pass, and what a trained closure gains
over the method without a near-contact force."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402
from oracle import mlp as OM  # noqa: E402
from oracle.sim import OracleSim, OracleParams  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _handle(storage="f32", nc="explicit", shape=(16, 16, 16), **kw):
    return lb.Simulation(lattice="D3Q27", storage=storage, nc=nc, shape=shape, **kw)


def _net(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-1, 1, OM.N_PARAMS) * scale
    W1, b1, W2, b2, W3, b3 = OM.unpack(th)
    return OM.pack(W1 * 0.4, b1 * 0.2, W2 * 0.3, b2 * 0.2, W3, b3 * 0.2).astype(np.float32)


def _rows(rng, m):
    X = np.zeros((m, 32), dtype=np.float32)
    X[:, :27] = rng.uniform(-1, 1, (m, 27))
    n = rng.normal(size=(m, 3))
    X[:, 27:30] = n / np.linalg.norm(n, axis=1, keepdims=True)
    X[:, 30] = rng.uniform(0.01, 0.5, m)
    return X


def test_gradient_matches_oracle_backprop():
    say("case closure gradient")
    rng = np.random.default_rng(1)
    th = _net(2)
    X = _rows(rng, 300)
    T = rng.uniform(-0.5, 0.5, (300, 3)).astype(np.float32)
    sim = _handle()
    sim.mlp_set_weights(th)
    np.testing.assert_array_equal(sim.mlp_get_weights(), th)
    loss, g = sim.mlp_gradient(torch.from_numpy(X), torch.from_numpy(T))
    L, gref = OM.gradient(th.astype(np.float64), X[:, :30], T)
    g = g.cpu().numpy().astype(np.float64)
    err = np.abs(g - gref).max() / np.abs(gref).max()
    say(f"  loss {loss:.6e} vs {L:.6e}; gradient rel err {err:.2e}")
    assert abs(loss - L) <= 1e-5 * L
    assert err < 1e-4
    sim.close()


def test_training_matches_oracle_adam():
    """30 Adam steps from the same start on the same mini-batches: FP32 device
    training against FP64 training (losses and parameters to 1e-3)."""
    say("case closure training vs oracle")
    rng = np.random.default_rng(3)
    teacher = _net(4).astype(np.float64)
    X = _rows(rng, 2048)
    T = OM.forward(teacher, X[:, :30])["y"].astype(np.float32)
    th0 = W.closure_init_weights(seed=5)
    order = rng.integers(0, 2048, (30, 96)).astype(np.int32)
    sim = _handle()
    sim.mlp_set_weights(th0)
    log = sim.mlp_train(torch.from_numpy(X), torch.from_numpy(T), torch.from_numpy(order), lr=2e-3).cpu().numpy()
    th_gpu = sim.mlp_get_weights().astype(np.float64)
    th_ref, log_ref = OM.train(th0.astype(np.float64), X[:, :30], T, order, lr=2e-3)
    el = np.abs(log - log_ref).max() / log_ref.max()
    et = np.linalg.norm(th_gpu - th_ref) / np.linalg.norm(th_ref - th0)
    say(f"  loss {log_ref[0]:.4e} -> {log_ref[-1]:.4e}; loss rel err {el:.2e}; update rel err {et:.2e}")
    assert log_ref[-1] < log_ref[0]
    assert el < 1e-3
    assert et < 1e-3
    # ranges come from the training rows
    lo, hi, gmin = sim.mlp_get_ranges()
    np.testing.assert_array_equal(lo, X[:, :30].min(0))
    np.testing.assert_array_equal(hi, X[:, :30].max(0))
    assert gmin == X[:, 30].min()
    # an out-of-range index is reported
    bad = order.copy()
    bad[3, 5] = 2048
    with pytest.raises(lb.LBError):
        sim.mlp_train(torch.from_numpy(X), torch.from_numpy(T), torch.from_numpy(bad), lr=2e-3)
    sim.close()


def _bf16_tolerance(th):
    """Worst change of an output when one or two hidden values round to the
    neighbouring BF16 value (relative step 2^-8, |tanh| <= 1), plus FP32
    accumulation."""
    W1, b1, W2, b2, W3, b3 = OM.unpack(th.astype(np.float64))
    W2b, W3b = np.abs(OM.bf16_round(W2)), np.abs(OM.bf16_round(W3))
    flip2 = W3b.max(1)                        # one layer-2 value
    flip1 = (W3b @ W2b).max(1)                # one layer-1 value through layer 2
    return 2.0 * 2.0 ** -8 * np.maximum(flip1, flip2).max() + 1e-4


def test_inference_matches_bf16_reference():
    say("case closure inference")
    rng = np.random.default_rng(6)
    th = _net(7)
    X = _rows(rng, 5000)
    sim = _handle()
    sim.mlp_set_weights(th)
    out = sim.mlp_infer(torch.from_numpy(X)).cpu().numpy().astype(np.float64)
    ref = OM.forward_bf16(th.astype(np.float64), X[:, :30])
    d = np.abs(out - ref)
    tol = _bf16_tolerance(th)
    say(f"  max diff {d.max():.3e} (tol {tol:.3e}), rows above 1e-4: {(d.max(1) > 1e-4).mean():.3%}")
    assert d.max() <= tol
    assert (d.max(1) > 1e-4).mean() < 0.25
    # ragged row counts
    for m in (1, 15, 17, 63, 65):
        o = sim.mlp_infer(torch.from_numpy(X[:m])).cpu().numpy()
        np.testing.assert_array_equal(o, out[:m].astype(np.float32))
    sim.close()


PAIR = dict(shape=(40, 22, 20), walls=(0, 1, 1), tau=1.0, A=0.01, beta=0.7, body_force=(1e-6, 0.0, 0.0))
PAIR_C = [[12.3, 10.7, 9.6], [26.9, 11.2, 10.1]]
PAIR_R = [6.0, 6.0]


def _oracle_pair(closure=None):
    nx, ny, nz = PAIR["shape"]
    p = OracleParams(lattice="D3Q27", nx=nx, ny=ny, nz=nz, walls=tuple(bool(w) for w in PAIR["walls"]),
                     tau=PAIR["tau"], A=PAIR["A"], beta=PAIR["beta"], body_force=PAIR["body_force"], nc=True,
                     closure=closure)
    return OracleSim(p).init_droplets(PAIR_C, PAIR_R)


def test_collect_matches_oracle():
    say("case closure collect fp64")
    o = _oracle_pair().step(2)
    ref = OM.collect(o)
    sim = _handle("f64", "explicit", **PAIR).init_droplets(PAIR_C, PAIR_R)
    sim.step(2)
    rows, tg, na, nf = sim.nc_collect()
    rows, tg = rows.cpu().numpy(), tg.cpu().numpy()
    say(f"  rows {na} active + {nf} free (oracle {ref['active'].sum()} + {(~ref['active']).sum()})")
    assert na == ref["active"].sum() and nf == (~ref["active"]).sum()
    order = np.concatenate([np.nonzero(ref["active"])[0], np.nonzero(~ref["active"])[0]])
    np.testing.assert_array_equal(rows[:, :27], ref["X"][order, :27])
    np.testing.assert_allclose(rows[:, 27:30], ref["X"][order, 27:30], rtol=0, atol=2e-7)
    np.testing.assert_allclose(rows[:, 30], ref["gnorm"][order], rtol=2e-7)
    assert np.all(rows[:, 31] == 0)
    np.testing.assert_allclose(tg, ref["T"][order].astype(np.float32), rtol=1e-6, atol=1e-9)
    sim.close()


def test_step_with_closure_matches_oracle():
    """One FP64 step from the same state with the closure in the collision
    pass: where the network or the explicit scan gave the force (flag bits)
    exactly, the force and the state within the BF16 tolerance."""
    say("case closure step fp64")
    o = _oracle_pair().step(2)
    ref = OM.collect(o)
    th = _net(8, scale=0.3)
    lo, hi, gmin = OM.input_ranges(ref["X"], ref["gnorm"])
    hi = hi.copy()
    hi[13] = np.float32(np.median(ref["X"][:, 13]))     # half the sites fall back to the scan
    clo = OM.Closure(th.astype(np.float64), lo, hi, gmin)
    o2 = _oracle_pair(closure=clo)
    o2.set_state(o.fA, o.fB, t=o.t)
    o2.step(1)
    sim = _handle("f64", "mlp", **PAIR)
    sim.mlp_set_weights(th)
    sim.mlp_set_ranges(lo, hi, gmin)
    sim.set_state(torch.from_numpy(np.stack([o.fA, o.fB])))
    sim.step(1)
    f = {k: v.cpu().numpy() for k, v in sim.fields(("f_nc", "flags")).items()}
    of = o2.fields()
    want_flags = of["flags"].astype(np.uint8) | (of["nc_source"] == 1) * 2 | (of["nc_source"] == 2) * 4
    n_net, n_exp = int((of["nc_source"] == 1).sum()), int((of["nc_source"] == 2).sum())
    say(f"  network sites {n_net}, explicit-scan sites {n_exp}")
    assert n_net > 50 and n_exp > 50
    np.testing.assert_array_equal(f["flags"], want_flags)
    gmax = np.sqrt((o2.gradient(of["phi"]) ** 2).sum(0)).max()
    tolF = o.p.nc_A * gmax * _bf16_tolerance(th)
    dF = np.abs(f["f_nc"] - of["f_nc"]).max()
    st = sim.get_state().cpu().numpy()
    dS = max(np.abs(st[0] - o2.fA).max(), np.abs(st[1] - o2.fB).max())
    say(f"  force diff {dF:.3e} (tol {tolF:.3e}); state diff {dS:.3e}")
    assert dF <= tolF
    # u = (j + F/2)/rho and the Guo source move each population by at most a
    # few times the force difference
    assert dS <= 4 * tolF
    sim.close()


def closure_force_error(F, Fexp, T):
    """||F - F_exp||_2 / ||F_exp||_2 over all rows, over force-active rows and
    per near-contact distance class of the explicit force (its magnitude per
    unit strength and |g| is 1/2 for h <= h_min = 2 and (2/3)^3 / 2 for h = 3);
    and the RMS of the closure's force at force-free rows relative to the RMS
    explicit force at active rows."""
    mag = torch.linalg.norm(T, dim=1)
    a = mag > 0
    out = {"all": float(torch.linalg.norm(F - Fexp) / torch.linalg.norm(Fexp)),
           "active": float(torch.linalg.norm(F[a] - Fexp[a]) / torch.linalg.norm(Fexp[a]))}
    for name, lvl in (("h<=2", 0.5), ("h=3", 0.5 * (2 / 3) ** 3)):
        m = (mag - lvl).abs() < 1e-3
        if m.any():
            out[name] = float(torch.linalg.norm(F[m] - Fexp[m]) / torch.linalg.norm(Fexp[m]))
    out["free/active rms"] = float(torch.linalg.norm(F[~a]) / max(1, int((~a).sum())) ** 0.5
                                   / (torch.linalg.norm(Fexp[a]) / max(1, int(a.sum())) ** 0.5))
    return out


def _pair3d(nc, steps, gap=3.0, R=8.0, net=None, ranges=None):
    n = int(2 * (2 * R + 12))
    d = R + gap / 2
    sim = lb.Simulation(lattice="D3Q27", storage="f32", nc=nc, shape=(n, 32, 32), walls=(0, 0, 0),
                        tau=1.0, A=0.01, beta=0.7)
    if net is not None:
        sim.mlp_set_weights(net)
        sim.mlp_set_ranges(*ranges)
    sim.init_droplets([[n / 2 - d + 0.13, 16.21, 15.87], [n / 2 + d + 0.13, 15.79, 16.09]], [R, R])
    sim.step(steps)
    count = int(sim.diagnostics()[6])
    sim.close()
    return count


_TRAINED = {}


def _trained_closure():
    """Train on rows the explicit force generates in a dense emulsion (10
    snapshots 100 steps apart; 20k Adam steps of 256 rows, half force-active,
    learning rate stepped down).  Returns the parameters, the input ranges,
    the loss log and a held-out snapshot's rows; trained once per process."""
    if _TRAINED:
        return _TRAINED
    w = W.dense_3d(shape=(96, 96, 64), count=1000)
    kw, cen, rad = W.sim_kwargs(w)
    sim = lb.Simulation(**kw).init_droplets(cen, rad)
    nas, nfs = 0, 0
    A_parts, F_parts = [], []
    for snap in range(10):
        sim.step(100)
        r, t, na, nf = sim.nc_collect()
        A_parts.append((r[:na], t[:na]))
        F_parts.append((r[na:], t[na:]))
        nas += na
        nfs += nf
    held = sim.step(100).nc_collect()
    sim.close()
    rows = torch.cat([a[0] for a in A_parts] + [f[0] for f in F_parts])
    tgs = torch.cat([a[1] for a in A_parts] + [f[1] for f in F_parts])
    say(f"  training rows: {nas} active, {nfs} free")
    tr = _handle()
    tr.mlp_set_weights(W.closure_init_weights())
    logs = []
    for k, (n_steps, lr) in enumerate(((12000, 2e-3), (6000, 5e-4), (2000, 1e-4))):
        order = W.closure_batches(nas, nfs, n_steps, 256, seed=k + 1)
        logs.append(tr.mlp_train(rows, tgs, torch.from_numpy(order), lr=lr).cpu().numpy())
    _TRAINED.update(theta=tr.mlp_get_weights(), ranges=tr.mlp_get_ranges(), log=np.concatenate(logs),
                    held=held, handle=tr)
    return _TRAINED


def applied_force(pred, rows):
    """The force per unit strength the collision pass applies for network
    outputs y at rows: |g| max(0, y . n) n (n the row's unit normal)."""
    n = rows[:, 27:30].double()
    gn = rows[:, 30:31].double()
    yn = torch.clamp((pred.double() * n).sum(1, keepdim=True), min=0.0)
    return gn * yn * n


def test_trained_closure_keeps_droplets_apart():
    """Train on rows of a dense emulsion, then run two droplets 3 sites apart:
    without a near-contact force they merge, with the explicit force or the
    trained closure they stay two.  The force error on a held-out snapshot is
    reported per near-contact distance class, for the raw network output and
    for the force the step applies (its repulsive normal part)."""
    say("case closure training + gain")
    tc = _trained_closure()
    log = tc["log"]
    say(f"  loss {log[:50].mean():.3e} -> {log[-200:].mean():.3e}")
    assert log[-200:].mean() < 0.2 * log[:50].mean()
    th, ranges = tc["theta"], tc["ranges"]
    r, t, na, nf = tc["held"]
    pred = tc["handle"].mlp_infer(r).double()
    t = t.double()
    gn = r[:, 30:31].double()                  # F = A_nc |g| y
    raw = closure_force_error(pred * gn, t * gn, t)
    err = closure_force_error(applied_force(pred, r), t * gn, t)
    say("  held-out force error, network output: " + ", ".join(f"{k} {v:.3f}" for k, v in raw.items()))
    say("  held-out force error, applied force:  " + ", ".join(f"{k} {v:.3f}" for k, v in err.items()))
    # just above the measured 0.377 (applied) and 0.387 (raw): a 3x3x3
    # stencil cannot see the opposing interface at h = 2..3, which bounds
    # what any network of this input can reach
    assert err["active"] < 0.42
    assert raw["active"] < 0.43
    off = _pair3d("off", 3000)
    on = _pair3d("explicit", 3000)
    learned = _pair3d("mlp", 3000, net=th, ranges=ranges)
    say(f"  droplets after 3000 steps: off {off}, explicit {on}, closure {learned}")
    assert off == 1 and on == 2
    assert learned == 2


def _dense_run(nc, steps, net=None, ranges=None):
    w = W.dense_3d()
    kw, cen, rad = W.sim_kwargs(w)
    sim = lb.Simulation(**dict(kw, nc=nc))
    if net is not None:
        sim.mlp_set_weights(net)
        sim.mlp_set_ranges(*ranges)
    sim.init_droplets(cen, rad)
    sim.step(steps)
    d = sim.diagnostics()
    sim.close()
    return int(d[6]), float(d[5])


def test_trained_closure_keeps_the_dense_emulsion():
    """The full dense emulsion (384 x 384 x 192, 2000 droplets R = 8 whose
    films start 3.6 sites or more apart), 3000 steps: without a near-contact
    force the films drain and the droplets merge; with the explicit force and
    with the trained closure all 2000 stay apart, and the closure's flow
    stays bounded."""
    say("case closure on the dense emulsion")
    tc = _trained_closure()
    off, u_off = _dense_run("off", 3000)
    exp, u_exp = _dense_run("explicit", 3000)
    learned, u_net = _dense_run("mlp", 3000, net=tc["theta"], ranges=tc["ranges"])
    say(f"  droplets after 3000 steps: off {off}, explicit {exp} (max|u| {u_exp:.4f}), "
        f"closure {learned} (max|u| {u_net:.4f})")
    assert off < 100
    assert exp == 2000 and learned == 2000
    # the closure's force error (tens of percent) shows in the flow: 0.028
    # measured against 0.009 with the explicit force.  Runs that differ only
    # in rounding (the read-once and two-pass steps) moved it by up to 2x, so
    # the bar sits above that spread, well below the watchdog's 0.3
    assert u_net < 0.06
