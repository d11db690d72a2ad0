"""GPU: the read-once step (the collision pass scatters the next step's colour
densities, a combine pass finishes the phase field) against the two-pass step
(a separate pass pulls the populations again) and against the FP64 oracle.

Both steps compute the phase field of the neighbours after streaming (paper
Sec. III.C.1); they differ only in the order in which the colour sums are
rounded.  FP64: the two paths agree within 1e-13 over 30 steps and the
read-once path meets the oracle at 1e-12.  The first step after an
initialisation or a restore scatters the stored state (the bootstrap pass);
other storages agree within their rounding, and a restored run repeats the
uninterrupted one bit for bit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb  # noqa: E402
from oracle.sim import OracleSim, OracleParams  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def droplets(shape, lattice, n=3, seed=5):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    r = max(2.0, min(shape[:2] if lattice == "D2Q9" else shape) / 4.0)
    cen = np.stack([rng.uniform(0.2, 0.8, n) * nx + 0.31, rng.uniform(0.3, 0.7, n) * ny + 0.17,
                    (rng.uniform(0.3, 0.7, n) * nz + 0.23) if lattice != "D2Q9" else np.zeros(n)], 1)
    return cen, np.full(n, r)


def oparams(kw):
    nx, ny, nz = kw["shape"]
    return OracleParams(lattice=kw["lattice"], nx=nx, ny=ny, nz=nz,
                        walls=tuple(bool(v) for v in kw.get("walls", (0, 0, 0))),
                        tau=kw.get("tau", 1.0), A=kw.get("A", 0.01), beta=kw.get("beta", 0.7),
                        body_force=tuple(kw.get("body_force", (0, 0, 0))), u0=tuple(kw.get("u0", (0, 0, 0))),
                        nc=kw.get("nc", "off") == "explicit")


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def run(kw, steps, phase, cen, rad, zb=None):
    sim = lb.Simulation(**dict(kw, phase=phase))
    if zb is not None:
        sim.set_z_per_block(zb)
    sim.init_droplets(cen, rad)
    sim.step(steps)
    st = sim.get_state().double().cpu().numpy()
    f = {k: v.double().cpu().numpy() for k, v in sim.fields(("rho_a", "rho_b", "phi", "u")).items()}
    fl = sim.fields(("flags",))["flags"].cpu().numpy()
    sim.close()
    return st, f, fl


# geometries: ragged tiles in x (nx not a multiple of 64, a one-site last
# tile), rows not a multiple of 4, walls on each axis, very short axes,
# marches of one plane and marches longer than the lattice
GEOMS = [
    ("D3Q27", (40, 24, 20), (0, 1, 1), "explicit", None),
    ("D3Q27", (65, 9, 7), (1, 0, 0), "off", None),
    ("D3Q27", (70, 13, 16), (0, 0, 1), "explicit", 3),
    ("D3Q27", (130, 10, 12), (1, 1, 1), "explicit", 1),
    ("D3Q27", (64, 4, 5), (0, 0, 0), "off", 16),
    ("D3Q27", (3, 2, 2), (0, 0, 0), "off", None),
    ("D3Q19", (66, 11, 9), (0, 1, 0), "explicit", 2),
    ("D3Q19", (48, 16, 24), (0, 1, 1), "explicit", None),
    ("D2Q9", (128, 64, 1), (0, 0, 0), "off", None),
    ("D2Q9", (67, 13, 1), (1, 1, 0), "explicit", None),
]


@pytest.mark.parametrize("geom", GEOMS, ids=lambda g: f"{g[0]}_{'x'.join(map(str, g[1]))}_w{''.join(map(str, g[2]))}_"
                                                     f"{g[3]}_zb{g[4]}")
def test_fp64_read_once_equals_two_pass_and_oracle(geom):
    lattice, shape, walls, nc, zb = geom
    kw = dict(lattice=lattice, storage="f64", nc=nc, shape=shape, walls=walls, tau=0.9, A=0.02,
              body_force=(2e-5, 1e-5, 0.0) if lattice == "D2Q9" else (2e-5, 1e-5, -1e-5), u0=(0.01, 0.0, 0.0))
    cen, rad = droplets(shape, lattice)
    steps = 30
    say(f"case f64 {lattice} {shape} walls={walls} nc={nc} zb={zb} steps={steps}")
    st_ro, f_ro, fl_ro = run(kw, steps, "scatter", cen, rad, zb)
    st_tp, f_tp, fl_tp = run(kw, steps, "pass", cen, rad, zb)
    e = rel(st_ro, st_tp)
    assert e < 1e-13, f"read-once vs two-pass state {e:.2e}"
    assert rel(f_ro["phi"], f_tp["phi"]) < 1e-13
    assert np.array_equal(fl_ro, fl_tp)
    orc = OracleSim(oparams(kw)).init_droplets(cen, rad).step(steps)
    e_or = max(rel(st_ro[0], orc.fA), rel(st_ro[1], orc.fB))
    assert e_or < 1e-12, f"read-once vs oracle {e_or:.2e}"
    assert rel(f_ro["phi"], orc.fields()["phi"]) < 1e-12


STORAGES = ["f32", "f16", "bf16", "f32s", "f32t", "f16t", "bf16t", "f16ct", "f16t_sr", "bf16t_sr"]
# phase-field bar after three steps: FP32 rounding of the colour sums, or one
# step of the 16-bit storage where a stored value rounded the other way
PHI_BAR = {"f32": 1e-6, "f32s": 1e-6, "f32t": 1e-6, "f16": 2e-3, "f16t": 2e-3, "f16ct": 2e-3, "f16t_sr": 2e-3,
           "bf16": 2e-2, "bf16t": 2e-2, "bf16t_sr": 2e-2}


def stored_values(sim):
    """The stored state as float64 values: (populations or totals decoded,
    the total layout's FP32 scalars or an empty array)."""
    raw = sim.get_state()
    if not sim.total:
        return raw.double().cpu().numpy().ravel(), np.zeros(0)
    T, sc = sim.split_total_state(raw)
    if sim.storage == "f16ct":
        from oracle.fp16c import decode
        t = decode(T.cpu().numpy().view(np.uint16))
    else:
        t = T.double().cpu().numpy()
    return np.asarray(t, np.float64).ravel(), sc.double().cpu().numpy().ravel()


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("streaming", ["two_copies", "in_place"])
def test_other_storages_match_the_two_pass_step(storage, streaming):
    """Every storage and streaming mode: after one step the stored values are
    within the storage's rounding of each other (both steps differ only in
    the rounding order of the phase field they use), and after three steps
    the phase field the read-once path scattered matches the two-pass one
    within the storage's rounding."""
    st_name, rounding = (storage[:-3], "stochastic") if storage.endswith("_sr") else (storage, "nearest")
    kw = dict(lattice="D3Q27", storage=st_name, nc="explicit", shape=(70, 20, 18), walls=(0, 1, 1),
              body_force=(1e-5, 0, 0), u0=(0.02, 0.0, 0.0), streaming=streaming, rounding=rounding)
    cen, rad = droplets(kw["shape"], "D3Q27")
    say(f"case {storage} {streaming}")
    out = {}
    for phase in ("scatter", "pass"):
        sim = lb.Simulation(**dict(kw, phase=phase)).init_droplets(cen, rad)
        sim.step(1)
        v1 = stored_values(sim)
        sim.step(2)
        out[phase] = (v1, sim.fields(("phi",))["phi"].double().cpu().numpy())
        sim.close()
    (v_ro, s_ro), (v_tp, s_tp) = out["scatter"][0], out["pass"][0]
    ulp = {"f32": 2.0 ** -23, "f32s": 2.0 ** -23, "f32t": 2.0 ** -23, "bf16": 2.0 ** -7, "bf16t": 2.0 ** -7,
           "bf16t_sr": 2.0 ** -7}.get(storage, 2.0 ** -10)
    d1 = np.abs(v_ro - v_tp)
    if ulp == 2.0 ** -23:
        # FP32: the phase fields differ in the last bits
        bound = 64 * ulp * np.abs(v_tp).max()
    else:
        # 16-bit: a value that rounded the other way differs by one step
        bound = 2 * ulp * np.maximum(np.abs(v_tp), 2.0 ** -14)
    assert np.all(d1 <= bound), f"first step: stored values differ by {d1.max():.2e}"
    if s_tp.size:
        # recolouring scalars (FP32; the unit normal is sensitive where |g| is small)
        ds = np.abs(s_ro - s_tp).max()
        assert ds <= 1e-4 * np.abs(s_tp).max(), f"first step: scalars differ by {ds:.2e}"
    d = np.abs(out["scatter"][1] - out["pass"][1]).max()
    assert d < PHI_BAR[storage], f"phase field after three steps differs by {d:.2e}"


@pytest.mark.parametrize("shape", [(64, 16, 16), (70, 13, 12)])
@pytest.mark.parametrize("storage", ["f32", "f16t", "f64"])
def test_restore_repeats_the_uninterrupted_run_bit_for_bit(storage, shape):
    """lb_set_state drops the scattered phase field; the bootstrap pass
    scatters the restored state exactly as the collision pass that stored it
    did, so the restored run repeats the uninterrupted one bit for bit (also
    after a second restore on the same handle).  70 sites per row: the FP32
    and FP64 population rows are padded on the device, and the state moves
    through pitched copies."""
    kw = dict(lattice="D3Q27", storage=storage, nc="explicit", shape=shape, walls=(0, 1, 1),
              body_force=(1e-5, 0, 0))
    cen, rad = droplets(kw["shape"], "D3Q27")
    say(f"case restore {storage} {shape}")
    a = lb.Simulation(**kw).init_droplets(cen, rad)
    a.step(5)
    saved = a.get_state().clone()
    a.step(7)
    ref = a.get_state().cpu().numpy()
    b = lb.Simulation(**kw).init_droplets(cen, rad)
    b.set_state(saved)
    b.step(1)           # a step from the restored state ...
    b.set_state(saved)  # ... then a second restore: the scattered field is dropped again
    b.step(7)
    got = b.get_state().cpu().numpy()
    a.close()
    b.close()
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


@pytest.mark.parametrize("storage", ["f32", "f64", "f32t"])
def test_padded_population_rows_hold_the_canonical_state(storage):
    """The read-once two-copy step keeps FP32 / FP64 population rows padded to
    128 bytes on the device (70 sites per row here).  Its state after
    initialisation equals the unpadded two-pass handle's bit for bit, and any
    state set on it reads back unchanged."""
    kw = dict(lattice="D3Q27", storage=storage, nc="explicit", shape=(70, 13, 12), walls=(0, 1, 1),
              body_force=(1e-5, 0, 0))
    cen, rad = droplets(kw["shape"], "D3Q27")
    say(f"case padded rows {storage}")
    a = lb.Simulation(**dict(kw, phase="scatter")).init_droplets(cen, rad)
    b = lb.Simulation(**dict(kw, phase="pass")).init_droplets(cen, rad)
    sa, sb = a.get_state(), b.get_state()
    assert sa.shape == sb.shape
    assert torch.equal(sa.contiguous().view(torch.uint8), sb.contiguous().view(torch.uint8))
    g = torch.Generator(device="cpu").manual_seed(3)
    raw = torch.randint(0, 256, (sa.numel() * sa.element_size(),), generator=g, dtype=torch.uint8)
    a.set_state(raw.to(sa.device).view(sa.dtype).reshape(sa.shape))
    back = a.get_state().contiguous().view(torch.uint8).reshape(-1).cpu()
    assert torch.equal(back, raw)
    a.close()
    b.close()


def test_learned_closure_read_once_matches_two_pass():
    """Learned near-contact closure (BF16 matrix-core inference in the
    collision pass, explicit scan outside its input range): the read-once
    step against the two-pass step over five steps.  The network's BF16
    inputs can round differently where the phase fields differ in their last
    bits, so the bar is the closure's own resolution."""
    from paper_2405_14551_amd import workloads as W
    kw = dict(lattice="D3Q27", storage="f32", nc="mlp", shape=(70, 24, 20), walls=(0, 1, 1),
              body_force=(1e-5, 0, 0), u0=(0.02, 0.0, 0.0))
    cen = np.array([[20.3, 11.7, 9.6], [38.9, 12.2, 10.1]])
    rad = np.array([7.0, 7.0])
    lo = np.full(30, -2.0, np.float32)
    hi = np.full(30, 2.0, np.float32)
    res = {}
    for phase in ("scatter", "pass"):
        say(f"case closure {phase}")
        sim = lb.Simulation(**dict(kw, phase=phase))
        sim.mlp_set_weights(W.closure_init_weights())
        sim.mlp_set_ranges(lo, hi, 0.0)
        sim.init_droplets(cen, rad).step(5)
        f = sim.fields(("phi", "f_nc", "flags"))
        res[phase] = ({k: v.cpu().numpy() for k, v in f.items()}, sim.get_state().double().cpu().numpy())
        sim.close()
    (f_ro, s_ro), (f_tp, s_tp) = res["scatter"], res["pass"]
    assert (f_tp["flags"] & 2).sum() > 100, "the network should serve the interface sites"
    assert np.abs(f_ro["phi"] - f_tp["phi"]).max() < 1e-4
    assert np.abs(f_ro["f_nc"] - f_tp["f_nc"]).max() <= 0.02 * np.abs(f_tp["f_nc"]).max() + 1e-9
    assert rel(s_ro, s_tp) < 1e-4
