"""GPU: the padded device layout of the populations (rows padded to 128
bytes, plane and scalar strides offset from the plane size) changes where
values live, not what is computed.  For every storage, streaming mode and
scheme, on a lattice whose rows are not a multiple of 128 bytes, a run with
the padded layout equals a run with plain rows and planes (LB_ROW_PAD=0,
LB_PLANE_PAD=0) bit for bit: the state, the phase field and the velocity
after several steps, and the state after a restore."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CEN = np.array([[20.3, 9.7, 8.6], [44.9, 10.2, 9.1]])
RAD = np.array([6.0, 6.0])

CASES = [
    dict(storage="f64"), dict(storage="f32"), dict(storage="f32s"), dict(storage="f16"), dict(storage="bf16"),
    dict(storage="f32t"), dict(storage="f16t"), dict(storage="bf16t"), dict(storage="f16ct"),
    dict(storage="f16t", rounding="stochastic"), dict(storage="f32", phase="pass"),
    dict(storage="f32", streaming="in_place"), dict(storage="f16t", streaming="in_place"),
    dict(storage="f32", scheme="moments"), dict(storage="f64", scheme="moments"),
]


def run(case, plain, monkeypatch):
    if plain:
        monkeypatch.setenv("LB_ROW_PAD", "0")
        monkeypatch.setenv("LB_PLANE_PAD", "0")
    else:
        monkeypatch.delenv("LB_ROW_PAD", raising=False)
        monkeypatch.delenv("LB_PLANE_PAD", raising=False)
    kw = dict(lattice="D3Q27", nc="explicit", shape=(70, 20, 18), walls=(0, 1, 1), body_force=(1e-5, 0, 0),
              u0=(0.02, 0.0, 0.0), tau=0.9, A=0.02)
    kw.update(case)
    sim = lb.Simulation(**kw).init_droplets(CEN, RAD)
    sim.step(7)
    sim.sync()
    st = sim.get_state().contiguous().view(torch.uint8).reshape(-1).cpu()
    f = {k: v.cpu() for k, v in sim.fields(("phi", "u")).items()}
    # restore and step again
    sim.set_state(sim.get_state().clone())
    sim.step(4)
    sim.sync()
    st2 = sim.get_state().contiguous().view(torch.uint8).reshape(-1).cpu()
    sim.close()
    return st, f, st2


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(f"{v}" for v in c.values()))
def test_padded_layout_equals_plain_layout_bitwise(case, monkeypatch):
    say(f"case padded vs plain layout {case}")
    pad = run(case, False, monkeypatch)
    plain = run(case, True, monkeypatch)
    assert torch.equal(pad[0], plain[0]), "state after 7 steps"
    assert torch.equal(pad[1]["phi"], plain[1]["phi"]) and torch.equal(pad[1]["u"], plain[1]["u"])
    assert torch.equal(pad[2], plain[2]), "state after a restore and 4 more steps"
