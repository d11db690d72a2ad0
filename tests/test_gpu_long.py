"""The 256 x 128 x 128 channel (64 droplets R = 10, near contact, walls y/z,
body force 1e-6) over its full length of 10000 steps, through the C ABI, in
five modes: plain FP32, FP16 total rounded to nearest and stochastically,
FP16C total, and the moment scheme.
Properties that hold at this size: the near-contact force keeps all 64
droplets apart, colour-A mass stays within the accumulated FP32 rounding of
10000 steps, and the flow stays far below the lattice sound speed."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402


@pytest.mark.parametrize("storage,scheme,rounding", [("f32", "populations", "nearest"),
                                                     ("f16t", "populations", "nearest"),
                                                     ("f16t", "populations", "stochastic"),
                                                     ("f16ct", "populations", "nearest"),
                                                     ("f32", "moments", "nearest")])
def test_channel_ten_thousand_steps(storage, scheme, rounding):
    print(f"case channel 10000 steps {storage} {scheme} {rounding}", flush=True)
    w = W.channel_3d()
    kw, cen, rad = W.sim_kwargs(w)
    sim = lb.Simulation(**dict(kw, storage=storage, scheme=scheme, rounding=rounding)).init_droplets(cen, rad)
    d0 = sim.diagnostics()
    assert int(d0[6]) == 64
    sim.step(10000)
    d = sim.diagnostics()
    sim.close()
    drift = abs(d[0] / d0[0] - 1)
    print(f"  droplets {int(d[6])}, max|u| {d[5]:.5f}, colour-A mass drift {drift:.2e}", flush=True)
    assert np.all(np.isfinite(d[:6]))
    assert int(d[6]) == 64
    # FP32 sums of O(1) populations lose about 1e-8 of the mass per step
    assert drift < 5e-4
    assert 1e-3 < d[5] < 0.05
