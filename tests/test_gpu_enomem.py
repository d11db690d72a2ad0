"""GPU: a handle larger than the device's free memory is refused with
LB_ENOMEM, everything allocated before the failing allocation is released,
and the library keeps working afterwards."""
import math
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


def test_out_of_device_memory_is_reported_and_released():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, total = torch.cuda.mem_get_info()
    # FP64 D3Q27 channels of 512^3 sites: two copies of 54 populations take
    # 116 GB per channel, so this many channels cannot all fit
    per = 2 * 54 * 8 * 512 ** 3
    n = math.ceil(free0 / per) + 1
    say(f"case ENOMEM: {n} channels of 512^3 FP64 D3Q27, {n * per / 1e9:.0f} GB of populations, "
        f"{free0 / 1e9:.0f} GB free")
    chans = [dict(shape=(512, 512, 512)) for _ in range(n)]
    with pytest.raises(lb.LBError) as err:
        lb.Ensemble(chans, lattice="D3Q27", storage="f64", nc="off")
    assert err.value.code == lb.LB_ENOMEM, err.value
    assert "out of device memory" in str(err.value) and "hipMalloc" in str(err.value), err.value
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    say(f"  free before {free0 / 1e9:.2f} GB, after {free1 / 1e9:.2f} GB")
    assert free1 >= free0 - (256 << 20), (free0, free1)
    # the library still creates and steps a handle
    sim = lb.Simulation(lattice="D3Q27", storage="f32", nc="explicit", shape=(32, 24, 20), walls=(0, 1, 1))
    sim.init_droplets(np.array([[15.3, 11.7, 9.6]]), np.array([6.0])).step(3)
    sim.sync()
    rho = sim.fields(("rho_a",))["rho_a"]
    assert torch.isfinite(rho).all() and float(rho.max()) > 0.5
    sim.close()
