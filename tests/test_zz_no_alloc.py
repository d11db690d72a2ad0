"""GPU test of lb_nc_collect_noalloc, the collection of closure training rows
that allocates no device memory: through the C ABI, its rows, targets and
counts must equal those of lb_nc_collect bit for bit, on two calls in a row
(the second on a smaller lattice, so that the static scratch holds the first
call's larger contents when the second runs), and with a capacity below the
row count."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_14551_amd import lb, workloads as W  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _noalloc(sim, cap):
    """lb_nc_collect_noalloc through the C ABI into fresh buffers of cap rows
    (filled with NaN so that unwritten rows show)."""
    rows = torch.full((max(cap, 1), lb.MLP_ROW), float("nan"), dtype=torch.float32, device="cuda:0")
    tg = torch.full((max(cap, 1), 3), float("nan"), dtype=torch.float32, device="cuda:0")
    na, nf = ctypes.c_longlong(-1), ctypes.c_longlong(-1)
    torch.cuda.synchronize()
    rc = lb.lib().lb_nc_collect_noalloc(sim.h, 0, ctypes.c_void_p(rows.data_ptr()), ctypes.c_void_p(tg.data_ptr()),
                                        cap, ctypes.byref(na), ctypes.byref(nf))
    assert rc == lb.LB_OK, lb.lib().lb_last_error()
    return rows.cpu().numpy(), tg.cpu().numpy(), na.value, nf.value


def _compare(sim, label):
    ref_rows, ref_tg, na, nf = sim.nc_collect()
    ref_rows, ref_tg = ref_rows.cpu().numpy(), ref_tg.cpu().numpy()
    m = na + nf
    say(f"  {label}: {na} active + {nf} free rows")
    assert na > 0 and nf > 0
    rows, tg, na2, nf2 = _noalloc(sim, m)
    assert (na2, nf2) == (na, nf)
    np.testing.assert_array_equal(rows[:m].view(np.uint32), ref_rows.view(np.uint32))
    np.testing.assert_array_equal(tg[:m].view(np.uint32), ref_tg.view(np.uint32))
    # a capacity below the row count: the first cap rows, nothing beyond
    cap = m // 3
    rows, tg, na3, nf3 = _noalloc(sim, cap)
    assert (na3, nf3) == (na, nf)
    np.testing.assert_array_equal(rows[:cap].view(np.uint32), ref_rows[:cap].view(np.uint32))
    np.testing.assert_array_equal(tg[:cap].view(np.uint32), ref_tg[:cap].view(np.uint32))
    # counts only
    _, _, na4, nf4 = _noalloc(sim, 0)
    assert (na4, nf4) == (na, nf)


def test_noalloc_collection_matches_the_allocating_one_on_two_calls():
    # first call: 128 x 64 x 64 (2048 workgroups of the count kernel, more
    # than one per scan thread), droplets packed closer than the force range
    shape = (128, 64, 64)
    cen = W.fcc_slab_centres(shape, 7.0, 40, gap=2.5)
    say(f"noalloc call 1: D3Q27 f32 {shape}, {len(cen)} droplets")
    big = lb.Simulation(lattice="D3Q27", storage="f32", nc="explicit", shape=shape, walls=(0, 0, 1),
                        tau=1.0, A=0.01, beta=0.7, nc_A=0.02, nc_hmin=2.0, nc_hmax=3.0)
    big.init_droplets(cen, np.full(len(cen), 7.0))
    big.step(3)
    _compare(big, "128x64x64 D3Q27 f32")
    big.close()
    # second call: a smaller, ragged lattice (40 x 22 x 20 = 17600 sites, the
    # last count workgroup partly filled) on another velocity set and storage
    say("noalloc call 2: D3Q19 f64 (40, 22, 20), two droplets")
    small = lb.Simulation(lattice="D3Q19", storage="f64", nc="explicit", shape=(40, 22, 20), walls=(0, 1, 1),
                          tau=1.0, A=0.01, beta=0.7, body_force=(1e-6, 0.0, 0.0))
    small.init_droplets([[12.3, 10.7, 9.6], [26.9, 11.2, 10.1]], [6.0, 6.0])
    small.step(2)
    _compare(small, "40x22x20 D3Q19 f64")
    small.close()


def test_noalloc_collection_rejects_bad_arguments():
    sim = lb.Simulation(lattice="D3Q27", storage="f32", nc="explicit", shape=(16, 16, 16))
    L = lb.lib()
    na, nf = ctypes.c_longlong(), ctypes.c_longlong()
    # no step taken yet
    assert L.lb_nc_collect_noalloc(sim.h, 0, None, None, 0, ctypes.byref(na), ctypes.byref(nf)) == lb.LB_EINVAL
    sim.init_droplets([[8.0, 8.0, 8.0]], [4.0]).step(1)
    assert L.lb_nc_collect_noalloc(sim.h, 1, None, None, 0, ctypes.byref(na), ctypes.byref(nf)) == lb.LB_EINVAL
    assert L.lb_nc_collect_noalloc(sim.h, 0, None, None, 5, ctypes.byref(na), ctypes.byref(nf)) == lb.LB_EINVAL
    assert L.lb_nc_collect_noalloc(sim.h, 0, None, None, 0, ctypes.byref(na), ctypes.byref(nf)) == lb.LB_OK
    sim.close()
