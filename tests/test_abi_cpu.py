"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every symbol the header declares, its velocity tables agree with the
oracle's, and argument validation rejects bad parameters before touching a
device.  No compute call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2405_14551_amd import lb
from oracle.lattice import make_lattice, LATTICES

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.skipif(not os.path.exists(lb.LIB_PATH), reason="library not built")


def _declared_symbols():
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(lb_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = lb.lib()
    declared = _declared_symbols()
    assert {"lb_create", "lb_init_droplets", "lb_step", "lb_fields", "lb_destroy"} <= declared
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} declared in include/ but not exported"
    assert set(lb.EXPORTED) <= declared


@pytest.mark.parametrize("name", LATTICES)
def test_tables_agree_with_oracle(name):
    c, w, opp, B = lb.lattice_table(name)
    ref = make_lattice(name)
    assert np.array_equal(c, ref.c)
    assert np.array_equal(opp, ref.opp)
    np.testing.assert_array_equal(w, ref.w)
    np.testing.assert_allclose(B, ref.B, rtol=0, atol=2e-16)


def _create(**kw):
    p = lb.make_params(**kw)
    h = ctypes.c_void_p()
    rc = lb.lib().lb_create(ctypes.byref(p), 1, None, ctypes.byref(h))
    if rc == 0:
        lb.lib().lb_destroy(h)
    return rc


@pytest.mark.parametrize("kw", [
    dict(tau=0.5),
    dict(tau=0.3),
    dict(tau_b=0.5),
    dict(scheme="moments", storage="f16"),                  # moments in FP64 / FP32 only
    dict(scheme="moments", storage="f32t"),
    dict(scheme="moments", nc="mlp"),
    dict(scheme="moments", streaming="in_place"),
    dict(tau_b=-1.0),
    dict(tau_b=float("nan")),
    dict(shape=(0, 4, 4)),
    dict(lattice="D2Q9", shape=(8, 8, 2)),
    dict(lattice="D2Q9", shape=(8, 8, 1), walls=(0, 0, 1)),
    dict(lattice="D2Q9", shape=(8, 8, 1), body_force=(0, 0, 1e-5)),
    dict(phi_interface=1.0),
    dict(nc="explicit", nc_hmax=5.0),
    dict(nc="explicit", nc_hmin=0.0),
    dict(nc="explicit", shape=(64, 3, 8)),
    dict(rho0=-1.0),
    dict(shape=(2048, 2048, 2048)),
    dict(nc="mlp", lattice="D2Q9", shape=(16, 16, 1)),      # the learned closure is 3D
    dict(nc="mlp", storage="f16"),                          # per-colour 16-bit storage
    dict(nc="mlp", shape=(64, 3, 8)),
    dict(rounding="stochastic"),                            # FP32 storage rounds nothing
    dict(rounding="stochastic", storage="f16"),             # per-colour 16-bit
    dict(rounding="stochastic", storage="f16ct"),           # FP16C has its own encoder
    dict(rounding="stochastic", storage="f16t", nc="mlp"),  # not with the learned closure
])
def test_invalid_params_rejected(kw):
    assert _create(**kw) == lb.LB_EINVAL


def test_bad_enum_and_null():
    L = lb.lib()
    p = lb.make_params()
    p.lattice = 7
    h = ctypes.c_void_p()
    assert L.lb_create(ctypes.byref(p), 1, None, ctypes.byref(h)) == lb.LB_EINVAL
    p = lb.make_params()
    p.storage = 9
    assert L.lb_create(ctypes.byref(p), 1, None, ctypes.byref(h)) == lb.LB_EINVAL
    p = lb.make_params()
    p.wall[0] = 2
    assert L.lb_create(ctypes.byref(p), 1, None, ctypes.byref(h)) == lb.LB_EINVAL
    p = lb.make_params()
    p.scheme = 2
    assert L.lb_create(ctypes.byref(p), 1, None, ctypes.byref(h)) == lb.LB_EINVAL
    p = lb.make_params()
    p.streaming = 2
    assert L.lb_create(ctypes.byref(p), 1, None, ctypes.byref(h)) == lb.LB_EINVAL
    p = lb.make_params(storage="f16t")
    p.rounding = 2
    assert L.lb_create(ctypes.byref(p), 1, None, ctypes.byref(h)) == lb.LB_EINVAL
    p = lb.make_params()
    assert L.lb_create(ctypes.byref(p), 2, None, ctypes.byref(h)) == lb.LB_EINVAL
    assert L.lb_create(None, 1, None, ctypes.byref(h)) == lb.LB_EINVAL
    assert L.lb_destroy(None) == lb.LB_OK
    assert L.lb_step(None, 1) == lb.LB_EINVAL
    assert L.lb_error_string(lb.LB_ENUMERIC).decode().startswith("numerical watchdog")


def test_valid_params_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    assert _create() == lb.LB_ENODEV


def test_ensemble_argument_checks():
    L = lb.lib()
    h = ctypes.c_void_p()
    arr = (lb.LbParams * 2)()
    arr[0] = lb.make_params(lattice="D3Q19", storage="f32", shape=(16, 8, 8))
    arr[1] = lb.make_params(lattice="D3Q27", storage="f32", shape=(16, 8, 8))
    assert L.lb_create(arr, 2, None, ctypes.byref(h)) == lb.LB_EINVAL      # lattices differ
    arr[1] = lb.make_params(lattice="D3Q19", storage="f16", shape=(16, 8, 8))
    assert L.lb_create(arr, 2, None, ctypes.byref(h)) == lb.LB_EINVAL      # storages differ
    arr[0] = lb.make_params(lattice="D3Q19", storage="f16", shape=(16, 8, 8))
    assert L.lb_create(arr, 2, None, ctypes.byref(h)) == lb.LB_EINVAL      # per-colour 16-bit ensemble
    assert L.lb_create(arr, 0, None, ctypes.byref(h)) == lb.LB_EINVAL
    arr[0] = lb.make_params(lattice="D3Q19", storage="f32", nc="mlp", shape=(16, 8, 8))
    arr[1] = lb.make_params(lattice="D3Q19", storage="f32", nc="mlp", shape=(16, 8, 8))
    assert L.lb_create(arr, 2, None, ctypes.byref(h)) == lb.LB_EINVAL      # no closure in ensembles
    arr[0] = lb.make_params(lattice="D3Q19", storage="f32", shape=(16, 8, 8))
    arr[1] = lb.make_params(lattice="D3Q19", storage="f32", shape=(16, 8, 8), streaming="in_place")
    assert L.lb_create(arr, 2, None, ctypes.byref(h)) == lb.LB_EINVAL      # ensembles use two copies
    arr[1] = lb.make_params(lattice="D3Q19", storage="f32", shape=(16, 8, 8), scheme="moments")
    assert L.lb_create(arr, 2, None, ctypes.byref(h)) == lb.LB_EINVAL      # and the population scheme
    arr[0] = lb.make_params(lattice="D3Q19", storage="f16t", shape=(16, 8, 8))
    arr[1] = lb.make_params(lattice="D3Q19", storage="f16t", shape=(16, 8, 8), rounding="stochastic")
    assert L.lb_create(arr, 2, None, ctypes.byref(h)) == lb.LB_EINVAL      # and round to nearest


def test_closure_calls_reject_null_arguments():
    L = lb.lib()
    na, nf = ctypes.c_longlong(), ctypes.c_longlong()
    assert L.lb_nc_collect(None, 0, None, None, 0, ctypes.byref(na), ctypes.byref(nf)) == lb.LB_EINVAL
    assert L.lb_nc_collect_noalloc(None, 0, None, None, 0, ctypes.byref(na), ctypes.byref(nf)) == lb.LB_EINVAL
    assert L.lb_mlp_set_weights(None, None, lb.MLP_PARAMS) == lb.LB_EINVAL
    assert L.lb_mlp_get_weights(None, None, lb.MLP_PARAMS) == lb.LB_EINVAL
    assert L.lb_mlp_train(None, None, None, 1, None, 1, 32, 1e-3, None) == lb.LB_EINVAL
    assert L.lb_mlp_gradient(None, None, None, 1, None, None) == lb.LB_EINVAL
    assert L.lb_mlp_infer(None, None, None, 1) == lb.LB_EINVAL
