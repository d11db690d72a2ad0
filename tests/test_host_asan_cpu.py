"""The library's host code under AddressSanitizer, on the CPU.

The C-ABI translation unit (api.hip) is compiled with the sanitizer on its
host side only (its device code is built as usual), linked with the other
translation units' objects of the in-tree build and a C driver
(tests/asan_driver.c), and run without a GPU: defaults, lattice tables,
parameter validation of single lattices and ensembles, NULL arguments of
every entry point, error strings and the no-device error of lb_create.  The
sanitizer aborts on an invalid host memory access and reports leaks at
exit."""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"


def test_host_code_under_address_sanitizer(tmp_path):
    if os.path.exists("/dev/kfd"):
        pytest.skip("the driver expects a machine without a GPU")
    from paper_2405_14551_amd import build as B
    objs = [o for o in sorted(glob.glob(os.path.join(B.BUILD, "*.o"))) if os.path.basename(o) != "api.hip.o"]
    if not objs:
        pytest.skip("build the library first: the other translation units' objects are linked from its build")
    if not os.path.exists(CLANG):
        pytest.skip("no ROCm clang")
    flags = [f for f in B.CFLAGS if f != "-O3"]
    api = str(tmp_path / "api_asan.o")
    cmd = [B.HIPCC, *flags, "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
           "-c", os.path.join(B.CSRC, "api.hip"), "-o", api]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    drv_o = str(tmp_path / "drv.o")
    r = subprocess.run([CLANG, "-g", "-O1", "-fsanitize=address", "-fno-omit-frame-pointer",
                        "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "asan_driver.c"),
                        "-o", drv_o], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "drv")
    r = subprocess.run([CLANG + "++", "-fsanitize=address", "-o", exe, drv_o, api, *objs, "-L/opt/rocm/lib",
                        "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "0 failed expectations" in r.stdout, out[-2000:]
