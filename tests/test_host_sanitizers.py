"""Host code of both libraries under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The libraries' sources are compiled with the sanitizers on their host side
(the device side is compiled without optimisation, only so that the objects
link; nothing here launches a kernel), linked with `host_abi_driver.c`, and
run: every C-ABI entry point that needs no GPU (descriptor validation,
workspace sizing and layout for many field sets, precisions and sizes up to
and past the 4 GiB per-lattice bound, argument checks on create, calls on a
NULL handle, error strings, the network's descriptor checks) must give the
status it should, with no sanitizer finding.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/bin/amdclang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm compilers not installed")
def test_c_abi_host_code_under_asan_and_ubsan(tmp_path):
    inc = os.path.join(ROOT, "include")
    src = os.path.join(ROOT, "paper_1003_0282_amd", "csrc")
    common = ["-O1", "-g", "--offload-arch=gfx950", "-std=c++17", "-I" + inc] + SAN + \
             ["-Xarch_device", "-O0", "-Xarch_device", "-g0"]
    objs = []
    for name in ("lbaxi", "lbnn"):
        o = str(tmp_path / (name + ".o"))
        _run([HIPCC] + common + ["-c", "-o", o, os.path.join(src, name + ".hip")])
        objs.append(o)
    drv = str(tmp_path / "driver.o")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I" + inc, "-c", "-o", drv, os.path.join(ROOT, "tests", "host_abi_driver.c")])
    exe = str(tmp_path / "driver")
    _run([HIPCC, "--offload-arch=gfx950", "-o", exe, drv] + objs +
         ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-4000:])
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert r.stdout.rstrip().endswith("ok")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    shutil.rmtree(tmp_path, ignore_errors=True)
