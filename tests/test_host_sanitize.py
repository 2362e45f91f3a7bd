"""The host side of the library (lattice validation, update schedule, gates,
option checks) under AddressSanitizer and UndefinedBehaviorSanitizer: the
host source is compiled with g++ and the sanitizers, linked with the
kernel objects of the regular build, and driven through the C ABI by
tests/host_sanitize/abi_fuzz.cpp on 3000 random and broken lattices.  No
GPU is touched: every call exercised is host-only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1910_09142_amd")
# every kernel object of the regular build (the sources besides hmps.cpp)
from paper_1910_09142_amd import build as _build  # noqa: E402
KERNEL_OBJS = [os.path.join(PKG, "_build", os.path.splitext(n)[0] + ".o")
               for n in _build.SOURCES if n.endswith(".hip")]


def test_host_code_is_clean_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    if not all(os.path.exists(o) for o in KERNEL_OBJS):
        pytest.skip("kernel objects not built (run the build first)")
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    host_obj = tmp_path / "hmps_san.o"
    subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", "-fPIC", *san,
         "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
         "-I", os.path.join(ROOT, "include"), "-c",
         os.path.join(PKG, "csrc", "hmps.cpp"), "-o", str(host_obj)],
        check=True, timeout=300)
    exe = tmp_path / "abi_fuzz"
    subprocess.run(
        ["g++", "-std=c++17", "-O1", "-g", *san,
         "-I", os.path.join(ROOT, "include"),
         os.path.join(ROOT, "tests", "host_sanitize", "abi_fuzz.cpp"),
         str(host_obj), *KERNEL_OBJS, "-L/opt/rocm/lib", "-lamdhip64",
         "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)],
        check=True, timeout=300)
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True,
                       timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "valid" in r.stdout
