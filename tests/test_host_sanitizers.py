"""The library's host code (lbm_api.cpp, lbm_batch.cpp, thermo.cpp: validation, derived
constants, the Maxwell construction, batch bookkeeping, checkpoint argument checks)
built with AddressSanitizer and UndefinedBehaviorSanitizer by the host compiler and
driven through the C ABI on the CPU (tests/sanitize/driver.c).  The device launchers
are replaced by stand-ins that report no device (tests/sanitize/stubs.cpp); no GPU code
is built or run here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2106_01557_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

pytestmark = pytest.mark.slow


def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("host compilers not available")
    if not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("HIP headers not available")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include"),
           "-D__HIP_PLATFORM_AMD__"]
    objs = []
    for src in (os.path.join(CSRC, "lbm_api.cpp"), os.path.join(CSRC, "lbm_batch.cpp"),
                os.path.join(CSRC, "thermo.cpp"), os.path.join(HERE, "stubs.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", "-std=c++17", "-c", src, "-o", obj, "-Wall"] + san + inc, check=True)
        objs.append(obj)
    drv = str(tmp_path / "driver.o")
    subprocess.run(["gcc", "-std=c99", "-c", os.path.join(HERE, "driver.c"), "-o", drv, "-Wall", "-Wextra"] + san + inc,
                   check=True)
    exe = str(tmp_path / "host_paths")
    libdir = os.path.join(ROCM, "lib")
    subprocess.run(["g++", drv] + objs + ["-o", exe] + san + ["-L", libdir, "-lamdhip64", "-Wl,-rpath," + libdir],
                   check=True)
    supp = tmp_path / "lsan.supp"
    # the HIP runtime keeps process-lifetime allocations of its own
    supp.write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:librocprofiler-register\n")
    # (the runtime-library order check is off: the environment may preload a library of its own)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", LSAN_OPTIONS=f"suppressions={supp}")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, (out.returncode, out.stdout[-2000:], out.stderr[-4000:])
    assert "host paths ok" in out.stdout
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr
