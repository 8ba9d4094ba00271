"""The library's host code (argument validation, planner, offset tables, autotune cache parser) built
with AddressSanitizer and UndefinedBehaviorSanitizer and driven through the C ABI on valid and invalid
trees (tests/sanitize/planner_driver.cpp). Host only: the kernels' objects are linked unchanged and
never launched."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_19650_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
KERNEL_OBJECTS = ["chol.hip.o", "eig.hip.o", "eig_band.hip.o", "gemm.hip.o", "noalloc.hip.o"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    if not all(os.path.exists(os.path.join(BUILD, o)) for o in KERNEL_OBJECTS):
        from paper_2601_19650_amd import build_lib
        build_lib.build(verbose=False)
    d = tmp_path_factory.mktemp("sanitized")
    inc = ["-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    api = str(d / "cbc_api.o")
    drv = str(d / "driver.o")
    exe = str(d / "driver")
    steps = [
        ["g++", "-std=c++17", "-O1", "-g"] + SAN + inc + ["-c", os.path.join(CSRC, "cbc_api.cpp"),
                                                        "-o", api],
        ["g++", "-std=c++17", "-O1", "-g"] + SAN + inc + [
            "-c", os.path.join(ROOT, "tests", "sanitize", "planner_driver.cpp"), "-o", drv],
        ["g++"] + SAN + [api, drv] + [os.path.join(BUILD, o) for o in KERNEL_OBJECTS] + [
            "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
    return exe, d


def test_planner_under_address_and_undefined_sanitizers(driver):
    exe, d = driver
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([exe, str(d / "tune.txt")], capture_output=True, text=True, env=env,
                       timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "failures 0" in r.stdout
    # every tree went through query, plan_info and plan_bonds
    assert r.stdout.count("plan_bonds ") == 14
