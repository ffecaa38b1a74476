"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers are built in a temporary directory and run:
  * the FP64 oracle (plain C, OpenMP), compiled by gcc with both sanitizers,
    through every one of its entry points on small systems;
  * libtbsma's host code (wire builder, argument and layout checks, workspace
    sizes, error messages), compiled by hipcc with the sanitizers on the host side only;
    every call there returns before a device is touched.
A sanitizer report or a failed check makes the driver exit non-zero.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = {**os.environ,
       "ASAN_OPTIONS": "abort_on_error=0:halt_on_error=1:exitcode=99:detect_leaks=1",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=98",
       "OMP_NUM_THREADS": "4"}


def _run(exe, env=ENV):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-ffp-contract=off", "-o", exe,
                           os.path.join(HERE, "oracle_driver.c"), "-lm"])
    out = _run(exe)
    assert "all checks passed" in out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_library_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1311_3890_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    # host-side instrumentation only (the device code is built as usual)
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    objs = []
    for src in ("tbsma_api.hip", "tbsma_kernels.hip"):
        o = str(tmp_path / (src + ".o"))
        subprocess.check_call(["hipcc", "-c", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
                               "-fPIC", "-Xclang", "-target-feature", "-Xclang",
                               "-packed-fp32-ops", *host_san, *inc, "-o", o,
                               os.path.join(csrc, src)],
                              stderr=subprocess.DEVNULL)
        objs.append(o)
    drv = str(tmp_path / "abi_host_driver.o")
    clang = "/opt/rocm/llvm/bin/clang++"
    sanitize_link = "-fsanitize=address,undefined"
    subprocess.check_call([clang, "-c", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                           sanitize_link, *inc, "-o", drv,
                           os.path.join(HERE, "abi_host_driver.cpp")])
    exe = str(tmp_path / "abi_host_driver")
    subprocess.check_call([clang, sanitize_link, "-o", exe, drv, *objs,
                           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    # the HIP runtime's own allocations are not this library's: leaks are
    # checked in the oracle driver only
    env = {**ENV, "ASAN_OPTIONS": ENV["ASAN_OPTIONS"].replace("detect_leaks=1",
                                                              "detect_leaks=0")}
    out = _run(exe, env)
    assert "all checks passed" in out
