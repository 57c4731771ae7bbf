"""CPU sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer): the
FP64 oracle, and the library's host code (lowering, lazy-qubit rewrite, pass
scheduler, kernel argument checks, Monte Carlo group schedule, argument
checks) compiled host-only, each driven by a small program in
tests/sanitize/.  No GPU is used; the sanitizers stop the program at the
first memory or undefined-behaviour error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_quant_ph_9804039_amd", "csrc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-ffp-contract=off",
                    "-o", exe, os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "qsim_oracle.c"), "-lm"])
    assert rc == 0, out
    rc, out = _run([exe], env=SAN_ENV, timeout=300)
    assert rc == 0 and "oracle driver: ok" in out, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out


def test_library_host_code_under_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    # the host sources as they are; the kernels' launchers are stubbed (no GPU)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".cpp"))
    srcs.append(os.path.join(ROOT, "tests", "sanitize", "kernel_stubs.cpp"))
    objs = []
    flags = ["-O1", "-g", "-std=c++17", "--cuda-host-only", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    drv = os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")
    for s in srcs + [drv]:
        o = str(tmp_path / (os.path.splitext(os.path.basename(s))[0] + "_host.o"))
        rc, out = _run([hipcc] + flags + ["-c", s, "-o", o])
        assert rc == 0, out
        objs.append(o)
    # link with the ROCm clang (the sanitizer runtime of the compiler that
    # instrumented the objects)
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "lib", "llvm", "bin",
                         "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/lib/llvm/bin/clang++"
    exe = str(tmp_path / "host_driver")
    rc, out = _run([clang, "-fsanitize=address,undefined", "-o", exe] + objs +
                   ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    assert rc == 0, out
    rc, out = _run([exe], env=SAN_ENV, timeout=600)
    assert rc == 0 and "0 failure(s)" in out, out
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out
