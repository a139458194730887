"""Host sanitizer runs (CPU only): the oracle's C code (gcc) and the library's
host code (hipcc, sanitizers on the host side only) built with
AddressSanitizer and UndefinedBehaviorSanitizer and driven over their edge
cases by tests/c/oracle_sanitize.c and tests/c/host_sanitize.c; any finding
aborts the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "c", "oracle_sanitize.c"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("ok"), r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CSRC = os.path.join(os.path.dirname(HERE), "paper_2405_04253_amd", "csrc")
SOURCES = ["fnt_api.cpp", "fnt_session.cpp", "fnt_noalloc.hip", "fnt_kernels.hip", "fnt_cdc_long.hip"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not available")
def test_host_code_asan_ubsan(tmp_path):
    """The library's host code with AddressSanitizer and UndefinedBehaviorSanitizer
    (host side only: -fsanitize= after -Xarch_host; the device code is built as
    usual), driven by tests/c/host_sanitize.c through every argument check and,
    without a GPU, the no-device paths of plan and session creation."""
    d = str(tmp_path)
    flags = ["-x", "hip", "-std=c++17", "-O1", "-g", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-fno-omit-frame-pointer", "-I", CSRC]
    procs = [subprocess.Popen([HIPCC] + flags + ["-c", os.path.join(CSRC, s), "-o", os.path.join(d, s + ".o")],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for s in SOURCES]
    for p, s in zip(procs, SOURCES):
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, (s, err[-3000:])
    lib = os.path.join(d, "libfnt_asan.so")
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined"] + [os.path.join(d, s + ".o") for s in SOURCES]
                   + ["-o", lib], check=True, capture_output=True, text=True)
    exe = os.path.join(d, "host_sanitize")
    subprocess.run([CLANG, "-std=c11", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    os.path.join(HERE, "c", "host_sanitize.c"), "-o", exe, "-L", d, "-lfnt_asan",
                    "-Wl,-rpath," + d, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert r.stdout.startswith("ok"), (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
