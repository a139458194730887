"""Build libfnt.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfnt.so")
SOURCES = ["fnt_kernels.hip", "fnt_api.cpp", "fnt_session.cpp", "fnt_noalloc.hip", "fnt_cdc_long.hip"]
# measured GPU ceilings for the benchmark's roofline objects (not the receiver path)
PROBE_LIB = os.path.join(HERE, "libfntprobe.so")
PROBE_SOURCE = "peak_probe.hip"
ARCH = os.environ.get("FNT_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are kept out of every device code object.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    # the host pass warns that it does not know the packed-fp32 feature: harmless
    noise = "is not a recognized feature for this target"
    for line in r.stdout.splitlines():
        if noise not in line and line.strip():
            sys.stderr.write(line + "\n")


def build(force: bool = True, jobs: int = 3, out: str | None = None, defines=()) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    deps = srcs + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    deps.append(os.path.join(HERE, "..", "include", "fnt.h"))
    lib = out or LIB
    if not force and os.path.exists(lib) and all(os.path.getmtime(lib) >= os.path.getmtime(d) for d in deps):
        return lib
    objdir = os.path.join(HERE, "_build" if not defines else "_build_" + "_".join(d.replace("=", "") for d in defines))
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        lang = ["-x", "hip"]
        procs.append(["hipcc", *lang, *HIP_FLAGS, *["-D" + d for d in defines], "-c", s, "-o", o])
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, procs))
    tmp = lib + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, lib)
    if out is None and not defines:
        build_probe()
    return lib


COUNT_LIB = os.path.join(HERE, "libfnt_count.so")


def build_counting() -> str:
    """The test-only counting build: the same library with every Fermat-domain
    spectral product of the CDC and AEQ kernels counted (fnt_debug_product_counts)."""
    return build(force=True, out=COUNT_LIB, defines=("FNT_COUNT_PRODUCTS=1",))


def build_probe() -> str:
    tmp = PROBE_LIB + ".tmp"
    _run(["hipcc", "-x", "hip", *HIP_FLAGS, "-shared", "-o", tmp, os.path.join(CSRC, PROBE_SOURCE)])
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
