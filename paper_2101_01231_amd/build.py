"""Build libridg.so in-tree with hipcc for gfx950.

Usage: python -m paper_2101_01231_amd.build   (or build() from Python)

Host code (C ABI, FP64 precompute) and device code (kernels.hip) are compiled
into one shared library next to this file. All HIP code is compiled with the
packed-FP32 instructions disabled.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libridg.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = os.environ.get("RIDG_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I", os.path.join(HERE, "..", "include")]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
# per-unit device flags: the MFMA kernels keep their loop-carried accumulators in VGPRs (the
# default AGPR form copies them in and out around every tap and waits for the MFMA chain)
UNIT_FLAGS = {"k_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _stale(obj, src):
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    deps.append(os.path.join(HERE, "..", "include", "ridg.h"))
    return any(os.path.getmtime(x) > os.path.getmtime(obj) for x in deps)


def build(force=True):
    """Compile every source (force=True) or only the stale ones, then link libridg.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    objs = []
    for src in sorted(os.listdir(CSRC)):
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        if src.endswith(".cpp"):
            cmd = [HIPCC, "-x", "c++", *COMMON, "-I", os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__",
                   "-c", path, "-o", obj]
        elif src.endswith(".hip"):
            cmd = [HIPCC, "-x", "hip", *COMMON, *DEVICE, *UNIT_FLAGS.get(src, []), "-c", path, "-o", obj]
        else:
            continue
        objs.append(obj)
        if force or _stale(obj, path):
            jobs.append(cmd)
    procs = []
    for cmd in jobs:  # independent translation units compile in parallel
        print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    bad = [p.args for p in procs if p.wait() != 0]
    if bad:
        raise RuntimeError(f"compilation failed: {bad[0]}")
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(force="--force" in sys.argv)
    sys.exit(0)
