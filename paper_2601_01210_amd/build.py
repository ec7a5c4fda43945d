"""Build libjbfd.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with -ffp-contract=off (the
projection's double-precision arithmetic must not be fused; the filter
kernels call fma explicitly where they want it) and with packed FP32
instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjbfd.so")
SOURCES = ["api.hip", "project.hip", "densify.hip", "backward.hip",
           "stage2.hip", "cloud.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc",
              shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer: each -fsanitize=
# applies to the host pass only (-Xarch_host); the device code is unchanged.
# The resulting library needs the compiler's ASan runtime preloaded.
HOST_SANITIZE_FLAGS = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g",
]


def build(verbose: bool = False, out: str = LIB, extra_flags=()) -> str:
    """Compile every source into ``out`` (default: the in-tree libjbfd.so).
    The sources are compiled to objects in parallel, then linked."""
    objs, procs = [], []
    for s in SOURCES:
        obj = f"{out}.{os.path.splitext(s)[0]}.o"
        cmd = [hipcc(), *[f for f in HIPCC_FLAGS if f != "-shared"],
               *extra_flags, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, s), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
    failed = False
    for p in procs:
        log, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(log)
            failed = True
    try:
        if failed:
            raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
        tmp = out + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC",
               *extra_flags, *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed linking {os.path.basename(out)}")
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
