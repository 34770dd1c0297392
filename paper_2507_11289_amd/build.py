"""Compile libmd.so (HIP, gfx950) in-tree: ``python -m paper_2507_11289_amd.build``."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmd.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("md_device.hip", "md_host.hip")]
ARCH = os.environ.get("MD_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (hipcc would otherwise form them from float code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def command(out=LIB, extra=()):
    return ["/opt/rocm/bin/hipcc", *FLAGS, *extra, "-o", out, *SOURCES]


def build(verbose: bool = False, extra=()) -> str:
    cmd = command(extra=extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = LIB + ".tmp"
    cmd[cmd.index("-o") + 1] = tmp
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
