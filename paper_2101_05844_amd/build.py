"""Builds libasdual.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libasdual.so")
SOURCES = [os.path.join(HERE, "csrc", "asd_api.hip")]
HEADERS = [os.path.join(HERE, "csrc", "asd_internal.h"), os.path.join(HERE, "csrc", "asd_kernels.h"),
           os.path.join(HERE, "csrc", "asd_fast.h"), os.path.join(HERE, "csrc", "asd_adjoint.h"),
           os.path.join(ROOT, "include", "asdual.h")]


def hipcc_command(out=LIB, extra=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    return [hipcc, "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
            # packed FP32 instructions stay off (the compiler forms them from float code)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), *extra, "-o", out, *SOURCES]


def build(verbose: bool = True) -> str:
    cmd = hipcc_command()
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = LIB + ".tmp"
    cmd[cmd.index("-o") + 1] = tmp
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
