"""Builds libasdual.so (HIP, gfx950) in-tree with hipcc.

The library is one host/general translation unit (asd_api.hip), the
iteration-kernel launches of asd_iter.hip compiled once per active-mask
count (-DASD_NM=0..ASD_MAX_MASKS), the Saddle Point unit (asd_sp.hip,
compiled without floating-point contraction), and the bound-gradient
launches of asd_grad.hip and the FP64 final sums of asd_final.hip, again once
per active-mask count; the objects compile in
parallel and are linked into one shared library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libasdual.so")
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
MAX_MASKS = 8  # ASD_MAX_MASKS in include/asdual.h
SOURCES = [os.path.join(CSRC, "asd_api.hip"), os.path.join(CSRC, "asd_iter.hip"), os.path.join(CSRC, "asd_sp.hip"),
           os.path.join(CSRC, "asd_grad.hip"), os.path.join(CSRC, "asd_final.hip")]
HEADERS = [os.path.join(CSRC, h) for h in ("asd_internal.h", "asd_kernels.h", "asd_fast.h", "asd_adjoint.h",
                                           "asd_plan.h")] + [os.path.join(ROOT, "include", "asdual.h")]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def compile_flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
            # packed FP32 instructions stay off (the compiler forms them from float code)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def units():
    """(source, object, extra flags) of every translation unit."""
    out = [(SOURCES[0], os.path.join(OBJDIR, "asd_api.o"), [])]
    for nm in range(MAX_MASKS + 1):
        out.append((SOURCES[1], os.path.join(OBJDIR, f"asd_iter_nm{nm}.o"), [f"-DASD_NM={nm}"]))
    out.append((SOURCES[2], os.path.join(OBJDIR, "asd_sp.o"), ["-ffp-contract=off"]))
    for nm in range(MAX_MASKS + 1):
        out.append((SOURCES[3], os.path.join(OBJDIR, f"asd_grad_nm{nm}.o"), [f"-DASD_NM={nm}"]))
        out.append((SOURCES[4], os.path.join(OBJDIR, f"asd_final_nm{nm}.o"), [f"-DASD_NM={nm}"]))
    return out


def hipcc_command(out=LIB, extra=()):
    """Link command of the shared library (after the objects are built)."""
    return [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *extra, "-o", out,
            *[o for _, o, _ in units()]]


def build(verbose: bool = True, jobs: int = 0) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(units()), os.cpu_count() or 4)
    cmds = [[_hipcc(), *compile_flags(), *fl, "-c", "-o", obj, srcf] for srcf, obj, fl in units()]

    def run(cmd):
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return cmd, r.returncode, r.stdout

    failed = []
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, rc, log in ex.map(run, cmds):
            if verbose:
                print(" ".join(cmd), flush=True)
            # hipcc's host pass does not know the packed-FP32 feature: harmless
            lines = [ln for ln in log.splitlines() if "packed-fp32-ops" not in ln]
            if lines and (verbose or rc):
                print("\n".join(lines), flush=True)
            if rc:
                failed.append(cmd)
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = hipcc_command(out=tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
