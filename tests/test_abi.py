"""The C-ABI library loads and exports every symbol the header declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2101_05844_amd", "libasdual.so")
HEADER = os.path.join(ROOT, "include", "asdual.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("asd_net_create", "asd_plan_create", "asd_solve", "asd_run", "asd_bound", "asd_eval",
              "asd_oracle", "asd_interval_bounds", "asd_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (shares the HIP runtime the library links)
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n
    lib.asd_abi_version.restype = ctypes.c_int32
    assert lib.asd_abi_version() == 3
    lib.asd_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.asd_last_error(), bytes)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_validation_without_gpu():
    """Argument checks happen before any device work."""
    from paper_2101_05844_amd import asdual as A
    L = A.lib()
    descs = (A.LayerDesc * 2)()
    h = ctypes.c_void_p()
    assert L.asd_net_create(descs, 2, ctypes.byref(h)) == 1  # NULL weights
    assert L.asd_net_create(descs, 1, ctypes.byref(h)) == 1  # too few layers
    fake = ctypes.c_void_p(256)
    for i in range(2):
        descs[i].kind = A.ASD_LAYER_DENSE
        descs[i].W = fake
        descs[i].b = fake
    descs[0].in_c, descs[0].out_c = 5, 8
    descs[1].in_c, descs[1].out_c = 7, 1   # mismatch
    assert L.asd_net_create(descs, 2, ctypes.byref(h)) == 1
    assert b"inputs" in L.asd_last_error()
    descs[1].in_c = 8
    assert L.asd_net_create(descs, 2, ctypes.byref(h)) == 0
    p = A.asd_params_default()
    nbytes = ctypes.c_size_t()
    assert L.asd_plan_workspace_size(h, 4, ctypes.byref(p), ctypes.byref(nbytes)) == 0
    assert nbytes.value > 0
    assert L.asd_plan_workspace_size(h, 0, ctypes.byref(p), ctypes.byref(nbytes)) == 1  # empty batch
    assert b"S must be" in L.asd_last_error()
    p.max_masks = 99
    assert L.asd_plan_workspace_size(h, 4, ctypes.byref(p), ctypes.byref(nbytes)) == 1
    L.asd_net_destroy(h)


STRUCTS = {"asd_layer_desc": "LayerDesc", "asd_params": "Params", "asd_batch": "Batch", "asd_counts": "Counts",
           "asd_kernel_time": "KernelTime", "asd_tuning": "Tuning", "asd_eval_out": "EvalOut"}


def test_binding_structs_match_header(tmp_path):
    """Every struct the binding passes through ctypes has the size and field
    offsets the C compiler gives the header's declaration (gcc, host only)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("gcc or the HIP headers are missing")
    from paper_2101_05844_amd import asdual as A
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "asdual.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(A, pyname)._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    for cname, pyname in STRUCTS.items():
        cls = getattr(A, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
