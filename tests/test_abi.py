"""The C-ABI library loads and exports every function include/ladlasso.h
declares (no GPU needed: nothing is computed)."""
import ctypes
import os
import re

import pytest

import paper_2510_15649_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "ladlasso.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ladl_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    lib = ctypes.CDLL(L.LIB_PATH)
    names = header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(L.EXPORTED)


def test_host_only_entry_points():
    lib = L.lib()
    o = L.default_options()
    assert o.max_sweeps == 8 and o.max_rounds == 1 and o.schedule == -1
    assert abs(o.tol_s - 2 ** -20) < 1e-12
    assert o.chop_range == 2 ** -5
    assert lib.ladl_error_string(L.EINVAL).startswith(b"LADL_EINVAL")
    assert lib.ladl_error_string(L.OK) == b"LADL_OK"
    # NULL arguments are rejected before any device work
    assert lib.ladl_create(None) == L.EINVAL
    assert lib.ladl_plan_create(None, None, None, None) == L.EINVAL
    assert lib.ladl_solve_f32(*([None] * 12)) == L.EINVAL
    assert b"NULL" in lib.ladl_last_error_detail()
    assert lib.ladl_cv_create(None, None, None, None) == L.EINVAL
    assert lib.ladl_cv_run(*([None] * 9)) == L.EINVAL
    assert lib.ladl_cv_destroy(None) == L.OK


def test_no_packed_fp32_or_scalar_stores_in_device_code():
    """Device code is built without packed fp32 instructions and without
    stores through the scalar data cache (checked on the assembly hipcc
    emits for the kernels of this repository)."""
    import subprocess
    import tempfile
    csrc = os.path.join(ROOT, "paper_2510_15649_amd", "csrc")
    srcs = sorted(f for f in os.listdir(csrc) if f.endswith(".hip"))
    assert len(srcs) >= 3
    for name in srcs:
        with tempfile.TemporaryDirectory() as td:
            out = os.path.join(td, "k.s")
            subprocess.check_call(["/opt/rocm/bin/hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "-x", "hip",
                                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only",
                                   "-S", os.path.join(csrc, name), "-I", os.path.join(ROOT, "include"), "-o", out],
                                  stderr=subprocess.DEVNULL)
            asm = open(out).read()
        assert "v_pk_fma_f32" not in asm and "v_pk_add_f32" not in asm and "v_pk_mul_f32" not in asm, name
        assert not re.search(r"\bs_(store|atomic|buffer_store|dcache_wb)", asm), name


def test_binding_rejects_bad_tensors():
    """The binding checks dtype, device, contiguity and size before any
    pointer reaches the C ABI (CPU tensors are rejected before the library
    is asked for anything device-side)."""
    import torch
    from paper_2510_15649_amd import _check
    t = torch.zeros(8, dtype=torch.float32)
    with pytest.raises(ValueError, match="device tensor"):
        _check(t, "X", "f32", 8)
    with pytest.raises(ValueError, match="float32"):
        _check(t.double(), "X", "f32", 8)
    with pytest.raises(ValueError, match="int32"):
        _check(t, "status", "i32", 8)
    with pytest.raises(ValueError, match="required"):
        _check(None, "X", "f32", 8)
    _check(None, "b_init", "f32", 8, optional=True)


def header_structs():
    """Field names, in order, of every `typedef struct { ... } name;`."""
    src = open(os.path.join(ROOT, "include", "ladlasso.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", src, flags=re.S):
        fields = [re.findall(r"(\w+)\s*;", decl.strip() + ";")[0] for decl in body.split(";") if decl.strip()]
        out[name] = fields
    return out


BINDINGS = {"ladl_options": L.Options, "ladl_layout": L.Layout, "ladl_cv_layout": L.CVLayout}


def test_binding_structs_match_header(tmp_path):
    """The ctypes structures of the binding have the header's fields in the
    header's order, and the same size and offsets as a C compiler gives
    them: the library writes into them (ladl_default_options), so a
    mismatch would corrupt memory."""
    import shutil
    import subprocess
    structs = header_structs()
    assert set(BINDINGS) <= set(structs), structs.keys()
    for cname, cls in BINDINGS.items():
        assert [f for f, _ in cls._fields_] == structs[cname], cname
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ladlasso.h"', 'int main(void) {']
    for cname in BINDINGS:
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in structs[cname]:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, cls in BINDINGS.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)
