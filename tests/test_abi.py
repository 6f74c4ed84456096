"""The C-ABI library loads and exports every function include/ltl4c.h
declares; host-side behaviour that needs no GPU."""
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ltl4c.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ltl4c_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("ltl4c_create", "ltl4c_eval", "ltl4c_wait", "ltl4c_workspace_bytes", "ltl4c_set_layout",
                 "ltl4c_add_monitor", "ltl4c_add_property"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1411_2239_amd import lib
    so = lib.load()
    raw = ctypes.CDLL(lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name
    bound = {n for n, _, _ in lib.SIGNATURES}
    assert bound == set(declared_functions())


def test_status_strings():
    from paper_1411_2239_amd import lib
    so = lib.load()
    assert so.ltl4c_status_str(0) == b"ok"
    assert so.ltl4c_status_str(lib.ERANGE) == b"key wider than declared"
    assert so.ltl4c_status_str(12345) == b"unknown status"


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1411_2239_amd import lib
    so = lib.load()
    h = ctypes.c_void_p()
    st = so.ltl4c_create(ctypes.byref(h), 0)
    assert st in (lib.EDEVICE, lib.EINVAL)
    assert so.ltl4c_last_error()


def test_struct_sizes_match_header_layout(tmp_path):
    from paper_1411_2239_amd import lib
    # 8 u32 + 3*4 u32 + 2*256 bytes + 2 u32 + 3 predicates of 4 u32 + parent_events
    assert ctypes.sizeof(lib.Layout) == 4 * (4 + 4 * 3 + 1) + 512 + 4 * (2 + 3 * 4) + 4
    # and the header as a C compiler lays it out
    import os
    import subprocess
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "sizes.c"
    src.write_text('#include "ltl4c.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void) { printf("%zu %zu %zu %zu", sizeof(ltl4c_layout), '
                   'offsetof(ltl4c_layout, n_preds), sizeof(ltl4c_quant), sizeof(ltl4c_property)); return 0; }\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    sz, off_preds, qsz, psz = map(int, subprocess.run([str(exe)], check=True, capture_output=True,
                                                      text=True).stdout.split())
    assert sz == ctypes.sizeof(lib.Layout)
    assert off_preds == lib.Layout.n_preds.offset
    assert qsz == ctypes.sizeof(lib.Quant) and psz == ctypes.sizeof(lib.PropertyDesc)
    assert ctypes.sizeof(lib.Quant) == 16
    assert ctypes.sizeof(lib.PropertyDesc) == 8 + 4 * 16
