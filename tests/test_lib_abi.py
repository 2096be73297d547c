"""The C-ABI library loads and exports every function include/*.h declares (no GPU needed).

Only host-side entry points that touch no device are called here (version, status strings,
workspace sizing).  If the library has not been built in this checkout it is built first
(hipcc cross-compiles gfx950 code on a machine without a GPU).
"""
import ctypes
import os

import pytest

from paper_1101_0265_amd import build_lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(build_lib.LIB):
        build_lib.build()
    return ctypes.CDLL(build_lib.LIB)


def test_every_declared_symbol_is_exported(lib):
    declared = build_lib.header_symbols()
    assert "snf_purify_dense" in declared and "snf_step_dense" in declared
    missing = [s for s in declared if not hasattr(lib, s)]
    assert not missing, missing


def test_host_only_entry_points(lib):
    lib.snf_version.restype = ctypes.c_char_p
    assert lib.snf_version().decode().count(".") == 2
    lib.snf_strerror.restype = ctypes.c_char_p
    lib.snf_strerror.argtypes = [ctypes.c_int]
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        assert lib.snf_strerror(code)
    lib.snf_workspace_bytes.restype = ctypes.c_size_t
    lib.snf_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
    assert lib.snf_workspace_bytes(0, 0) == 0
    b64 = lib.snf_workspace_bytes(4096, 0)
    assert b64 >= 3 * 4096 * 4096 * 8
    assert lib.snf_workspace_bytes(4096, 3) > b64          # BF16 operand copies on top
    assert lib.snf_workspace_bytes(1000, 0) >= 3 * 1024 * 1024 * 8   # padded to 128


def test_binding_structs_match_header():
    """Field layout of the ctypes mirrors against the sizes the header implies."""
    from paper_1101_0265_amd import snf
    assert ctypes.sizeof(snf.Params) == 6 * 8 + 8 + 8 + 4 + 4 + 8 + 8 + 4 + 4 + 8
    assert ctypes.sizeof(snf.LogRec) == 4 * 4 + 6 * 8
    assert ctypes.sizeof(snf.Result) == 6 * 4 + 8 * 8 + snf.LOG_MAX + 8 + 8


def test_binding_offsets_match_compiled_header(tmp_path):
    """Every field offset and struct size of the ctypes mirrors against what a C compiler
    makes of include/snf.h."""
    import shutil
    import subprocess
    from paper_1101_0265_amd import snf
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"snf_params": snf.Params, "snf_log_rec": snf.LogRec, "snf_result": snf.Result,
               "snf_bsr": snf.Bsr}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "snf.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1101_0265_amd import snf
    monkeypatch.setattr(snf, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(snf, "_lib", None)
    with pytest.raises(ImportError):
        snf.lib()
