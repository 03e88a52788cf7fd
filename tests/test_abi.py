"""The C-ABI library loads and exports every symbol that include/detlsh.h
declares; the ctypes binding declares exactly those (no compute calls: these
run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "detlsh.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(detlsh_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("detlsh_build_index", "detlsh_query", "detlsh_free", "detlsh_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2406_10938_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2406_10938_amd import build as b
        b.build(verbose=False)
    so = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(so, name), name


def test_binding_matches_header():
    from paper_2406_10938_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_struct_layouts(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals the C
    compiler's for the header's structs."""
    import subprocess

    from paper_2406_10938_amd import _lib
    structs = {"detlsh_build_opts": _lib.BuildOpts, "detlsh_query_opts": _lib.QueryOpts,
               "detlsh_info": _lib.Info, "detlsh_request_info": _lib.RequestInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "detlsh.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_server_rejects_null_handles_without_a_device():
    """The serving entry points check their handles before any HIP call."""
    from paper_2406_10938_amd import _lib
    L = _lib.lib()
    out = ctypes.c_void_p()
    assert L.detlsh_server_create(None, 1 << 30, 2, 64, ctypes.byref(out)) == _lib.EINVAL
    assert out.value is None
    assert b"NULL index" in L.detlsh_last_error()
    t = ctypes.c_uint64(7)
    assert L.detlsh_server_submit(None, None, 1, 10, 1.5, 0.1, None, None, None, ctypes.byref(t)) == _lib.EINVAL
    assert L.detlsh_server_wait(None, 1, 0, None) == _lib.EINVAL
    assert L.detlsh_server_cancel(None, 1) == _lib.EINVAL
    L.detlsh_server_destroy(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2406_10938_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()


def test_trim_without_cached_workspaces():
    """detlsh_trim with nothing cached makes no HIP call and is idempotent."""
    from paper_2406_10938_amd import _lib
    L = _lib.lib()
    L.detlsh_trim()
    L.detlsh_trim()
