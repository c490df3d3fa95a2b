"""The C-ABI library loads and exports every entry point its header declares (no GPU needed)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kron_regress.h")
LIB = os.path.join(ROOT, "paper_2209_04876_amd", "libkron_regress.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:kr_status|const char\*|int64_t)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("kron_regress", "kron_ridge", "kron_loss", "kron_exact", "kr_create", "kr_destroy"):
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        import subprocess, sys
        subprocess.check_call([sys.executable, os.path.join(ROOT, "paper_2209_04876_amd", "build.py")])
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.kr_version.restype = ctypes.c_char_p
    assert lib.kr_version().startswith(b"kron_regress")


def test_binding_names_match_the_abi():
    import paper_2209_04876_amd as kr
    for n in ("kron_regress", "kron_ridge", "kron_loss", "kron_exact"):
        assert callable(getattr(kr, n))


def test_struct_layouts_match_the_header(tmp_path):
    """ctypes mirrors of kr_problem / kr_opts / kr_info have the C layout (gcc)."""
    import subprocess
    import paper_2209_04876_amd as kr
    structs = {"kr_problem": kr.Problem, "kr_opts": kr.Opts, "kr_info": kr.Info,
               "kr_response_gen": kr.ResponseGenC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "kron_regress.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
