"""The ctypes structures of the Python binding against the C header.

gcc compiles a small program that includes include/genpcg.h and prints
sizeof and offsetof of every field of every struct the binding mirrors; the
binding's ctypes classes must give the same names, order, offsets and sizes
(a field added on one side only shifts every later one)."""
import re
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "genpcg.h"
STRUCTS = ["gn_grid", "gn_material", "gn_loads", "gn_dd_opts", "gn_setup_report", "gn_solve_opts",
           "gn_server_opts", "gn_solve_report"]


def _header_fields(name):
    text = HEADER.read_text()
    m = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, re.S)
    assert m, name
    body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        # "double a, b, c" declares three fields
        for piece in decl.split(","):
            fm = re.search(r"([A-Za-z_][A-Za-z_0-9]*)\s*(\[[^\]]*\])?\s*$", piece.strip())
            assert fm, decl
            fields.append(fm.group(1))
    return fields


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "genpcg.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f in _header_fields(s):
            lines.append(f'  printf("{s} {f} %zu %zu\\n", offsetof({s}, {f}), sizeof((({s}*)0)->{f}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", str(ROOT / "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    lay = {}
    for line in out.splitlines():
        parts = line.split()
        if parts[1] == "size":
            lay.setdefault(parts[0], {})["__size__"] = int(parts[2])
        else:
            lay.setdefault(parts[0], {})[parts[1]] = (int(parts[2]), int(parts[3]))
    return lay


@pytest.mark.parametrize("name", STRUCTS)
def test_binding_struct_matches_the_header(name, c_layout):
    import ctypes

    from paper_1901_05188_amd import binding

    cls = getattr(binding, name)
    py_fields = [f for f, _ in cls._fields_]
    assert py_fields == _header_fields(name)
    lay = c_layout[name]
    assert ctypes.sizeof(cls) == lay["__size__"]
    for f in py_fields:
        off, size = lay[f]
        assert getattr(cls, f).offset == off, (name, f)
        assert getattr(cls, f).size == size, (name, f)
