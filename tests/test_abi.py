"""C-ABI contract checks that need no GPU: the built library loads, exports
every function include/tomoadmm.h declares, and its structs have the sizes the
binding assumes.  Nothing here launches a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tomoadmm.h")
LIB = os.path.join(ROOT, "paper_2410_06106_amd", "libtomoadmm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtomoadmm.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("tomo_project", "tomo_backproject", "admm_local_update", "admm_consensus",
                 "quantize_kmeans", "quantize_dct", "tomo_create", "tomo_destroy"):
        assert must in names, names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in tomoadmm.h but not exported"


def test_binding_covers_every_declared_symbol():
    from paper_2410_06106_amd import tomoadmm
    assert sorted(tomoadmm.EXPORTED) == declared_functions()


def test_struct_layouts():
    from paper_2410_06106_amd import tomoadmm as T
    assert ctypes.sizeof(T.tomo_node) == 80
    assert ctypes.sizeof(T.tomo_msg) == 48
    assert ctypes.sizeof(T.tomo_quant) == 16
    assert ctypes.sizeof(T.tomo_geom) == 8
    assert ctypes.sizeof(T.tomo_proj_item) == 40
    assert ctypes.sizeof(T.tomo_reg) == 56


def test_binding_structs_match_the_c_header(tmp_path):
    """Every field offset and struct size of the ctypes binding equals what a C
    compiler makes of include/tomoadmm.h (compiled as C with gcc)."""
    import shutil
    import subprocess
    from paper_2410_06106_amd import tomoadmm as T
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = [T.tomo_geom, T.tomo_node, T.tomo_quant, T.tomo_msg, T.tomo_proj_item, T.tomo_reg]
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void) {']
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in st._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for st in structs:
        name = st.__name__
        assert got[(name, "size")] == ctypes.sizeof(st), name
        for field, _ in st._fields_:
            assert got[(name, field)] == getattr(st, field).offset, (name, field)


def test_status_strings_and_null_context(lib):
    lib.tomo_status_string.restype = ctypes.c_char_p
    assert lib.tomo_status_string(0) == b"ok"
    assert lib.tomo_status_string(1) == b"invalid argument"
    assert lib.tomo_status_string(99) == b"unknown status"
    # a null context is rejected before any HIP call
    assert lib.tomo_destroy(None) == 1
    assert lib.tomo_project(None, ctypes.c_int64(0), None, 0, None, None, None) == 1
