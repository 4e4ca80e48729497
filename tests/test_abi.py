"""CPU checks of the C ABI: the header is valid C, and the built library
loads and exports every function the header declares (no GPU calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lobpcg.h")
LIB = os.path.join(ROOT, "paper_2305_06668_amd", "liblobpcg.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(lobpcg_\w+)\s*\(", text, re.M)))


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "lobpcg.h"\nint main(void){ lobpcg_stats s; (void)s; return 0; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), "-c", str(src), "-o", str(tmp_path / "t.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    names = declared()
    assert len(names) >= 20
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_names_match_header():
    import paper_2305_06668_amd as P

    assert sorted(P.EXPORTED) == declared()
    for n in declared():
        assert callable(getattr(P, n))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings_and_null_handle():
    import paper_2305_06668_amd as P

    assert P.lobpcg_status_string(P.OK) == "ok"
    assert "orthonormalisation" in P.lobpcg_status_string(P.ERR_ORTHO_FAILED)
    lib = ctypes.CDLL(LIB)
    lib.lobpcg_solve.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
    assert lib.lobpcg_solve(None, 1, 1e-8) == P.ERR_INVALID_ARG
    lib.lobpcg_create.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    assert lib.lobpcg_create(0, 0, ctypes.byref(h)) == P.ERR_INVALID_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_constants_equal_header_defines():
    """Every integer #define LOBPCG_X of the header is the binding's X."""
    import paper_2305_06668_amd as P

    defs = {m.group(1): int(m.group(2))
            for m in re.finditer(r"#define LOBPCG_([A-Z0-9_]+)\s+(-?\d+)\b", open(HEADER).read())}
    assert len(defs) >= 30
    for name, value in defs.items():
        assert getattr(P, name) == value, name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("struct", ["lobpcg_stats", "lobpcg_ortho_info"])
def test_struct_layouts_match_the_c_compiler(tmp_path, struct):
    """Field offsets and sizes of the ctypes mirrors equal what a C compiler
    lays out from the header (a reordered or resized field would otherwise
    shift every later statistic silently)."""
    import paper_2305_06668_amd as P

    cls = getattr(P, struct)
    fields = [f for f, _ in cls._fields_]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lobpcg.h"', "int main(void) {",
             f'  printf("sizeof %zu\\n", sizeof({struct}));']
    lines += [f'  printf("{f} %zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    assert int(out["sizeof"]) == ctypes.sizeof(cls)
    for f in fields:
        assert int(out[f]) == getattr(cls, f).offset, f
