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
