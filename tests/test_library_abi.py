"""CPU checks of the C-ABI library: it is built, loads, and exports every
entry point the public header declares.  No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmd.h")
LIB = os.path.join(ROOT, "paper_1306_0788_amd", "liblbmd.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|int64_t|const char\*)\s+(lbmd_\w+)\s*\(", src, re.M)))


def test_header_declares_the_core_calls():
    names = declared()
    for core in ("lbmd_create", "lbmd_set_particles", "lbmd_step", "lbmd_get_fields"):
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("liblbmd.so not built (python -m paper_1306_0788_amd.build)")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lbmd_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_matches_header():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n)
    from paper_1306_0788_amd import lbmd
    assert sorted(lbmd.EXPORTS) == declared()


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_1306_0788_amd import lbmd
    monkeypatch.setattr(lbmd, "_lib", None)
    monkeypatch.setattr(lbmd, "LIBPATH", "/nonexistent/liblbmd.so")
    with pytest.raises(RuntimeError):
        lbmd.load()


def test_params_struct_layout_matches_header():
    """The ctypes mirror of lbmd_params has the C layout (checked with the C
    compiler on the header)."""
    from paper_1306_0788_amd import lbmd
    src = ('#include "lbmd.h"\n#include <stdio.h>\n#include <stddef.h>\n'
           'int main(){printf("%zu %zu %zu %zu %zu\\n", sizeof(lbmd_params), offsetof(lbmd_params, tau),'
           ' offsetof(lbmd_params, seed), offsetof(lbmd_params, check_every), offsetof(lbmd_params, rho0));'
           'return 0;}\n')
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", os.path.join(d, "t")])
        got = subprocess.run([os.path.join(d, "t")], capture_output=True, text=True).stdout.split()
    P = lbmd.Params
    want = [ctypes.sizeof(P), P.tau.offset, P.seed.offset, P.check_every.offset, P.rho0.offset]
    assert [int(g) for g in got] == want
