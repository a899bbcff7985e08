"""The C-ABI library loads and exports every entry point the header declares (CPU only)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spdem.h")
LIB = os.path.join(ROOT, "paper_2303_07819_amd", "libspdem.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sp_[a-z_]+)\s*\(", txt)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libspdem.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    names = declared()
    assert len(names) >= 13
    missing = [n for n in names if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libspdem.so not built")
def test_binding_loads_and_names_match_header():
    import paper_2303_07819_amd as sp
    lib = sp.load_library()
    for n in declared():
        assert hasattr(lib, n)
    assert sorted(sp.EXPORTED) == sorted(declared())


def test_binding_refuses_missing_library(tmp_path):
    import paper_2303_07819_amd as sp
    with pytest.raises(ImportError):
        sp._lib = None
        try:
            sp.load_library(str(tmp_path / "nope.so"))
        finally:
            sp._lib = None
