"""CPU checks of the C ABI: the library loads and exports every function the
header declares; the binding's struct layouts match the header's."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pod2g.h")
LIB = os.path.join(ROOT, "paper_2207_02543_amd", "libpod2g.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("pod2g_", "pcg_"))))


def test_header_declares_the_boundary():
    d = _declared()
    for name in ["pod2g_assemble", "pod2g_setup", "pod2g_apply", "pcg_solve", "pod2g_strerror",
                 "pod2g_pattern_build", "pod2g_pod_basis"]:
        assert name in d


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_structs_match():
    import ctypes as C
    from paper_2207_02543_amd import capi
    assert set(capi.exported_symbols()) == set(_declared())
    assert C.sizeof(capi.Mesh) == 32
    assert C.sizeof(capi.Pattern) == 72
    assert capi.Prec.omega.offset == 96
    assert C.sizeof(capi.Prec) == 96 + 8 + 13 * 8 + 8
    assert capi.Prec.smoother.offset == 96 + 8 + 13 * 8
    assert C.sizeof(capi.SlotInfo) == 24 and C.sizeof(capi.Group) == 56
    assert C.sizeof(capi.Timer) == 40
    assert capi.strerror(capi.ENOTSPD).startswith("coarse matrix")
    # size queries are host-only and validate their arguments
    m = capi.make_mesh(2, 32, 8)
    assert capi.pod2g_pattern_bytes(m) > 0
    assert capi.pod2g_pattern_bytes(capi.make_mesh(4, 32, 8)) == 0
    assert capi.pod2g_pod_basis_bytes(100, 300, 5) == 0   # more than 256 snapshots


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2207_02543_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, flags=re.M), fn
