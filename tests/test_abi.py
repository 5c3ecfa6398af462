"""The C-ABI library loads on the CPU and exports every symbol its header declares.

No compute call is made here (there is no GPU in the CPU suite)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmg.h")
LIB = os.path.join(ROOT, "paper_2307_04886_amd", "libgmg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ["gmg_build_hierarchy", "gmg_solve", "gmg_free"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgmg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgmg.so not built")
def test_binding_symbol_list_matches_header():
    from paper_2307_04886_amd.binding import SYMBOLS, Options
    assert sorted(SYMBOLS) == declared_functions()
    # host-only calls that touch no device
    lib = ctypes.CDLL(LIB)
    o = Options()
    lib.gmg_default_options.argtypes = [ctypes.POINTER(Options)]
    assert lib.gmg_default_options(ctypes.byref(o)) == 0
    assert o.struct_size == ctypes.sizeof(Options)
    assert o.coarsening_ratio == 0.125 and o.min_coarse_points == 1000 and o.nu_pre == 2
    lib.gmg_status_string.restype = ctypes.c_char_p
    assert lib.gmg_status_string(-4) == b"matrix not symmetric positive definite"
    lib.gmg_free(None)


def test_oracle_and_library_share_no_code():
    """The oracle and the HIP path are independent: no include, import or source sharing."""
    osrc = open(os.path.join(ROOT, "oracle", "oracle.cpp")).read()
    assert "#include \"" not in osrc
    csrc = os.path.join(ROOT, "paper_2307_04886_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower()
    for f in ["binding.py", "__init__.py", "build.py"]:
        assert "oracle" not in open(os.path.join(ROOT, "paper_2307_04886_amd", f)).read()
