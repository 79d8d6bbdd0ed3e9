"""The C-ABI library loads and exports every entry point the header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psmdem.h")
LIB = os.path.join(ROOT, "paper_2512_04997_amd", "libpsmdem.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psmdem_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("psmdem_create", "psmdem_step", "psmdem_read_populations", "psmdem_read_particles",
              "psmdem_read_fields", "psmdem_destroy", "psmdem_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpsmdem.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.psmdem_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.psmdem_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpsmdem.so not built")
def test_invalid_description_is_rejected_without_a_device():
    from paper_2512_04997_amd import psmdem as P
    L = P.lib()
    d = P.make_desc(dict(n=(8, 8, 8), tau=0.4))
    h = ctypes.c_void_p()
    code = L.psmdem_create(ctypes.byref(d), None, None, P.ALLOC_FN(), P.FREE_FN(), None, ctypes.byref(h))
    assert code == P.E_INVALID
    assert b"tau" in L.psmdem_last_error()
    d = P.make_desc(dict(n=(8, 8, 8), tau=0.8, bc=["periodic", "noslip", "periodic", "periodic",
                                                    "periodic", "periodic"]))
    code = L.psmdem_create(ctypes.byref(d), None, None, P.ALLOC_FN(), P.FREE_FN(), None, ctypes.byref(h))
    assert code == P.E_INVALID
