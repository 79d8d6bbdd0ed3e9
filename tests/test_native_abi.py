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
    d = P.make_desc(dict(n=(8, 8, 8), tau=0.8, collision="trt"))
    d.collision = 2
    code = L.psmdem_create(ctypes.byref(d), None, None, P.ALLOC_FN(), P.FREE_FN(), None, ctypes.byref(h))
    assert code == P.E_INVALID and b"collision" in L.psmdem_last_error()
    d = P.make_desc(dict(n=(8, 8, 8), tau=0.8, collision="trt", trt_magic=-0.1))
    code = L.psmdem_create(ctypes.byref(d), None, None, P.ALLOC_FN(), P.FREE_FN(), None, ctypes.byref(h))
    assert code == P.E_INVALID and b"trt_magic" in L.psmdem_last_error()


PROBE_HEADER = os.path.join(ROOT, "include", "psmprobe.h")
PROBE_LIB = os.path.join(ROOT, "paper_2512_04997_amd", "libpsmprobe.so")


@pytest.mark.skipif(not os.path.exists(PROBE_LIB), reason="libpsmprobe.so not built")
def test_stream_probe_is_its_own_library_and_rejects_bad_arguments_without_a_device():
    """The measurement probe lives in libpsmprobe.so, not in the method's ABI."""
    assert "stream" not in " ".join(declared_functions())
    text = re.sub(r"/\*.*?\*/", "", open(PROBE_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(psmprobe_[a-z_]+)\s*\(", text)))
    L = ctypes.CDLL(PROBE_LIB)
    assert names and all(hasattr(L, n) for n in names)
    assert not hasattr(ctypes.CDLL(LIB), "psmdem_stream_probe")
    from paper_2512_04997_amd import probe
    L = probe.lib()
    ms = ctypes.c_double()
    for kind, src, dst, nbytes, grid, reps, out in ((3, 16, 16, 1 << 20, 8, 1, True), (0, None, 16, 1 << 20, 8, 1, True),
                                                   (2, None, None, 1 << 20, 8, 1, True), (0, 16, 16, 8, 8, 1, True),
                                                   (0, 16, 16, 1 << 20, 0, 1, True), (0, 16, 16, 1 << 20, 8, 0, True),
                                                   (1, 16, 16, 1 << 20, 8, 1, False)):
        code = L.psmprobe_stream(kind, src, dst, nbytes, grid, reps, ctypes.byref(ms) if out else None)
        assert code == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpsmdem.so not built")
def test_state_calls_reject_bad_arguments_without_a_device():
    from paper_2512_04997_amd import psmdem as P
    L = P.lib()
    n = ctypes.c_size_t()
    assert L.psmdem_read_state(None, None, 0, ctypes.byref(n)) == P.E_INVALID
    assert L.psmdem_write_state(None, None, 0) == P.E_INVALID


def _r256(n):
    return (n + 255) // 256 * 256


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpsmdem.so not built")
def test_footprint_memory_model_without_a_device():
    """The admission memory model is the allocation plan of creation: the
    population array is 19 N storage bytes, the per-cell solid slots hold a
    B_k in the compute type and a double beta per kept solid."""
    from paper_2512_04997_amd import psmdem as P
    from paper_2512_04997_amd import workloads as W
    n = (70, 9, 6)
    N = 70 * 9 * 6
    plane = 2 * 3 * 2 * 1024          # tiles of 64 x 4 x 4 cells, 1024 slots each
    fp = {p: P.footprint(W.base_config(n, 0.7, precision=p)) for p in ("fp64", "fp32", "bf16", "fp16")}
    assert fp["bf16"] == fp["fp16"]
    assert fp["fp32"] - fp["bf16"] == _r256(19 * N * 4) - _r256(19 * N * 2)
    assert fp["fp64"] - fp["fp32"] == _r256(19 * N * 8) - _r256(19 * N * 4) + _r256(8 * plane * 2) - _r256(
        4 * plane * 2)
    ms3 = P.footprint(W.base_config(n, 0.7, precision="fp32", max_solids=3))
    assert ms3 - fp["fp32"] == _r256(4 * plane * 3) - _r256(4 * plane * 2) + _r256(8 * plane * 3) - _r256(
        8 * plane * 2)
    cfg, parts, _ = W.couette_suspension(n=48, nsph=20, radius=4.0)
    assert P.footprint(cfg, parts) > P.footprint(cfg, None)
    with pytest.raises(P.PsmdemError):
        P.footprint(W.base_config(n, 0.4))
