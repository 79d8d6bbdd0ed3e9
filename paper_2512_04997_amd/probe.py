"""ctypes binding of libpsmprobe.so (include/psmprobe.h): the device's
attainable streaming bandwidth, a measurement utility stated beside the
roofline figures and the calibration copy of the HBM traffic counters.  It is
not part of the method and the method's library does not contain it."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsmprobe.so")
KINDS = {"copy": 0, "read": 1, "write": 2}
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        import torch  # noqa: F401  (one HIP runtime per process: torch's)
        L = C.CDLL(LIB_PATH)
        L.psmprobe_stream.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_double)]
        L.psmprobe_stream.restype = C.c_int32
        _lib = L
    return _lib


def stream(kind, src, dst, nbytes, grid=16384, reps=10):
    """Average milliseconds of one plain streaming pass over device buffers
    src, dst (addresses)."""
    ms = C.c_double()
    rc = lib().psmprobe_stream(KINDS[kind], C.c_void_p(src), C.c_void_p(dst), int(nbytes), int(grid), int(reps),
                               C.byref(ms))
    if rc != 0:
        raise RuntimeError(f"psmprobe_stream failed ({rc})")
    return ms.value
