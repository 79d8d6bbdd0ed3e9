"""Builds libpsmdem.so (HIP, gfx950) in-tree with hipcc, and libpsmprobe.so,
the streaming-bandwidth measurement utility kept apart from the method.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
generation disabled.  The DEM and voxelisation sources are compiled without
floating-point contraction: their predicates decide integer results (cell
indices, contact flags, sample counts) and must round each operation.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpsmdem.so")
PROBE_LIB = os.path.join(PKG, "libpsmprobe.so")
ARCH = "gfx950"

SOURCES = [
    ("scan.hip", []),
    ("dem.hip", ["-ffp-contract=off"]),
    ("voxel.hip", ["-ffp-contract=off"]),
    ("lbm.hip", []),
    ("psmdem.hip", []),
    ("fields.hip", []),
    ("server.hip", []),
]
PROBE_SOURCES = [("probe.hip", [])]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, extra, verbose):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [_hipcc(), "-c"] + COMMON + extra + [os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, lib, verbose):
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + PROBE_SOURCES
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s[0], s[1], verbose), srcs))
    _link(objs[:len(SOURCES)], LIB, verbose)
    _link(objs[len(SOURCES):], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
