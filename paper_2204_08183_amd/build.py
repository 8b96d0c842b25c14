"""Builds ``libsurvscan.so`` in-tree with hipcc for gfx950.

Usage: ``python -m paper_2204_08183_amd.build`` (or ``__graft_entry__.build()``).
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsurvscan.so")
SOURCES = ["adjoint.hip", "api.hip", "cv.hip", "fused.hip", "mixed.hip", "noalloc.hip", "prepare.hip", "sweep.hip", "tune.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions stay off in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose=False):
    """Compile every HIP source (in parallel, one object each) and link the
    shared library (always rebuilds)."""
    import concurrent.futures as cf
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    tag = "%d" % os.getpid()
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".%s.o" % tag))
        jobs.append(([hipcc()] + compile_flags + ["-I", INCLUDE, "-I", CSRC, "-c",
                                                   os.path.join(CSRC, src), "-o", obj], obj))
    workers = min(len(jobs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda j: _run(j[0], verbose), jobs))
    tmp = LIB + ".tmp" + tag
    _run([hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + [o for _, o in jobs] +
         ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    for _, o in jobs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
