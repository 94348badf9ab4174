"""Build libhisq.so (HIP for gfx950) in-tree with hipcc.

dslash.hip is compiled once per (precision, Naik storage, epilogue) so the
objects build in parallel; everything links into paper_1411_4439_amd/libhisq.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhisq.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# packed FP32 instructions are switched off (see the build notes in the design document)
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wno-unused-command-line-argument"]

DSLASH_VARIANTS = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 0), (1, 1), (1, 2), (2, 0), (2, 1), (2, 2),
                   (3, 0), (3, 1), (3, 2), (4, 0), (4, 1), (4, 2)]
OTHER_SOURCES = ["blas.hip", "pack.hip", "force.hip", "dmu.hip", "dispatch.cpp", "api.cpp",
                 "noalloc.hip"]


def _jobs():
    out = []
    src = os.path.join(CSRC, "dslash.hip")
    for prec, epi in DSLASH_VARIANTS:
        obj = os.path.join(BUILD, "dslash_p%d_e%d.o" % (prec, epi))
        out.append((src, obj, ["-DHISQ_KPREC=%d" % prec, "-DHISQ_KEPI=%d" % epi]))
    for name in OTHER_SOURCES:
        out.append((os.path.join(CSRC, name), os.path.join(BUILD, os.path.splitext(name)[0] + ".o"), []))
    return out


def _compile(job):
    src, obj, defs = job
    cmd = [HIPCC] + FLAGS + defs + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(jobs: int | None = None, verbose: bool = False, defines=(), out: str | None = None,
          build_dir: str | None = None) -> str:
    """Compile every HIP source for gfx950 and link libhisq.so; returns its path.

    `defines` adds -D flags (tuning variants), `out` / `build_dir` redirect the
    library and its objects."""
    bdir = build_dir or BUILD
    os.makedirs(bdir, exist_ok=True)
    work = [(src, os.path.join(bdir, os.path.basename(obj)), list(d) + ["-D" + x for x in defines])
            for src, obj, d in _jobs()]
    n = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(_compile, work))
    lib = out or LIB
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(int(sys.argv[1]) if len(sys.argv) > 1 else None, verbose=True)
