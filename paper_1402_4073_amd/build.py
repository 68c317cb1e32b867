"""Build libtq.so (and the input generator library) for gfx950 with hipcc.

Objects are compiled in parallel and linked into an in-tree shared library
next to this file, so the built library travels with the source tree.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtq.so")
GEN_SRC = os.path.join(ROOT, "tqgen", "gen.hip")
GEN_LIB = os.path.join(ROOT, "tqgen", "libtqgen.so")
OBJDIR = os.path.join(ROOT, "_build")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
# Packed FP32 instructions stay disabled in every HIP build of this project.
COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]


def _compile(src: str, obj: str) -> None:
    cmd = [HIPCC, "-x", "hip", "-c", src, "-o", obj] + COMMON
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, r.stdout, r.stderr))


def _link(objs, out: str) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s%s" % (r.stdout, r.stderr))
    os.replace(tmp, out)


def build_lib(jobs: int = 8) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [os.path.join(OBJDIR, os.path.basename(s) + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda so: _compile(*so), zip(srcs, objs)))
    _link(objs, LIB)
    return LIB


def build_gen() -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    obj = os.path.join(OBJDIR, "gen.hip.o")
    _compile(GEN_SRC, obj)
    _link([obj], GEN_LIB)
    return GEN_LIB


def build_all(jobs: int = 8) -> None:
    build_lib(jobs)
    build_gen()


if __name__ == "__main__":
    build_all()
    print(LIB)
    print(GEN_LIB)
