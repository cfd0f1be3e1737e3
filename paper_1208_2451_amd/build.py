"""Build the gfx950 shared library libprrp.so in-tree with hipcc.

Usage: python -m paper_1208_2451_amd.build   (or __graft_entry__.build())
Compiles every source under csrc/ for gfx950 into objects (in parallel) and
links them into paper_1208_2451_amd/libprrp.so.  Always rebuilds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libprrp.so")
SOURCES = ["srrqr.hip", "gepp.hip", "gemm.hip", "misc.hip", "solve.hip", "block.hip", "api.cpp"]
# The strong-RRQR kernel keeps panel rows in registers; its fully unrolled
# back substitution must stay unrolled (a partial unroll makes register-array
# indices dynamic and spills them), which needs a higher pragma limit.
EXTRA = {"srrqr.hip": ["-mllvm", "-pragma-unroll-threshold=200000"]}


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return [
        "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-Wno-unused-result",
    ]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    objs = []

    def one(src):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc] + flags() + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc] + flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    workers = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    with open(LIB + ".srchash", "w") as fh:
        fh.write(source_hash() + "\n")
    return LIB


def source_hash() -> str:
    """Hash of every file the library is built from (and the flags)."""
    import hashlib
    h = hashlib.sha256(" ".join(flags()).encode())
    for d in (CSRC, os.path.join(ROOT, "include")):
        for name in sorted(os.listdir(d)):
            with open(os.path.join(d, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def is_current() -> bool:
    """True when libprrp.so was built from the sources as they are now."""
    try:
        with open(LIB + ".srchash") as fh:
            return os.path.exists(LIB) and fh.read().strip() == source_hash()
    except OSError:
        return False


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--if-stale":
        print("libprrp.so current" if is_current() else build(verbose=True))
    else:
        print(build(verbose=True))
