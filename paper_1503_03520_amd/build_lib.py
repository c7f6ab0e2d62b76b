"""Compile the HIP sources of the l1ls library into libl1ls.so (gfx950).

Each .hip file is compiled to an object in parallel, then linked into a
shared library next to this file.  Used by ``__graft_entry__.build()``.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libl1ls.so")
ARCH = os.environ.get("L1LS_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off (hipcc warns on the host pass)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
SOURCES = ["generator.hip", "fista.hip", "operator.hip", "newton.hip", "mf.hip", "batch.hip", "path.hip", "serve.hip",
           "blocks.hip", "onchip.hip", "sgt.hip", "alloc.hip", "pcdm.hip", "tune.hip", "window.hip", "igen2.hip"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    return src, obj, res.returncode, err


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        results = list(ex.map(_compile, SOURCES))
    failed = False
    for src, obj, rc, err in results:
        if err.strip() and verbose:
            print(f"[{src}]\n{err}", file=sys.stderr)
        if rc != 0:
            failed = True
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [r[1] for r in results]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
