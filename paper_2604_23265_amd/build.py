"""Compile librte.so for gfx950 in-tree with hipcc.

Usage: python -m paper_2604_23265_amd.build   (or build() from Python).
Every call recompiles every source; objects go to _build/ at the repo root
and the shared library lands next to this file.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librte.so")
SOURCES = ["abi.cpp", "setup.cpp", "mgn1.cpp", "solver.cpp", "serve.cpp",
           "apply.hip", "mgnet.hip", "krylov.hip", "noalloc.hip",
           "tfps.hip", "tfps_setup.cpp", "atfps_setup.cpp", "block_jacobi.hip"]
ARCH = "gfx950"
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall",
         "-Wno-unused-function", "-Wno-unused-variable",
         # packed FP32 VALU ops are kept out of every code object
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _compile(hipcc, src, obj):
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [hipcc] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
    if r.returncode != 0:
        raise RuntimeError("compiling %s failed:\n%s" % (src, "\n".join(msgs)))
    return "\n".join(msgs)


def build(verbose=False, jobs=None):
    hipcc = _hipcc()
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_compile, hipcc, s, o) for s, o in zip(SOURCES, objs)]
        for f, s in zip(futs, SOURCES):
            msg = f.result()
            if verbose and msg.strip():
                print("[%s]\n%s" % (s, msg))
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("linking librte.so failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
