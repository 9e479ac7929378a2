"""Build the HIP libraries (gfx950) in-tree with hipcc:

  libkmpp.so          every source in csrc/ but noalloc.hip
  libkmpp_noalloc.so  noalloc.hip (kmpp_seed_noalloc and its fixed device
                      array), linked to libkmpp.so; kept apart so that only
                      callers of that entry point load the code object with
                      the array
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkmpp.so")
LIB_NOALLOC = os.path.join(HERE, "libkmpp_noalloc.so")
NOALLOC_SRC = "noalloc.hip"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile_all(verbose):
    odir = os.path.join(HERE, "_build")
    os.makedirs(odir, exist_ok=True)
    procs, objs = [], {}
    for src in sources():
        obj = os.path.join(odir, os.path.basename(src) + ".o")
        cmd = ["hipcc", *FLAGS, "-c", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs[os.path.basename(src)] = obj
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        txt = out.decode(errors="replace")
        if pr.returncode != 0:
            failed.append((src, txt))
        elif verbose and txt.strip():
            print(txt)
    if failed:
        for src, txt in failed:
            sys.stderr.write(f"---- {src}\n{txt}\n")
        raise RuntimeError("hipcc failed for: " + ", ".join(os.path.basename(s) for s, _ in failed))
    return objs


def build(verbose: bool = False) -> str:
    objs = _compile_all(verbose)
    main = [o for name, o in sorted(objs.items()) if name != NOALLOC_SRC]
    tmp = LIB + ".tmp"
    subprocess.run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *main], check=True)
    os.replace(tmp, LIB)
    tmp = LIB_NOALLOC + ".tmp"
    subprocess.run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, objs[NOALLOC_SRC],
                    "-L" + HERE, "-l:libkmpp.so", "-Wl,-rpath,$ORIGIN"], check=True)
    os.replace(tmp, LIB_NOALLOC)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
