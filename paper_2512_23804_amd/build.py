"""Build the HIP library libsgkkt.so for gfx950 in the package directory.

Every source under csrc/ is compiled to an object file in parallel (objects in
_build/ at the repository root), then linked into the shared library.

Usage: python paper_2512_23804_amd/build.py  (standalone: importing the package needs the built library)
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsgkkt.so")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
HIPCC = "/opt/rocm/bin/hipcc"

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-result",
]
NOISE = "is not a recognized feature for this target"


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _run(cmd):
    proc = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (proc.stdout + proc.stderr).splitlines() if ln.strip() and NOISE not in ln]
    return proc.returncode, "\n".join(msgs)


def build(verbose: bool = False) -> str:
    """Compile every source and link LIB (always recompiles).  Returns the path."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for src in sources():
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append((src, obj, [HIPCC, *FLAGS, "-c", src, "-o", obj]))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with cf.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: (j, _run(j[2])), jobs))
    failed = False
    for (src, _, cmd), (rc, msg) in results:
        if verbose:
            print(" ".join(cmd), flush=True)
        if rc != 0:
            failed = True
            sys.stderr.write(f"{os.path.basename(src)}:\n{msg}\n")
        elif msg and verbose:
            sys.stderr.write(msg + "\n")
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    rc, msg = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for _, o, _ in jobs], "-o", tmp])
    if rc != 0:
        sys.stderr.write(msg + "\n")
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
