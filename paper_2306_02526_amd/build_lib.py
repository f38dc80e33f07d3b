"""Compile the HIP library (libhps.so) for gfx950 in-tree.

    python -m paper_2306_02526_amd.build_lib
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhps.so")
SOURCES = ["hps_solve_kernels.hip", "hps_leaf_kernels.hip", "hps_cx_kernels.hip", "hps_build_kernels.hip",
           "hps_api.hip", "hps_drivers.hip", "hps_batch.hip", "hps_serve.hip",
           "hps_noalloc.hip", "hps_tune.hip", "hps_compose.hip"]
OBJDIR = os.path.join(HERE, "_build")


def hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
         # hipcc forms packed FP32 instructions from plain float code; keep them off
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed: {what}")
    return r.stderr


def build(verbose=False, out=LIB):
    """Compile every source to an object (in parallel), then link libhps.so."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[hipcc()] + FLAGS + ["-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as ex:
        errs = list(ex.map(lambda c: _run(c, c[-3]), cmds))
    tmp = out + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], "link")
    if verbose:
        for e in errs:
            if e.strip():
                sys.stderr.write(e)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
