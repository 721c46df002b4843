"""Compile the HIP sources into the in-tree shared library ``libdemag.so`` for gfx950.

Usage: ``python -m paper_2308_08447_amd.build`` (also called by
``__graft_entry__.build()``).  Always recompiles.
"""

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdemag.so")
SOURCES = ["capi.hip", "stages_x.hip", "stages_y.hip", "stages_z.hip", "stages_xz.hip", "tensor.hip",
           "dynamics.hip",
           "serve.hip", "noalloc.hip"]
ARCH = os.environ.get("DEMAG_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # packed FP32 ops (v_pk_*_f32) stay disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit multiply-add contraction: the kernels spell out every fmaf, so
    # their rounding does not depend on unrolling (tile variants agree bitwise)
    "-ffp-contract=off",
    "-Wno-unused-command-line-argument",
]
FLAGS_OBJ = [f for f in FLAGS if f != "-shared"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}: {' '.join(cmd)}")


def build(verbose=False):
    """Compile every source to an object in parallel, then link; returns the library path."""
    from concurrent.futures import ThreadPoolExecutor
    inc = ["-I", os.path.join(HERE, "..", "include")]
    with tempfile.TemporaryDirectory(dir=HERE, prefix="_build") as tmpd:
        objs = [os.path.join(tmpd, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[hipcc()] + FLAGS_OBJ + inc + ["-c", os.path.join(CSRC, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        out = os.path.join(tmpd, "libdemag.so")
        _run([hipcc(), "-shared", f"--offload-arch={ARCH}"] + objs + ["-o", out], verbose)
        os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
