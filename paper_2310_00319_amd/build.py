"""Build libtvolap.so for gfx950 in-tree with hipcc.

The kernel file is compiled once per supported hop (64, 128, 256, 512) and
spectra storage type (f32, bf16, f16); all translation units compile in
parallel and are then linked into one shared library.

Usage: python -m paper_2310_00319_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtvolap.so")
HOPS = (64, 128, 256, 512)
# (source, extra flags, object name)
DTYPES = (0, 1, 2)   # f32, bf16, f16 storage
UNITS = [("tvolap_kernels.hip", [f"-DTVX_HOP={L}", f"-DTVX_DT={d}"], f"tvolap_kernels_L{L}_d{d}.o")
         for L in HOPS for d in DTYPES] + [
    ("tvolap_offline.hip", [], "tvolap_offline.o"),
    ("tvolap_compare.hip", [], "tvolap_compare.o"),
    ("tvolap_nup.hip", [], "tvolap_nup.o"),
    ("tvolap_dispatch.cpp", [], "tvolap_dispatch.o"),
    ("tvolap_capi.cpp", [], "tvolap_capi.o"),
]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep the compiler from emitting packed FP32 vector ALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + proc.stdout + proc.stderr)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    cmds = []
    objs = []
    for src, extra, obj in UNITS:
        o = os.path.join(OBJ, obj)
        objs.append(o)
        cmds.append([cc, *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", o])
    jobs = jobs or max(1, min(len(cmds), (os.cpu_count() or 2) - 1))
    with ThreadPoolExecutor(jobs) as ex:
        futs = [(c, ex.submit(_run, c, verbose)) for c in cmds]
    failed = [c for c, f in futs if f.exception() is not None]
    # the device compiler has aborted now and then under a full parallel
    # load; a unit that failed is compiled once more on its own, and a
    # second failure is reported
    for c in failed:
        print("retrying alone: " + os.path.basename(c[-1]), file=sys.stderr, flush=True)
        _run(c, verbose)
    tmp = LIB + ".tmp"
    _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
