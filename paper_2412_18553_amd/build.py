"""Compile the HIP library libsie_triples.so for gfx950, in-tree.

Usage: python -m paper_2412_18553_amd.build   (or call build()).

Each translation unit of csrc/ (the host runtime and one per kernel family)
is compiled to an object in parallel, then linked into the shared library.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsie_triples.so")
# matrix-core peak microbenchmark (measurement only), a library of its own
PEAK_SRC = "mfma_peak.hip"
PEAK_LIB = os.path.join(HERE, "libsie_mfma_peak.so")

SOURCES = ["sie_triples.hip", "sie_mp2.hip", "tu_build_f64.hip", "tu_build_f64_l3.hip",
           "tu_bf16.hip", "tu_epilogue.hip", "tu_adj_f64.hip", "tu_adj_f32.hip",
           "tu_df.hip"]

# Packed-FP32 VALU instructions are disabled for all device code.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Always recompiles every translation unit; writes LIB atomically and
    returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1), 16)
    cmds = []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmds.append((obj, [cc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
                           os.path.join(CSRC, src), "-o", obj]))
    peak_tmp = PEAK_LIB + ".tmp"
    peak_cmd = (peak_tmp, [cc, *HIPCC_FLAGS, "-shared", os.path.join(CSRC, PEAK_SRC), "-o",
                           peak_tmp])
    pending = [peak_cmd] + list(cmds)
    running = []
    failed = []
    while pending or running:
        while pending and len(running) < jobs:
            obj, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((obj, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                      stderr=subprocess.STDOUT, text=True)))
        obj, cmd, proc = running.pop(0)
        out, _ = proc.communicate()
        if proc.returncode != 0:
            failed.append((cmd, out))
        elif verbose and out.strip():
            sys.stderr.write(out)
    if failed:
        for cmd, out in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + out)
        raise RuntimeError(f"hipcc failed for {len(failed)} translation unit(s)")
    os.replace(peak_tmp, PEAK_LIB)
    tmp = LIB + ".tmp"
    link = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in cmds], "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"link failed with status {res.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
