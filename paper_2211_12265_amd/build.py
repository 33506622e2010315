"""Compile the gfx950 HIP sources into the in-tree C-ABI library ``libdil.so``.

hipcc cross-compiles for gfx950 without a GPU present.  All device code is
built with packed FP32 instructions disabled (the kernels are integer-only;
the flag keeps the compiler from ever emitting v_pk_* FP32 forms).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdil.so")
SOURCES = ["api.hip", "server.hip"]
HEADERS = ["common.h", "keccak.h", "ntt.h", "poly.h", "sponge.h", "keccak_pair.h", "kernels.h", "ntt_ablation.h", "persist.h", "probe.h", "errwords.h", "batch_sched.h", "t0_ablation.h", "msg_words.h"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    """Always recompiles (the caller asked for a build)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-result", "-Wno-unused-value",
           "-I", os.path.join(os.path.dirname(HERE), "include"),
           "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libdil.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
