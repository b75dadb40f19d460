"""Build libhydro.so (HIP for gfx950) in-tree with hipcc.

Packed-FP32 instructions are disabled for every HIP source (the host pass
warns that it does not know the feature; that is harmless).
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhydro.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "api.hip")]
# measurement helper (stream-copy bandwidth probe), kept out of libhydro.so
PROBE_LIB = os.path.join(HERE, "libhydro_probe.so")
PROBE_SOURCES = [os.path.join(HERE, "csrc", "copy_probe.hip")]
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", os.path.join(HERE, "csrc"),
]


def _hipcc(out: str, sources: list, verbose: bool, extra: list | None) -> None:
    cmd = ["hipcc", *FLAGS, *(extra or []), "-o", out + ".tmp", *sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs.strip():
        print(msgs)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False, extra: list | None = None) -> str:
    _hipcc(LIB, SOURCES, verbose, extra)
    _hipcc(PROBE_LIB, PROBE_SOURCES, verbose, extra)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
