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
CSRC = os.path.join(HERE, "csrc")
# (source, extra flags): the stage-kernel instantiation unit is compiled once
# per (dimension, mixed precision, stage), so the instantiations build in
# parallel.
SOURCES = [(os.path.join(CSRC, f), []) for f in ("kernels.hip", "api.hip", "host_step.hip")] + [
    (os.path.join(CSRC, "kernels_inst.hip"), [f"-DHYD_DIM={d}", f"-DHYD_MIXED={m}", f"-DHYD_STAGE={st}"])
    for d in (2, 3) for m in (0, 1) for st in (1, 2)
]
# measurement helper (stream-copy bandwidth probe), kept out of libhydro.so
PROBE_LIB = os.path.join(HERE, "libhydro_probe.so")
PROBE_SOURCES = [(os.path.join(CSRC, "copy_probe.hip"), [])]
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


def _run(cmd: list, verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs.strip():
        print(msgs)


def _hipcc(out: str, sources: list, verbose: bool, extra: list | None) -> None:
    """Compile every (source, flags) pair to an object in parallel, then link
    the library."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    objs = [os.path.join(HERE, "_build", os.path.basename(src) + "".join(f.split("=")[-1] for f in fl) + ".o")
            for src, fl in sources]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    cmds = [["hipcc", *compile_flags, *(extra or []), *fl, "-c", "-o", o, src]
            for (src, fl), o in zip(sources, objs)]
    workers = max(1, min(len(cmds), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    _run(["hipcc", *FLAGS, *(extra or []), "-o", out + ".tmp", *objs], verbose)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False, extra: list | None = None) -> str:
    _hipcc(LIB, SOURCES, verbose, extra)
    _hipcc(PROBE_LIB, PROBE_SOURCES, verbose, extra)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
