"""ctypes binding of libhydro.so (C ABI in include/hydro.h).

Argument marshalling only: every step of the hydro path runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.  The
library is loaded on first use; if it is missing the call raises (there is no
CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import json
import os
import re
import tempfile
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libhydro.so")
HEADER = os.path.join(ROOT, "include", "hydro.h")

OK, EINVAL, EDEVICE, ENOMEM, ENONPHYS, ESTATE = range(6)
FP64, FP32_FP64 = 0, 1
EINFELDT = 0x100  # OR into a precision: HLLC with Einfeldt wave-speed bounds
PVRS = 0x200  # OR into a precision: HLLC with pressure-based (PVRS) wave-speed bounds
CONSERVED = 0x400  # OR into a precision: PLM on the conserved variables
CHARACTERISTIC = 0x800  # OR into a precision: PLM on the characteristic variables
GAS_RADIATION = 0x1000  # with FP64 only: the gas + radiation equation of state
NBR, OUTFLOW, PERIODIC_SELF = 0, 1, 2
_NAMES = {0: "OK", 1: "EINVAL", 2: "EDEVICE", 3: "ENOMEM", 4: "ENONPHYS", 5: "ESTATE"}


class HydroError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what}: {_NAMES.get(code, code)}: {msg}")
        self.code = code


class BlockDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3),
        ("face_kind", C.c_int32 * 6),
        ("nbr", C.c_int32 * 6),
        ("reserved", C.c_int32),
        ("offset", C.c_int64),
        ("dx", C.c_double * 3),
    ]


def declared_functions() -> list:
    """Names of the functions include/hydro.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:hydro_status|const char\s*\*)\s*(hydro_\w+)\s*\(", text, re.M)))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH}; build it with python -c "
                               "'import __graft_entry__ as g; g.build()'")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        pp = C.POINTER(C.c_void_p)
        sig = {
            "hydro_mesh_create": [C.POINTER(BlockDesc), i32, i32, vp, i64, vp, pp],
            "hydro_mesh_destroy": [vp],
            "hydro_packet_create": [vp, C.POINTER(C.c_int32), i32, i32, pp],
            "hydro_packet_advance": [vp, dbl, dbl],
            "hydro_packet_reduce_dt": [vp, dbl, dbl, C.POINTER(C.c_double)],
            "hydro_packet_destroy": [vp],
            "hydro_batch_create": [C.POINTER(C.c_void_p), i32, pp],
            "hydro_batch_advance_plain": [vp, dbl, dbl],
            "hydro_batch_run": [vp, i32, dbl, dbl, C.POINTER(C.c_double)],
            "hydro_batch_run_timed": [vp, i32, dbl, dbl, C.POINTER(C.c_double), C.POINTER(C.c_double)],
            "hydro_batch_destroy": [vp],
            "hydro_batch_set_tiling": [vp, i32, i32, i32],
            "hydro_batch_set_launch": [vp, i32, i32],
            "hydro_batch_set_occupancy": [vp, i32],
            "hydro_batch_autotune": [vp, dbl, i32],
            "hydro_batch_get_config": [vp, C.POINTER(C.c_int32), i32, C.POINTER(C.c_int32)],
            "hydro_batch_time_kernels": [vp, i32, dbl, dbl, C.POINTER(C.c_double)],
            "hydro_stream_create": [C.POINTER(BlockDesc), i32, i32, vp, i64, C.POINTER(C.c_int32), i32, i32, i32, pp],
            "hydro_stream_run": [vp, i32, dbl, dbl, C.POINTER(C.c_double)],
            "hydro_stream_destroy": [vp],
            "hydro_stream_set_cpu_share": [vp, i32, i32],
            "hydro_stream_set_unit_bytes": [vp, i64],
            "hydro_step_static": [C.POINTER(BlockDesc), i32, i32, vp, i64, i32, dbl, dbl, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.hydro_last_error.restype = C.c_char_p
        L.hydro_last_error.argtypes = []
        _lib = L
    return _lib


_lib_hash = None


def library_hash() -> str:
    """First 16 hex digits of the SHA-256 of the library file."""
    global _lib_hash
    if _lib_hash is None:
        import hashlib

        with open(LIB_PATH, "rb") as f:
            _lib_hash = hashlib.sha256(f.read()).hexdigest()[:16]
    return _lib_hash


def _check(rc: int, what: str):
    if rc != OK:
        raise HydroError(rc, what, lib().hydro_last_error().decode())


def descs_from_mesh(mesh) -> "C.Array":
    """Block descriptors of an ``inputs.BlockMesh`` (or any object with the
    same n, dx, kind, nbr, offset arrays)."""
    nb = int(mesh.n.shape[0])
    arr = (BlockDesc * nb)()
    for b in range(nb):
        d = arr[b]
        for a in range(3):
            d.n[a] = int(mesh.n[b, a])
            d.dx[a] = float(mesh.dx[b, a])
        for f in range(6):
            d.face_kind[f] = int(mesh.kind[b, f])
            d.nbr[f] = int(mesh.nbr[b, f])
        d.reserved = 0
        d.offset = int(mesh.offset[b])
    return arr


def _stream_handle(stream) -> int:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return int(getattr(stream, "cuda_stream", stream))


class Mesh:
    """A mesh over a caller-owned FP64 device arena (a torch tensor or a raw
    device pointer with its length)."""

    def __init__(self, block_mesh, arena, arena_len: int | None = None, stream=None):
        self._keep = arena
        if hasattr(arena, "data_ptr"):
            import torch

            if arena.dtype != torch.float64 or not arena.is_cuda or not arena.is_contiguous():
                raise ValueError("arena must be a contiguous float64 CUDA tensor")
            ptr, n = arena.data_ptr(), arena.numel()
        else:
            ptr, n = int(arena), int(arena_len)
        self.block_mesh = block_mesh
        self.ndim = int(block_mesh.ndim)
        self._children = weakref.WeakSet()  # live packets and batches, closed before the mesh
        self._descs = descs_from_mesh(block_mesh)
        h = C.c_void_p()
        _check(lib().hydro_mesh_create(self._descs, len(self._descs), self.ndim, C.c_void_p(ptr), n,
                                       C.c_void_p(_stream_handle(stream)), C.byref(h)), "hydro_mesh_create")
        self.h = h

    def close(self):
        if self.h:
            kids = list(self._children)
            for c in kids:
                if isinstance(c, Batch):
                    c.close()
            for c in kids:
                if isinstance(c, Packet):
                    c.close()
            _check(lib().hydro_mesh_destroy(self.h), "hydro_mesh_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Packet:
    def __init__(self, mesh: Mesh, block_ids, precision: int = FP64):
        ids = np.ascontiguousarray(block_ids, dtype=np.int32)
        h = C.c_void_p()
        _check(lib().hydro_packet_create(mesh.h, ids.ctypes.data_as(C.POINTER(C.c_int32)), int(ids.size),
                                         int(precision), C.byref(h)), "hydro_packet_create")
        self.mesh, self.h, self.ids, self.precision = mesh, h, ids, precision
        mesh._children.add(self)

    def advance(self, dt: float, gamma: float):
        _check(lib().hydro_packet_advance(self.h, float(dt), float(gamma)), "hydro_packet_advance")

    def reduce_dt(self, gamma: float, cfl: float) -> float:
        out = C.c_double(0.0)
        _check(lib().hydro_packet_reduce_dt(self.h, float(gamma), float(cfl), C.byref(out)), "hydro_packet_reduce_dt")
        return out.value

    def close(self):
        if self.h:
            _check(lib().hydro_packet_destroy(self.h), "hydro_packet_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    def __init__(self, packets):
        self.packets = list(packets)
        arr = (C.c_void_p * len(self.packets))(*[p.h.value for p in self.packets])
        h = C.c_void_p()
        _check(lib().hydro_batch_create(arr, len(self.packets), C.byref(h)), "hydro_batch_create")
        self.h = h
        self.packets[0].mesh._children.add(self)

    def advance_plain(self, dt: float, gamma: float):
        _check(lib().hydro_batch_advance_plain(self.h, float(dt), float(gamma)), "hydro_batch_advance_plain")

    def run(self, nsteps: int, cfl: float, gamma: float) -> float:
        t = C.c_double(0.0)
        _check(lib().hydro_batch_run(self.h, int(nsteps), float(cfl), float(gamma), C.byref(t)), "hydro_batch_run")
        return t.value

    def run_timed(self, nsteps: int, cfl: float, gamma: float) -> tuple[float, list]:
        """run() with HIP events around every graph replay: (t, per-step device ms)."""
        t = C.c_double(0.0)
        ms = (C.c_double * max(int(nsteps), 1))()
        _check(lib().hydro_batch_run_timed(self.h, int(nsteps), float(cfl), float(gamma), C.byref(t), ms),
               "hydro_batch_run_timed")
        return t.value, list(ms)[: int(nsteps)]

    def time_kernels(self, nsteps: int, cfl: float, gamma: float) -> dict:
        """Eager launches with HIP events: mean stage-1 / stage-2 kernel ms and ms per step."""
        out = (C.c_double * 3)()
        _check(lib().hydro_batch_time_kernels(self.h, int(nsteps), float(cfl), float(gamma), out),
               "hydro_batch_time_kernels")
        return {"stage1_ms": out[0], "stage2_ms": out[1], "step_ms": out[2]}

    def set_tiling(self, edge: int, tile: int, zchunk: int = 0):
        _check(lib().hydro_batch_set_tiling(self.h, int(edge), int(tile), int(zchunk)), "hydro_batch_set_tiling")

    def set_launch(self, grid: int, xcd_remap: int = 1):
        _check(lib().hydro_batch_set_launch(self.h, int(grid), int(xcd_remap)), "hydro_batch_set_launch")

    def set_occupancy(self, waves: int):
        """Register budget of `waves` (2..4) waves per SIMD for the stage kernels (0 = their own)."""
        _check(lib().hydro_batch_set_occupancy(self.h, int(waves)), "hydro_batch_set_occupancy")

    def autotune(self, gamma: float, reps: int = 3, cache: str | None = None) -> dict:
        """Tune the batched launches in the library (tiling per block class,
        then grid and XCD renumbering; every candidate parity-checked) and
        return the chosen configuration.  cache: path of a JSON file of earlier
        results, keyed by device, precision code, dimension and block classes;
        a stored entry is applied without timing, a new result is added."""
        key = self.tuning_key()
        data = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
            if key in data:
                self.apply_config(data[key])
                return data[key]
        _check(lib().hydro_batch_autotune(self.h, float(gamma), int(reps)), "hydro_batch_autotune")
        cfg = self.config()
        if cache:
            data[key] = cfg
            d = os.path.dirname(os.path.abspath(cache))
            fd, tmp = tempfile.mkstemp(dir=d, suffix=".json")
            with os.fdopen(fd, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return cfg

    def tuning_key(self) -> str:
        """Library build | device | precision code | ndim | (class edge: cells,
        ...) of this batch.  The build is a hash of the loaded library file, so
        an entry stored by another build of the kernels is never applied
        without its parity check."""
        try:
            import torch

            dev = torch.cuda.get_device_name(torch.cuda.current_device())
        except Exception:
            dev = "gpu"
        classes = ",".join(f"{c['edge']}:{c['cells']}" for c in self.config()["classes"])
        return f"lib={library_hash()}|{dev}|prec={self.packets[0].precision}|ndim={self.packets[0].mesh.ndim}|{classes}"

    def apply_config(self, cfg: dict):
        """Apply a configuration as returned by config() / autotune()."""
        for c in cfg["classes"]:
            self.set_tiling(c["edge"], c["tile"], c["zchunk"])
        self.set_launch(cfg["grid"], cfg["xcd_remap"])
        self.set_occupancy(cfg.get("occupancy", 0))

    def config(self) -> dict:
        buf = (C.c_int32 * (3 + 4 * 16))()
        n = C.c_int32(0)
        _check(lib().hydro_batch_get_config(self.h, buf, 16, C.byref(n)), "hydro_batch_get_config")
        classes = [{"edge": buf[3 + 4 * k], "tile": buf[4 + 4 * k], "zchunk": buf[5 + 4 * k], "cells": buf[6 + 4 * k]}
                   for k in range(min(n.value, 16))]
        return {"grid": buf[0], "xcd_remap": buf[1], "occupancy": buf[2], "classes": classes}

    def close(self):
        if self.h:
            _check(lib().hydro_batch_destroy(self.h), "hydro_batch_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_static(block_mesh, arena, precision: int, dt: float, gamma: float, stream=None):
    """One SSP-RK2 step of every block of `block_mesh` on the device arena (a
    contiguous float64 CUDA tensor) through the allocation-free entry point:
    the library's fixed scratch array holds every temporary."""
    import torch

    if arena.dtype != torch.float64 or not arena.is_cuda or not arena.is_contiguous():
        raise ValueError("arena must be a contiguous float64 CUDA tensor")
    descs = descs_from_mesh(block_mesh)
    _check(lib().hydro_step_static(descs, len(descs), int(block_mesh.ndim), C.c_void_p(arena.data_ptr()),
                                   arena.numel(), int(precision), float(dt), float(gamma),
                                   C.c_void_p(_stream_handle(stream))), "hydro_step_static")


class HostStream:
    """Host-resident packets streamed through device staging slots.

    host_arena: a pinned CPU float64 torch tensor (or any object with
    data_ptr() and numel(); pageable memory also works, without overlap).
    packets: list of consecutive block-id ranges covering 0..nblocks-1."""

    def __init__(self, block_mesh, host_arena, packets, precision: int = FP64, nslots: int = 4):
        self._keep = host_arena
        self._descs = descs_from_mesh(block_mesh)
        starts = [int(p[0]) for p in packets] + [int(packets[-1][-1]) + 1]
        st = (C.c_int32 * len(starts))(*starts)
        h = C.c_void_p()
        _check(lib().hydro_stream_create(self._descs, len(self._descs), int(block_mesh.ndim),
                                         C.c_void_p(host_arena.data_ptr()), int(host_arena.numel()), st,
                                         len(packets), int(precision), int(nslots), C.byref(h)),
               "hydro_stream_create")
        self.h = h

    def run(self, nsteps: int, cfl: float, gamma: float) -> float:
        t = C.c_double(0.0)
        _check(lib().hydro_stream_run(self.h, int(nsteps), float(cfl), float(gamma), C.byref(t)), "hydro_stream_run")
        return t.value

    def set_cpu_share(self, cpu_packets: int, nthreads: int = 0):
        """Advance the last `cpu_packets` packets on the host cores (FP64 host
        kernel, `nthreads` threads, 0 = all) while the GPU streams the rest."""
        _check(lib().hydro_stream_set_cpu_share(self.h, int(cpu_packets), int(nthreads)),
               "hydro_stream_set_cpu_share")

    def set_unit_bytes(self, min_bytes: int):
        """Copy and advance consecutive GPU packets together, in units of at
        least `min_bytes` (0 = one packet per unit, the default)."""
        _check(lib().hydro_stream_set_unit_bytes(self.h, int(min_bytes)), "hydro_stream_set_unit_bytes")

    def close(self):
        if self.h:
            _check(lib().hydro_stream_destroy(self.h), "hydro_stream_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
