"""Benchmark of the hydro packet step on one MI355X.

Workload (default): the large FP32-bulk run -- 32768 blocks of 16^3 cells on
the periodic unit cube (512^3 cells), Sedov deposit plus 1 % density noise,
gamma 1.4, CFL 0.4.  One "step" is one full SSP-RK2 step of the whole mesh.

Timed paths (same input, state reset between them):
  * batched mixed  -- all 512 packets of 64 blocks in one persistent launch per
                      RK stage, one HIP graph per step, dt on the device;
                      FP32 PLM + HLLC, FP64 recovery/accumulation/state.  This
                      is the headline `value`.
  * batched FP64   -- the same with every operation in FP64.
  * plain FP64     -- per-packet launches per stage (512 packets of 64
                      blocks) and a host reduce_dt per packet each step.

Metric: cell-updates/s (interior cells x steps / wall time, inputs resident in
HBM); the timed region (K steps) is repeated (5 times by default) and the
median is reported.  Roofline: HBM, 200 algorithmic bytes per cell-update
(FP64 state, five state passes: stage 1 reads Un and writes U1, stage 2 reads
U1 and Un and writes Un+1), 8.0 TB/s peak, over the step's device time (HIP
events on the mesh stream around every graph replay) and over the wall time;
per stage kernel over its own launch duration.  The practical ceiling comes
from a sweep of plain streaming kernels (copy, read, write; elements in
flight; workgroups per CU; 2 and 8 GiB buffers).  Errors vs the FP64 oracle
after K steps on the centred 512-block subset (the oracle runs the region
that holds its domain of dependence).  cpu_baseline: that oracle run (plain
FP64 C, OpenMP, all host cores) and a one-core run of the subset.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|smooth|uneven|sedov]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
import types

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s and % HBM roofline, FP32-batched vs FP64-plain, 1 MI355X"
HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_UPDATE = 200.0
HOST_UNIT_BYTES = 64 << 20  # transfer unit of the host-resident packet lines (0 = one packet per unit)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(name: str):
    from paper_2507_09337_amd import inputs as I

    if name == "large":
        return I.sedov_noise()
    if name == "smooth":
        return I.smooth3d()
    if name == "uneven":
        return I.uneven()
    if name == "sedov":
        return I.sedov3d()
    raise SystemExit(f"unknown workload {name}")


def sample_blocks(P, k=6):
    nb = P.mesh.nblocks
    rng = np.random.default_rng(0)
    ids = set(rng.choice(nb, size=min(k, nb), replace=False).tolist())
    sub = P.meta.get("subset")
    if sub is not None:  # include a block at the blast centre
        ids.add(int(sub[len(sub) // 2]))
    return sorted(ids)


def one_step_errors(P, arena, U0_dev, packets_fp64, packets_mixed):
    """Error of one step from the initial state vs the oracle on sampled blocks
    (used for workloads without a centred subset)."""
    import torch

    from oracle import oracle as O
    from paper_2507_09337_amd import hydro as H
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import l1_rho, rel_err

    ids = sample_blocks(P)
    dt = O.dt(P.mesh, P.U0, P.gamma, P.cfl)
    ref = O.step_subset(P.mesh, P.U0, dt, P.gamma, ids)
    out = {"kind": "one step from the initial state, sampled blocks", "sample_blocks": len(ids)}
    for name, pks in (("fp64", packets_fp64), ("mixed", packets_mixed)):
        arena.copy_(U0_dev)
        b = H.Batch(pks)
        b.run(1, P.cfl, P.gamma)
        b.close()
        torch.cuda.synchronize()
        U = np.empty_like(P.U0)
        for i in ids:  # copy back only the sampled blocks
            o, n = int(P.mesh.offset[i]), 5 * int(P.mesh.ncells[i])
            U[o:o + n] = arena[o:o + n].cpu().numpy()
        out[name] = {"max_rel_err": rel_err(P.mesh, U, ref, ids), "l1_rho_rel": l1_rho(P.mesh, U, ref, ids)}
    return out


def gather_blocks(P, arena, ids):
    """The listed blocks of a device arena, back to back (the layout of
    P.mesh.subset(ids))."""
    import torch

    torch.cuda.synchronize()
    return np.concatenate([arena[int(P.mesh.offset[i]):int(P.mesh.offset[i]) + 5 * int(P.mesh.ncells[i])].cpu().numpy()
                           for i in ids])


class RowCheck:
    """The error of a throughput row: one step from the initial state, the
    sampled blocks of the path's result against the oracle's step of a closed
    mesh around them (the sampled blocks themselves when they are
    self-contained, else the region that holds their one-step domain of
    dependence) with the path's own time step and the same method variant."""

    def __init__(self, P, ids, region=None):
        from oracle import oracle as O

        self.P, self.ids, self._O = P, [int(i) for i in ids], O
        region = self.ids if region is None else [int(i) for i in region]
        pos = {g: k for k, g in enumerate(region)}
        self.m = P.mesh.subset(np.asarray(region))
        self.U0 = P.mesh.gather(P.U0, np.asarray(region))
        self.local = [pos[i] for i in self.ids]
        self.ms = self.m.subset(np.asarray(self.local))

    def err(self, G, dt, speeds=0, recon=0, eos=0):
        """G: the sampled blocks after one step (gather_blocks layout); dt: the
        path's time step (its t after that step)."""
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from gpu_util import l1_rho, rel_err

        R = self.U0.copy()
        self._O.run(self.m, R, 1, self.P.cfl, self.P.gamma, dt, speeds, recon, eos)
        Rs = self.m.gather(R, np.asarray(self.local))
        return {"kind": f"one step from the initial state, {len(self.ids)} sampled blocks, vs the oracle with the "
                        "path's own dt", "dt": dt,
                "max_rel_err": rel_err(self.ms, G, Rs), "l1_rho_rel": l1_rho(self.ms, G, Rs)}


def class_sample(P, per_class=4):
    """Blocks of every block size, `per_class` of each (seeded)."""
    rng = np.random.default_rng(1)
    out = []
    for n in sorted(set(int(x) for x in P.mesh.n[:, 0])):
        cand = np.nonzero(P.mesh.n[:, 0] == n)[0]
        out += sorted(rng.choice(cand, size=min(per_class, cand.size), replace=False).tolist())
    return out


def region_around(P, steps):
    """Block ids of the centred subset grown by the domain of dependence of
    `steps` SSP-RK2 steps (two guard cells per stage, four cells per step),
    or None when that covers the whole mesh."""
    sub = P.meta.get("subset")
    if sub is None or P.mesh.grid is None:
        return None
    n = int(P.mesh.n[0, 0])
    margin = -(-4 * steps // n)
    nbx, nby, nbz = P.mesh.grid
    width = round(len(sub) ** (1 / 3))
    lo = [(d - width) // 2 - margin for d in (nbx, nby, nbz)]
    hi = [(d - width) // 2 + width + margin for d in (nbx, nby, nbz)]
    if any(l < 0 for l in lo) or any(h > d for h, d in zip(hi, (nbx, nby, nbz))):
        return None
    return np.asarray([(z * nby + y) * nbx + x for z in range(lo[2], hi[2]) for y in range(lo[1], hi[1])
                       for x in range(lo[0], hi[0])], dtype=np.int64)


def oracle_region_run(P, steps):
    """The oracle, as it stands, on the region around the centred subset for
    `steps` steps (dt from the region each step: the blast, which sets the
    global maximum rate, lies inside it).  Returns (region ids, state of the
    region, cpu timing dict)."""
    from oracle import oracle as O

    ids = region_around(P, steps)
    m = P.mesh.subset(ids)
    U = P.mesh.gather(P.U0, ids)
    t0 = time.perf_counter()
    dts, _ = O.run(m, U, steps, P.cfl, P.gamma)
    el = time.perf_counter() - t0
    cells = m.total_cells
    cpu = {"value": cells * steps / el, "unit": "cell-updates/s", "cores": O.num_threads(), "kind": "oracle",
           "host": host_cpu(), "sample": f"{len(ids)} blocks ({cells} cells) around the centred {len(P.meta['subset'])}-block subset "
                     f"of the same workload, {steps} steps, {el:.1f} s"}
    cpu["one_core"] = oracle_one_core(P)
    return ids, m, U, dts, cpu


def oracle_one_core(P, steps=2):
    """The oracle on one thread: the centred subset as its own mesh (links
    that leave it wrap), `steps` steps from the initial state."""
    from oracle import oracle as O

    ids = np.asarray(P.meta["subset"])
    m = P.mesh.subset(ids)
    U = P.mesh.gather(P.U0, ids)
    nthreads = O.num_threads()
    O.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.run(m, U, steps, P.cfl, P.gamma)
        el = time.perf_counter() - t0
    finally:
        O.set_num_threads(nthreads)
    return {"value": m.total_cells * steps / el, "unit": "cell-updates/s", "cores": 1,
            "sample": f"the centred {len(ids)}-block subset ({m.total_cells} cells) as its own mesh, {steps} steps, "
                      f"{el:.1f} s"}


def host_cpu() -> str:
    """The host CPU's model name (with family, model and stepping numbers) and
    the logical CPUs the machine has and this process may use."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" in line:
                    k, v = (x.strip() for x in line.split(":", 1))
                    if k in ("model name", "cpu family", "model", "stepping", "vendor_id") and k not in info:
                        info[k] = v
                if not line.strip() and info:
                    break
    except OSError:
        pass
    model = info.get("model name", "unknown CPU")
    ids = ", ".join(f"{k} {info[k]}" for k in ("vendor_id", "cpu family", "model", "stepping") if k in info)
    return (f"{model} ({ids}); {os.cpu_count()} logical CPUs on the host, "
            f"{len(os.sched_getaffinity(0))} available to this process")


def subset_errors(P, ids, m, Uref, U_gpu_sub):
    """Errors of GPU states (arrays of the subset blocks, subset layout) vs the
    oracle's region run on the centred subset: over every subset cell, and
    L1(rho) over only the cells whose density the oracle changed (the rest is
    gas at rest at uniform pressure, which the scheme leaves exactly as it
    was, so it dilutes the figure)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import l1_rho, rel_err

    pos = {int(b): k for k, b in enumerate(ids)}
    inner = [pos[int(b)] for b in P.meta["subset"]]
    ms = m.subset(inner)
    R = m.gather(Uref, inner)
    R0 = P.mesh.gather(P.U0, P.meta["subset"])
    nb = len(inner)
    rho_ref = R.reshape(nb, 5, -1)[:, 0]
    rho_gpu = U_gpu_sub.reshape(nb, 5, -1)[:, 0]
    changed = rho_ref != R0.reshape(nb, 5, -1)[:, 0]
    l1c = float(np.abs(rho_gpu - rho_ref)[changed].sum() / np.abs(rho_ref)[changed].sum()) if changed.any() else 0.0
    return {"max_rel_err": rel_err(ms, U_gpu_sub, R), "l1_rho_rel": l1_rho(ms, U_gpu_sub, R),
            "l1_rho_rel_changed_cells": l1c, "changed_cells": int(changed.sum()), "cells": int(changed.size)}


PROBE_MODES = {0: "copy", 1: "copy_nt", 2: "read", 3: "write"}


def copy_bandwidth(sizes=(1 << 28, 1 << 30), reps=5):
    """HBM bandwidth of the project's plain streaming kernels: copy (plain
    and nontemporal), read-only and write-only, each with 1, 2, 4 or 8
    16-byte elements per thread in flight and 2 to 32 workgroups per CU, on
    buffers of 2 GiB and 8 GiB (far larger than the 256 MB last-level cache).
    Bytes moved (read + written) / time.  Returns the best of each kind with
    its configuration; `gbs` is the best copy, the ceiling the stage kernels
    (which read and write) are compared with."""
    import ctypes as C

    import torch

    lib = C.CDLL(os.path.join(ROOT, "paper_2507_09337_amd", "libhydro_probe.so"))
    lib.stream_probe.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int,
                                 C.POINTER(C.c_double)]
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    best = {}
    table = []
    for n in sizes:
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for mode, kind in PROBE_MODES.items():
            for elems in (1, 2, 4, 8):
                for wg in (2, 4, 8, 16, 32):
                    ms = C.c_double(0.0)
                    rc = lib.stream_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n, stream, reps,
                                          mode, elems, wg, C.byref(ms))
                    if rc != 0:
                        raise RuntimeError(f"stream_probe failed with {rc}")
                    nbytes = 8 * n * (2 if mode in (0, 1) else 1)
                    gbs = nbytes / (ms.value * 1e-3) / 1e9
                    rec = {"kind": kind, "bytes": 8 * n, "elems_in_flight": elems, "wg_per_cu": wg, "gbs": gbs}
                    table.append(rec)
                    if kind not in best or gbs > best[kind]["gbs"]:
                        best[kind] = rec
            if mode in (0, 1):  # the copies must be exact
                assert torch.equal(src, dst), f"copy probe mode {mode} wrote wrong data"
        del src, dst
        torch.cuda.empty_cache()
    copy = max((best["copy"], best["copy_nt"]), key=lambda r: r["gbs"])
    return {"gbs": copy["gbs"], "best_copy": copy, "best_read": best["read"], "best_write": best["write"],
            "configs": len(table), "table": table}


KERNEL_SOURCES = [os.path.join(ROOT, "paper_2507_09337_amd", "csrc", f)
                  for f in ("stage_kernels.h", "kernels_inst.hip", "hydro_internal.h")]


def kernel_source_sha() -> str:
    """SHA-256 over the stage kernels' source files (their device code)."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel_names):
    """HBM bytes per step of the given stage kernels from the committed
    rocprofv3 counter summary, or None when the summary is missing or was
    taken on a different version of the kernel source."""
    path = os.path.join(ROOT, "profiles", "stage_kernels_large.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("TRAFFIC_JSON "):
            rec = json.loads(line[len("TRAFFIC_JSON "):])
    if not rec or rec.get("kernels_sha256") != kernel_source_sha():
        return None
    total = 0.0
    for k in kernel_names:
        t = rec["per_launch"].get(k)
        if t is None:
            return None
        total += t["fetch_bytes"] + t["write_bytes"]
    return total


def measured_valu(kernel_names):
    """VALU instructions per cell of the given kernels from the committed
    counter summary, or None when it is missing or was taken on a different
    version of the kernel source."""
    path = os.path.join(ROOT, "profiles", "stage_kernels_valu_large.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if kernel_source_sha() not in text:
        return None
    per = {}
    for line in text.splitlines():
        if line.startswith("| `"):
            cols = [c.strip() for c in line.strip("|").split("|")]
            per[cols[0].strip("`")] = cols[2]
    try:
        return sum(float(per[k]) for k in kernel_names)
    except (KeyError, ValueError):
        return None


def _csv_rows(directory, suffix):
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    return rows


def summarize_profiles(args):
    """Markdown summary of three rocprofv3 runs of this benchmark on the
    large workload (kernel trace with --stats; PMC FETCH_SIZE; PMC
    WRITE_SIZE), written to stdout.  The counters are scaled by what they
    read for the plain copy kernel of the streaming probe (known bytes).  A
    TRAFFIC_JSON line at the end feeds the benchmark's roofline.traffic."""
    cells = 32768 * 4096
    stats = _csv_rows(args.kt, "kernel_stats.csv")
    lines = ["# Stage kernels on the large workload (32768 blocks of 16^3 = 134217728 cells)", "",
             "Workload: Sedov deposit + 1 % density noise, periodic, gamma 1.4, CFL 0.4; batched launches (one "
             "per RK stage over all 512 packets).", "", "## Commands", "", "```", "cd /tmp && export TMPDIR=/tmp"]
    lines += [c for c in args.cmd] + ["```", "", "## Kernel trace summary (rocprofv3 --stats)", "",
                                      "| Kernel | Calls | Average ns | Min ns | Max ns | % |", "|---|---|---|---|---|---|"]
    avg = {}
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        avg[r["Name"]] = float(r["AverageNs"])
        lines.append(f"| `{r['Name']}` | {r['Calls']} | {float(r['AverageNs']):.0f} | {float(r['MinNs']):.0f} | "
                     f"{float(r['MaxNs']):.0f} | {float(r['Percentage']):.3g} |")
    s1 = "void hyd::k_stage<3, true, 1, 1, 0, 0, 0, 0>(hyd::StageArgs)"
    s2 = "void hyd::k_stage<3, true, 2, 1, 0, 0, 0, 0>(hyd::StageArgs)"
    # the headline kernels also run per packet in the host-resident paths: take the dispatches over the
    # large workload's whole work list (the largest grid)
    trace = _csv_rows(args.kt, "kernel_trace.csv")
    big = {}
    for name in (s1, s2):
        rows = [r for r in trace if r["Kernel_Name"] == name]
        if rows:
            g = max(int(r["Grid_Size_X"]) for r in rows)
            d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in rows if int(r["Grid_Size_X"]) == g]
            big[name] = (float(np.mean(d)), len(d), g)
    if s1 in big and s2 in big:
        t = (big[s1][0] + big[s2][0]) * 1e-9
        lines += ["", f"Headline kernels (mixed, Davis, primitive PLM), their {big[s1][1]} + {big[s2][1]} dispatches over "
                      f"the large workload's work list (grid {big[s1][2] // 256} workgroups): stage 1 "
                      f"{big[s1][0] / 1e6:.3f} ms + stage 2 {big[s2][0] / 1e6:.3f} ms = {t * 1e3:.3f} ms per step; "
                      f"200 B x {cells} cells / that = {200 * cells / t / 1e9:.0f} GB/s = "
                      f"{200 * cells / t / 1e9 / HBM_PEAK_GBS:.3f} of 8 TB/s; stage 2 alone "
                      f"{120 * cells / (big[s2][0] * 1e-9) / 1e9 / HBM_PEAK_GBS:.3f} (120 B)."]
    per = {}
    for kind, d in (("fetch", args.fetch), ("write", args.write)):
        for r in _csv_rows(d, "counter_collection.csv"):
            name = r.get("Kernel_Name", "")
            per.setdefault(name, {}).setdefault(kind, []).append(float(r["Counter_Value"]))
    calib = "k_copy_e<1, false>"
    cname = next((n for n in per if calib in n), None)
    if cname and per:
        # the probe's copies of 2 GiB buffers (2 GiB read and 2 GiB written per launch) are the smallest of
        # its dispatches of this kernel (the 8 GiB ones read four times as much)
        copy_bytes = 8 * (1 << 28)

        def small(vals):
            lo = min(vals)
            return float(np.median([v for v in vals if v <= 1.1 * lo]))

        fkib = small(per[cname]["fetch"])
        wkib = small(per[cname]["write"])
        ff, wf = copy_bytes / (fkib * 1024), copy_bytes / (wkib * 1024)
        lines += ["", "## HBM traffic (PMC FETCH_SIZE, WRITE_SIZE)", "",
                  f"Calibration with the plain copy kernel `{cname}` moving {copy_bytes} B each way (2 GiB buffers): "
                  f"FETCH_SIZE reads {fkib:.1f} KiB, WRITE_SIZE {wkib:.1f} KiB per dispatch, so bytes = KiB x 1024 x "
                  f"{ff:.4f} (fetch) and x {wf:.4f} (write).", "",
                  "| Kernel | Fetch B/launch | Write B/launch | Fetch B/cell | Write B/cell | Algorithmic B/cell |",
                  "|---|---|---|---|---|---|"]
        rec = {"kernels_sha256": kernel_source_sha(), "cells": cells, "fetch_factor": ff, "write_factor": wf,
               "per_launch": {}}
        for name, v in per.items():
            if "k_stage<3" not in name or "fetch" not in v or "write" not in v:
                continue
            fb = float(np.mean(v["fetch"])) * 1024 * ff
            wb = float(np.mean(v["write"])) * 1024 * wf
            targs = name[name.index("<") + 1:name.index(">")].split(", ")
            alg = 80 if targs[2] == "1" else 120  # k_stage<DIM, MIXED, STAGE, ...>
            rec["per_launch"][name] = {"fetch_bytes": fb, "write_bytes": wb}
            lines.append(f"| `{name}` | {fb:.4g} | {wb:.4g} | {fb / cells:.1f} | {wb / cells:.1f} | {alg} |")
        lines += ["", f"Kernel sources (stage_kernels.h, kernels_inst.hip, hydro_internal.h) sha256 at measurement: "
                      f"`{rec['kernels_sha256']}`", "", "TRAFFIC_JSON " + json.dumps(rec)]
    if args.bench_line:
        lines += ["", "## The benchmark line of the kernel-trace run", "", "```", open(args.bench_line).read().strip(),
                  "```"]
    print("\n".join(lines))


def host_packets_bench(args):
    """Uneven workload (self-periodic blocks, closed packets) with the state in
    pinned host memory: every step copies each packet in and out."""
    import torch

    from paper_2507_09337_amd import hydro as H
    from paper_2507_09337_amd import inputs as I

    P = I.uneven()
    cells = P.mesh.total_cells
    out = {}
    for prec, name in ((H.FP32_FP64, "mixed"), (H.FP64, "fp64")):
        for nslots, unit in ((1, 0), (3, 0), (4, 0), (3, HOST_UNIT_BYTES), (4, HOST_UNIT_BYTES)):
            host = torch.from_numpy(P.U0.copy()).pin_memory()
            hs = H.HostStream(P.mesh, host, P.packets, prec, nslots)
            hs.set_unit_bytes(unit)
            hs.run(args.warmup, P.cfl, P.gamma)
            ts = time.perf_counter()
            hs.run(args.steps, P.cfl, P.gamma)
            el = time.perf_counter() - ts
            hs.close()
            key = f"{name}_slots{nslots}" + (f"_unit{unit >> 20}MiB" if unit else "")
            out[key] = {"cell_updates_per_s": cells * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                        "pcie_gbs": 80.0 * cells * args.steps / el / 1e9, "unit_bytes": unit}
            log(name, nslots, unit, json.dumps(out[key]))
    # CPU/GPU split (the paper's blocks-per-cycle split between host cores and GPU): the last k packets on
    # the host cores, the rest streamed through four GPU slots in transfer units of HOST_UNIT_BYTES
    split = {}
    nthreads = len(os.sched_getaffinity(0))
    for prec, name in ((H.FP32_FP64, "mixed"), (H.FP64, "fp64")):
        for k in (0, 4, 8, 16, 24, 32, 48):
            host = torch.from_numpy(P.U0.copy()).pin_memory()
            hs = H.HostStream(P.mesh, host, P.packets, prec, 4)
            hs.set_unit_bytes(HOST_UNIT_BYTES)
            hs.set_cpu_share(k, nthreads)
            hs.run(args.warmup, P.cfl, P.gamma)
            ts = time.perf_counter()
            hs.run(args.steps, P.cfl, P.gamma)
            el = time.perf_counter() - ts
            hs.close()
            cpu_cells = int(sum(P.mesh.ncells[np.asarray(p)].sum() for p in P.packets[len(P.packets) - k:])) if k else 0
            split[f"{name}_cpu{k}"] = {"cpu_packets": k, "cpu_cells": cpu_cells, "cpu_threads": nthreads,
                                       "cell_updates_per_s": cells * args.steps / el, "ms_per_step": 1e3 * el / args.steps}
            log(name, "split", k, json.dumps(split[f"{name}_cpu{k}"]))
    best = max((v for k, v in out.items() if k.startswith("mixed")), key=lambda v: v["cell_updates_per_s"])
    print(json.dumps({"metric": "cell-updates/s, host-resident packets (PCIe-inclusive), uneven workload, 1 MI355X",
                      "value": best["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms_per_step"],
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32 (PLM+HLLC) / f64 (state, recovery, update, dt)", "data": "synthetic (seeded)",
                      "config": {"workload": f"uneven: {P.mesh.nblocks} self-periodic blocks, {cells} cells, "
                                             f"{len(P.packets)} packets, state in pinned host memory"},
                      "paths": out, "cpu_gpu_split": split}), flush=True)


def fused_class_study(P, steps, warmup, check=True):
    """The communication-avoiding fused step on the self-periodic 8^3 blocks
    of the uneven workload: those blocks as their own mesh, advanced by the
    two stage launches (200 algorithmic B per cell-update: U1 written and read
    back) and by the fused kernel (80 B: the block stays on chip between the
    stages), in both precisions; and the whole workload with the 8^3 class
    fused.  Device time per step from HIP events around the graph replays."""
    import torch

    from paper_2507_09337_amd import hydro as H

    ids = np.nonzero(P.mesh.n[:, 0] == 8)[0]
    m = P.mesh.subset(ids)
    U0h = P.mesh.gather(P.U0, ids)
    U0 = torch.from_numpy(U0h).cuda()
    cells = m.total_cells
    sub = types.SimpleNamespace(mesh=m, U0=U0h, gamma=P.gamma, cfl=P.cfl)
    chk = RowCheck(sub, np.random.default_rng(2).choice(m.nblocks, size=min(8, m.nblocks), replace=False)) \
        if check else None
    out = {"blocks": int(ids.size), "cells": int(cells)}
    for prec, pname in ((H.FP32_FP64, "mixed"), (H.FP64, "fp64")):
        for fused in (False, True):
            arena = U0.clone()
            mesh = H.Mesh(m, arena)
            b = H.Batch([H.Packet(mesh, range(m.nblocks), prec)])
            if fused:
                b.set_tiling(8, 5)
            b.run(warmup, P.cfl, P.gamma)
            _, ms = b.run_timed(steps, P.cfl, P.gamma)
            dev = float(np.median(ms))
            alg = 80.0 if fused else 200.0
            out[f"{pname}_{'fused' if fused else 'two_launch'}"] = {
                "device_ms_per_step": dev, "cell_updates_per_s": cells / (dev * 1e-3),
                "algorithmic_bytes_per_cell_update": alg,
                "achieved_gbs": alg * cells / (dev * 1e-3) / 1e9,
                "frac_of_hbm": alg * cells / (dev * 1e-3) / 1e9 / HBM_PEAK_GBS,
                "gbs_at_200B": 200.0 * cells / (dev * 1e-3) / 1e9}
            if chk is not None:
                arena.copy_(U0)
                b2 = H.Batch([H.Packet(mesh, range(m.nblocks), prec)])
                if fused:
                    b2.set_tiling(8, 5)
                dt = b2.run(1, P.cfl, P.gamma)
                b2.close()
                out[f"{pname}_{'fused' if fused else 'two_launch'}"]["errors_vs_oracle"] = \
                    chk.err(gather_blocks(sub, arena, chk.ids), dt)
            mesh.close()
            log("fused study", pname, fused, json.dumps(out[f"{pname}_{'fused' if fused else 'two_launch'}"]))
    return out


def secondary_paths(steps, warmup, check=True):
    """The uneven workload (6000 self-periodic blocks of 8^3/16^3/32^3, 147
    packets): the batched mixed and FP64 paths with the default tiling, the
    fused step of its 8^3 class, and its state held in pinned host memory
    (four GPU staging slots; GPU only, and with the last 8 packets on the host
    cores).  Each row carries its error after one step from the initial state
    on sampled blocks of every size.  Reported beside the headline, never as
    `value`."""
    import torch

    from paper_2507_09337_amd import hydro as H
    from paper_2507_09337_amd import inputs as I

    t0 = time.perf_counter()
    P = I.uneven()
    cells = P.mesh.total_cells
    log(f"secondary workload {P.name}: {P.mesh.nblocks} blocks, {cells} cells, built in {time.perf_counter() - t0:.1f} s")
    out = {"workload": f"uneven: {P.mesh.nblocks} self-periodic blocks of 8^3/16^3/32^3, {cells} cells, "
                       f"{len(P.packets)} packets, gamma {P.gamma}, CFL {P.cfl}", "steps": steps}
    chk = RowCheck(P, class_sample(P)) if check else None
    U0 = torch.from_numpy(P.U0).cuda()
    arena = U0.clone()
    mesh = H.Mesh(P.mesh, arena)
    for prec, name in ((H.FP32_FP64, "batched_mixed"), (H.FP64, "batched_fp64")):
        arena.copy_(U0)
        b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
        b.run(warmup, P.cfl, P.gamma)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, ms = b.run_timed(steps, P.cfl, P.gamma)
        el = time.perf_counter() - ts
        b.close()
        out[name] = {"cell_updates_per_s": cells * steps / el, "ms_per_step": 1e3 * el / steps,
                     "device_ms_per_step": float(np.mean(ms))}
        if chk is not None:
            arena.copy_(U0)
            b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
            dt = b.run(1, P.cfl, P.gamma)
            b.close()
            out[name]["errors_vs_oracle"] = chk.err(gather_blocks(P, arena, chk.ids), dt)
        log("secondary", name, json.dumps(out[name]))
    mesh.close()
    del arena, U0
    torch.cuda.empty_cache()
    out["fused_8cube_class"] = fused_class_study(P, steps, warmup, check)
    nthreads = len(os.sched_getaffinity(0))
    for k in (0, 8):
        host = torch.from_numpy(P.U0.copy()).pin_memory()
        hs = H.HostStream(P.mesh, host, P.packets, H.FP32_FP64, 4)
        hs.set_unit_bytes(HOST_UNIT_BYTES)
        hs.set_cpu_share(k, nthreads)
        hs.run(1, P.cfl, P.gamma)
        ts = time.perf_counter()
        hs.run(steps, P.cfl, P.gamma)
        el = time.perf_counter() - ts
        hs.close()
        key = "host_resident_mixed" + (f"_cpu{k}" if k else "")
        out[key] = {"cell_updates_per_s": cells * steps / el, "ms_per_step": 1e3 * el / steps,
                    "pcie_gbs": 80.0 * cells * steps / el / 1e9, "cpu_packets": k, "cpu_threads": nthreads,
                    "unit_bytes": HOST_UNIT_BYTES,
                    "note": "PCIe-inclusive (state in pinned host memory); four staging slots; consecutive GPU "
                            "packets copied and advanced in transfer units of at least unit_bytes"}
        if chk is not None:  # one step from the initial state through the same stream set-up
            host = torch.from_numpy(P.U0.copy()).pin_memory()
            hs = H.HostStream(P.mesh, host, P.packets, H.FP32_FP64, 4)
            hs.set_unit_bytes(HOST_UNIT_BYTES)
            hs.set_cpu_share(k, nthreads)
            dt = hs.run(1, P.cfl, P.gamma)
            hs.close()
            Uh = host.numpy()
            G = np.concatenate([Uh[int(P.mesh.offset[i]):int(P.mesh.offset[i]) + 5 * int(P.mesh.ncells[i])]
                                for i in chk.ids])
            out[key]["errors_vs_oracle"] = chk.err(G, dt)
        log("secondary", key, json.dumps(out[key]))
    return out


def summarize_valu(args):
    """Markdown summary of a rocprofv3 run with the VALU counters
    (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_WAVES, GRBM_GUI_ACTIVE) and,
    optionally, one with the L2 counters (TCC_HIT_sum, TCC_MISS_sum), per
    stage kernel of the large workload, written to stdout."""
    cells = 32768 * 4096
    vals = {}
    for d in (args.valu, args.tcc):
        if not d:
            continue
        for r in _csv_rows(d, "counter_collection.csv"):
            name = r.get("Kernel_Name", "")
            if "k_stage<3" not in name and "k_fused" not in name:
                continue
            disp = r.get("Dispatch_Id", "")
            vals.setdefault(name, {}).setdefault(r["Counter_Name"], {}).setdefault(disp, 0.0)
            vals[name][r["Counter_Name"]][disp] += float(r["Counter_Value"])
    lines = ["# VALU work and L2 hits of the stage kernels on the large workload (32768 blocks of 16^3 = "
             "134217728 cells)", "",
             "Workload: Sedov deposit + 1 % density noise, periodic, gamma 1.4, CFL 0.4; batched launches; every "
             "method variant the benchmark times.", "", "## Commands", "", "```", "cd /tmp && export TMPDIR=/tmp"]
    lines += list(args.cmd) + ["```", "",
                               "Per dispatch, averaged over the dispatches of each kernel: VALU instructions per cell = "
                               "SQ_INSTS_VALU (wave instructions, summed over all shader engines) x 64 lanes / cells; "
                               "VALU busy = 100 x SQ_ACTIVE_INST_VALU / 256 CUs / (GRBM_GUI_ACTIVE / 8 XCDs); L2 hit "
                               "rate = TCC_HIT / (TCC_HIT + TCC_MISS).", "",
                               "| Kernel | Dispatches | VALU instr / cell | VALU busy % | L2 hit % |",
                               "|---|---|---|---|---|"]

    def mean(name, counter):
        d = vals[name].get(counter)
        return (float(np.mean(list(d.values()))), len(d)) if d else (None, 0)

    for name in sorted(vals):
        iv, n = mean(name, "SQ_INSTS_VALU")
        av, _ = mean(name, "SQ_ACTIVE_INST_VALU")
        gg, _ = mean(name, "GRBM_GUI_ACTIVE")
        hit, _ = mean(name, "TCC_HIT_sum")
        mis, _ = mean(name, "TCC_MISS_sum")
        per = f"{iv * 64 / cells:.0f}" if iv is not None else "-"
        busy = f"{100 * av / 256 / (gg / 8):.1f}" if av is not None and gg else "-"
        hr = f"{100 * hit / (hit + mis):.1f}" if hit is not None and mis is not None and hit + mis > 0 else "-"
        lines.append(f"| `{name}` | {n} | {per} | {busy} | {hr} |")
    lines += ["", f"Kernel sources (stage_kernels.h, kernels_inst.hip, hydro_internal.h) sha256 at measurement: "
                  f"`{kernel_source_sha()}`"]
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=5, help="repetitions of the timed region (median reported)")
    ap.add_argument("--no-probe", action="store_true", help="skip the HBM streaming-kernel sweep")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the uneven-workload paths (batched, fused 8^3 class, host-resident, CPU/GPU split)")
    ap.add_argument("--workload", default="large")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-packet FP64 path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tune", action="store_true", help="autotune the batched launches first")
    ap.add_argument("--no-check", action="store_true", help="skip the one-step error check against the oracle")
    ap.add_argument("--host-packets", action="store_true",
                    help="instead: host-resident packets of the uneven workload streamed through device slots "
                         "(PCIe-inclusive rate; prints its own line)")
    ap.add_argument("--summarize-profiles", action="store_true",
                    help="instead: write the markdown summary of rocprofv3 runs (--kt, --fetch, --write dirs)")
    ap.add_argument("--kt", help="rocprofv3 --kernel-trace --stats output directory")
    ap.add_argument("--fetch", help="rocprofv3 --pmc FETCH_SIZE output directory")
    ap.add_argument("--write", help="rocprofv3 --pmc WRITE_SIZE output directory")
    ap.add_argument("--cmd", action="append", default=[], help="command line to list in the summary")
    ap.add_argument("--bench-line", help="file holding the JSON line of the kernel-trace run")
    ap.add_argument("--summarize-valu", action="store_true",
                    help="instead: write the markdown summary of the VALU (--valu dir) and L2 (--tcc dir) counters")
    ap.add_argument("--valu", help="rocprofv3 --pmc SQ_INSTS_VALU ... output directory")
    ap.add_argument("--tcc", help="rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum output directory")
    args = ap.parse_args()
    if args.summarize_profiles:
        return summarize_profiles(args)
    if args.summarize_valu:
        return summarize_valu(args)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from oracle import oracle as O
    from paper_2507_09337_amd import hydro as H

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.host_packets:
        return host_packets_bench(args)
    probe = None if args.no_probe else copy_bandwidth()
    if probe:
        log("HBM streaming probe:", json.dumps({k: v for k, v in probe.items() if k != "table"}))
    t0 = time.perf_counter()
    P = make_problem(args.workload)
    cells = P.mesh.total_cells
    log(f"workload {P.name}: {P.mesh.nblocks} blocks, {cells} cells, built in {time.perf_counter() - t0:.1f} s")

    U0_dev = torch.from_numpy(P.U0).to("cuda")
    arena = torch.empty_like(U0_dev)
    arena.copy_(U0_dev)
    mesh = H.Mesh(P.mesh, arena)
    pk64 = [H.Packet(mesh, ids, H.FP64) for ids in P.packets]
    pkmx = [H.Packet(mesh, ids, H.FP32_FP64) for ids in P.packets]
    log(f"{len(P.packets)} packets")

    region = None if args.no_check else region_around(P, args.steps)
    errs = None
    if not args.no_check and region is None:
        errs = one_step_errors(P, arena, U0_dev, pk64, pkmx)
        log("one-step errors vs oracle:", json.dumps(errs))

    results = {}
    kernel_ms = {}
    gpu_sub = {}
    for name, pks in (("batched_mixed", pkmx), ("batched_fp64", pk64)):
        arena.copy_(U0_dev)
        b = H.Batch(pks)
        if args.tune:
            b.autotune(P.gamma, reps=3)
        b.run(args.warmup, P.cfl, P.gamma)
        reps = []
        for _ in range(args.repeats):  # the timed region, repeated; the median is reported
            torch.cuda.synchronize()
            ts = time.perf_counter()
            _, step_ms = b.run_timed(args.steps, P.cfl, P.gamma)  # HIP events around every graph replay
            torch.cuda.synchronize()
            el = time.perf_counter() - ts
            reps.append({"wall_ms_per_step": 1e3 * el / args.steps, "device_ms_per_step": float(np.mean(step_ms))})
        wall = float(np.median([r["wall_ms_per_step"] for r in reps]))
        dev = float(np.median([r["device_ms_per_step"] for r in reps]))
        results[name] = {"cell_updates_per_s": cells / (wall * 1e-3), "ms_per_step": wall,
                         "device_ms_per_step": dev, "repeats": reps, "config": b.config()}
        # kernel durations: `steps` eager steps from the initial state
        arena.copy_(U0_dev)
        kernel_ms[name] = b.time_kernels(args.steps, P.cfl, P.gamma)
        b.close()
        if region is not None:  # the state after `steps` steps, centred subset blocks
            torch.cuda.synchronize()
            gpu_sub[name] = np.concatenate([arena[int(P.mesh.offset[i]):int(P.mesh.offset[i]) +
                                                  5 * int(P.mesh.ncells[i])].cpu().numpy()
                                            for i in P.meta["subset"]])
        log(name, json.dumps(results[name]), json.dumps(kernel_ms[name]))

    fused_study = None
    if P.name == "uneven":  # the whole workload with the 8^3 class on the fused step, and that class alone
        for name, pks in (("batched_mixed_fused8", pkmx), ("batched_fp64_fused8", pk64)):
            arena.copy_(U0_dev)
            b = H.Batch(pks)
            if args.tune:
                b.autotune(P.gamma, reps=3)
            b.set_tiling(8, 5)
            b.run(args.warmup, P.cfl, P.gamma)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            _, step_ms = b.run_timed(args.steps, P.cfl, P.gamma)
            torch.cuda.synchronize()
            el = time.perf_counter() - ts
            results[name] = {"cell_updates_per_s": cells * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                             "device_ms_per_step": float(np.mean(step_ms)), "config": b.config()}
            b.close()
            log(name, json.dumps(results[name]))
        fused_study = fused_class_study(P, args.steps, args.warmup)

    # method variants (Einfeldt, PVRS wave speeds; conserved, characteristic PLM; gas + radiation EOS):
    # kernel time of a few eager steps
    # each row's error: one step from the initial state on sampled blocks against the oracle with the same
    # method variant
    check = None
    if not args.no_check:  # sampled blocks: the centred subset where the workload has one
        sub = P.meta.get("subset")
        reg = region_around(P, 1) if sub is not None else None
        check = RowCheck(P, sub, reg) if reg is not None else RowCheck(P, sample_blocks(P), None) \
            if P.name == "uneven" else None
    variants = {}
    for name, prec, opts in (
            ("mixed_einfeldt", H.FP32_FP64 | H.EINFELDT, (O.EINFELDT, 0, 0)),
            ("fp64_einfeldt", H.FP64 | H.EINFELDT, (O.EINFELDT, 0, 0)),
            ("mixed_pvrs", H.FP32_FP64 | H.PVRS, (O.PVRS, 0, 0)), ("fp64_pvrs", H.FP64 | H.PVRS, (O.PVRS, 0, 0)),
            ("mixed_conserved", H.FP32_FP64 | H.CONSERVED, (0, O.CONSERVED, 0)),
            ("fp64_conserved", H.FP64 | H.CONSERVED, (0, O.CONSERVED, 0)),
            ("mixed_characteristic", H.FP32_FP64 | H.CHARACTERISTIC, (0, O.CHARACTERISTIC, 0)),
            ("fp64_characteristic", H.FP64 | H.CHARACTERISTIC, (0, O.CHARACTERISTIC, 0)),
            ("fp64_gas_radiation", H.FP64 | H.GAS_RADIATION, (0, 0, O.GAS_RADIATION))):
        arena.copy_(U0_dev)
        b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
        k = b.time_kernels(min(args.steps, 5), P.cfl, P.gamma)
        b.close()
        variants[name] = {"stage_ms_per_step": k["stage1_ms"] + k["stage2_ms"],
                          "cell_updates_per_s": cells / ((k["stage1_ms"] + k["stage2_ms"]) * 1e-3)}
        if check is not None:
            arena.copy_(U0_dev)
            b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
            dt = b.run(1, P.cfl, P.gamma)
            b.close()
            variants[name]["errors_vs_oracle"] = check.err(gather_blocks(P, arena, check.ids), dt, *opts)
        log(name, json.dumps(variants[name]))

    if not args.no_plain:
        arena.copy_(U0_dev)
        b = H.Batch(pk64)

        def plain_step():
            dt = min(pk.reduce_dt(P.gamma, P.cfl) for pk in pk64)
            b.advance_plain(dt, P.gamma)

        for _ in range(args.warmup):
            plain_step()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(args.steps):
            plain_step()
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        results["plain_fp64"] = {"cell_updates_per_s": cells * args.steps / el, "ms_per_step": 1e3 * el / args.steps}
        if check is not None:
            arena.copy_(U0_dev)
            dt = min(pk.reduce_dt(P.gamma, P.cfl) for pk in pk64)
            b.advance_plain(dt, P.gamma)
            results["plain_fp64"]["errors_vs_oracle"] = check.err(gather_blocks(P, arena, check.ids), dt)
        b.close()
        log("plain_fp64", json.dumps(results["plain_fp64"]))

    cpu = None
    if region is not None:
        ids, m, Uref, dts, cpu = oracle_region_run(P, args.steps)
        errs = {"kind": f"after {args.steps} steps from the initial state, on the centred "
                        f"{len(P.meta['subset'])}-block subset (full-size run on the GPU; oracle on the region "
                        f"around the subset that covers its domain of dependence)"}
        for name, key in (("batched_mixed", "mixed"), ("batched_fp64", "fp64")):
            errs[key] = subset_errors(P, ids, m, Uref, gpu_sub[name])
        log("subset errors vs oracle:", json.dumps(errs))
    if cpu is None and not args.no_cpu:
        from oracle import oracle as O

        ids = np.arange(min(512, P.mesh.nblocks))
        m = P.mesh.subset(ids)
        U = P.mesh.gather(P.U0, ids)
        t0, k = time.perf_counter(), 0
        while time.perf_counter() - t0 < 12.0 and k < 50:
            O.step(m, U, O.dt(m, U, P.gamma, P.cfl), P.gamma)
            k += 1
        el = time.perf_counter() - t0
        cpu = {"value": m.total_cells * k / el, "unit": "cell-updates/s", "cores": O.num_threads(), "kind": "oracle",
               "host": host_cpu(), "sample": f"first {len(ids)} blocks as their own mesh, {k} steps, {el:.1f} s"}
    if cpu:
        log("cpu_baseline", json.dumps(cpu))

    head = results["batched_mixed"]
    km = kernel_ms["batched_mixed"]
    step_dev_ms = head["device_ms_per_step"]  # the step graph's device time over the timed region (median)
    achieved = BYTES_PER_CELL_UPDATE * cells / (step_dev_ms * 1e-3) / 1e9
    achieved_wall = BYTES_PER_CELL_UPDATE * cells / (head["ms_per_step"] * 1e-3) / 1e9
    occ = head["config"].get("occupancy", 0)
    names = {1: f"void hyd::k_stage<3, true, 1, 1, 0, 0, 0, {occ}>(hyd::StageArgs)",
             2: f"void hyd::k_stage<3, true, 2, 1, 0, 0, 0, {occ}>(hyd::StageArgs)"}
    traffic = measured_traffic([names[1], names[2]]) if P.name == "sedov_noise" else None
    per_kernel = {}
    for st, alg in ((1, 80.0), (2, 120.0)):
        ms = km[f"stage{st}_ms"]
        per_kernel[f"stage{st}"] = {"kernel": names[st], "ms": ms, "algorithmic_bytes_per_cell": alg,
                                    "achieved_gbs": alg * cells / (ms * 1e-3) / 1e9,
                                    "frac": alg * cells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    roofline = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_note": "HBM bytes per step (stage-1 + stage-2 launch), PMC FETCH_SIZE + WRITE_SIZE scaled by the "
                        "copy-kernel calibration, from profiles/stage_kernels_large.md (null if the kernel source "
                        "changed since)",
        "kernel": "k_stage stage-1 + stage-2 launches of one step (80 + 120 algorithmic B per interior cell); "
                  "duration = device time of the replayed step graph (both stage kernels and the dt update) from "
                  "HIP events on the mesh stream around every replay, mean over the timed region, median over "
                  f"{args.repeats} repetitions",
        "step_device_ms": step_dev_ms,
        "frac_wall": achieved_wall / HBM_PEAK_GBS,
        "frac_wall_note": "the same 200 B per cell-update over the wall-clock ms_per_step (includes the first dt "
                          "reduction of each timed run and the final read-back)",
        "per_kernel": per_kernel,
        "per_kernel_note": "eager launches of the same kernels with HIP events around each, for `steps` steps "
                           "right after the timed region; stage 2 (120 B) is the dominant kernel",
        "algorithmic_bytes_per_step": BYTES_PER_CELL_UPDATE * cells,
    }
    if probe:
        roofline.update({"copy_probe_gbs": probe["gbs"], "frac_of_copy_probe": achieved / probe["gbs"],
                         "hbm_ceiling": {k: probe[k] for k in ("best_copy", "best_read", "best_write", "configs")}})
    ach64 = BYTES_PER_CELL_UPDATE * cells / (results["batched_fp64"]["device_ms_per_step"] * 1e-3) / 1e9
    # the FP64 path is bound by its vector ALU issue: one wave64 instruction per CU per cycle
    valu64 = measured_valu(["void hyd::k_stage<3, false, 1, 1, 0, 0, 0, 0>(hyd::StageArgs)",
                            "void hyd::k_stage<3, false, 2, 1, 0, 0, 0, 0>(hyd::StageArgs)"]) \
        if P.name == "sedov_noise" else None
    roof64 = None
    if valu64:
        issue = 256 * 2.4e9 * 64  # lane-instructions per second (256 CUs, 2.4 GHz, wave64)
        dev64 = results["batched_fp64"]["device_ms_per_step"] * 1e-3
        roof64 = {"bound": "alu", "achieved": valu64 * cells / dev64 / 1e12, "peak": issue / 1e12,
                  "unit": "T lane-instructions/s", "frac": valu64 * cells / dev64 / issue,
                  "valu_instructions_per_cell_update": valu64,
                  "note": "VALU instructions per cell of the FP64 stage kernels from "
                          "profiles/stage_kernels_valu_large.md (PMC SQ_INSTS_VALU) over the batched FP64 step's "
                          "device time, against one wave64 instruction per CU per cycle"}

    line = {
        "metric": METRIC,
        "value": head["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (PLM+HLLC) / f64 (state, recovery, update, dt)",
        "data": "synthetic (seeded)",
        "config": {"workload": f"{P.name}: {P.mesh.nblocks} blocks of {int(P.mesh.n[0, 0])}^3, {cells} cells, "
                               f"{len(P.packets)} packets, periodic, gamma {P.gamma}, CFL {P.cfl}",
                   "path": "batched mixed FP32/FP64, persistent launch per stage, HIP graph per step",
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paths": {k: {kk: vv for kk, vv in v.items() if kk != "config"} for k, v in results.items()},
        "batched_fp64_roofline_frac": ach64 / HBM_PEAK_GBS,
        "batched_fp64_valu_roofline": roof64,
        "tuning": results["batched_mixed"]["config"],
        "errors_vs_oracle": errs,
        "variants_kernel_time": variants,
        "fused_8cube_class": fused_study,
    }
    if "plain_fp64" in results:
        line["speedup_vs_plain_fp64"] = head["cell_updates_per_s"] / results["plain_fp64"]["cell_updates_per_s"]
    if P.name == "sedov_noise" and not args.no_secondary:
        del arena, U0_dev
        mesh.close()
        torch.cuda.empty_cache()
        line["secondary"] = secondary_paths(min(args.steps, 10), min(args.warmup, 2), not args.no_check)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
