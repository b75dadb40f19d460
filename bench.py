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
HBM).  Roofline: HBM, 200 algorithmic bytes per cell-update (FP64 state, five
state passes: stage 1 reads Un and writes U1, stage 2 reads U1 and Un and
writes Un+1), 8.0 TB/s peak; the stage kernel's launch durations are measured
with HIP events on the mesh stream.  Errors vs the FP64 oracle are measured on
sampled blocks after one step from the initial state.  cpu_baseline: the
oracle (plain FP64 C, OpenMP) on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large|smooth|uneven|sedov]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s and % HBM roofline, FP32-batched vs FP64-plain, 1 MI355X"
HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL_UPDATE = 200.0


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
    return ids, m, U, dts, cpu


def host_cpu() -> str:
    """The host CPU's model name and the logical CPUs this process may use."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {len(os.sched_getaffinity(0))} logical CPUs available"


def subset_errors(P, ids, m, Uref, U_gpu_sub):
    """Errors of GPU states (arrays of the subset blocks, subset layout) vs the
    oracle's region run on the centred subset."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import l1_rho, rel_err

    pos = {int(b): k for k, b in enumerate(ids)}
    inner = [pos[int(b)] for b in P.meta["subset"]]
    ms = m.subset(inner)
    R = m.gather(Uref, inner)
    return {"max_rel_err": rel_err(ms, U_gpu_sub, R), "l1_rho_rel": l1_rho(ms, U_gpu_sub, R)}


def copy_bandwidth(n_doubles=1 << 28, reps=5):
    """GB/s of the project's plain stream-copy kernels on two 2 GiB buffers
    (far larger than the 256 MB last-level cache): read + write bytes / time,
    best of the two kernel forms."""
    import ctypes as C

    import torch

    lib = C.CDLL(os.path.join(ROOT, "paper_2507_09337_amd", "libhydro_probe.so"))
    lib.copy_probe.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_int,
                               C.POINTER(C.c_double)]
    src = torch.ones(n_doubles, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    out = {"bytes_per_copy": 16 * n_doubles}
    for form in (0, 1):
        ms = C.c_double(0.0)
        dst.zero_()
        rc = lib.copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n_doubles,
                            C.c_void_p(torch.cuda.current_stream().cuda_stream), reps, form, C.byref(ms))
        if rc != 0:
            raise RuntimeError(f"copy_probe failed with {rc}")
        out[f"form{form}_gbs"] = 2 * 8 * n_doubles / (ms.value * 1e-3) / 1e9
        out[f"form{form}_verified"] = bool(torch.equal(src, dst))
    out["gbs"] = max(out["form0_gbs"], out["form1_gbs"])
    del src, dst
    torch.cuda.empty_cache()
    return out


def measured_traffic(kernel_names):
    """HBM bytes per step of the given stage kernels from the committed
    rocprofv3 counter summary, or None when the summary is missing or was
    taken on a different version of the kernel source."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "stage_kernels_large.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("TRAFFIC_JSON "):
            rec = json.loads(line[len("TRAFFIC_JSON "):])
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2507_09337_amd", "csrc", "kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["kernels_sha256"]:
        return None
    total = 0.0
    for k in kernel_names:
        t = rec["per_launch"].get(k)
        if t is None:
            return None
        total += t["fetch_bytes"] + t["write_bytes"]
    return total


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
        for nslots in (1, 3, 4):
            host = torch.from_numpy(P.U0.copy()).pin_memory()
            hs = H.HostStream(P.mesh, host, P.packets, prec, nslots)
            hs.run(args.warmup, P.cfl, P.gamma)
            ts = time.perf_counter()
            hs.run(args.steps, P.cfl, P.gamma)
            el = time.perf_counter() - ts
            hs.close()
            out[f"{name}_slots{nslots}"] = {"cell_updates_per_s": cells * args.steps / el,
                                            "ms_per_step": 1e3 * el / args.steps,
                                            "pcie_gbs": 80.0 * cells * args.steps / el / 1e9}
            log(name, nslots, json.dumps(out[f"{name}_slots{nslots}"]))
    best = max((v for k, v in out.items() if k.startswith("mixed")), key=lambda v: v["cell_updates_per_s"])
    print(json.dumps({"metric": "cell-updates/s, host-resident packets (PCIe-inclusive), uneven workload, 1 MI355X",
                      "value": best["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms_per_step"],
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32 (PLM+HLLC) / f64 (state, recovery, update, dt)", "data": "synthetic (seeded)",
                      "config": {"workload": f"uneven: {P.mesh.nblocks} self-periodic blocks, {cells} cells, "
                                             f"{len(P.packets)} packets, state in pinned host memory"},
                      "paths": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-packet FP64 path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tune", action="store_true", help="autotune the batched launches first")
    ap.add_argument("--no-check", action="store_true", help="skip the one-step error check against the oracle")
    ap.add_argument("--host-packets", action="store_true",
                    help="instead: host-resident packets of the uneven workload streamed through device slots "
                         "(PCIe-inclusive rate; prints its own line)")
    args = ap.parse_args()
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
    probe = copy_bandwidth()
    log("copy probe:", json.dumps(probe))
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
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, step_ms = b.run_timed(args.steps, P.cfl, P.gamma)  # HIP events around every graph replay
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        results[name] = {"cell_updates_per_s": cells * args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                         "device_ms_per_step": float(np.mean(step_ms)), "config": b.config()}
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

    # method variants (Einfeldt, PVRS wave speeds; conserved, characteristic PLM; gas + radiation EOS):
    # kernel time of a few eager steps
    variants = {}
    for name, prec in (("mixed_einfeldt", H.FP32_FP64 | H.EINFELDT), ("fp64_einfeldt", H.FP64 | H.EINFELDT),
                       ("mixed_pvrs", H.FP32_FP64 | H.PVRS), ("fp64_pvrs", H.FP64 | H.PVRS),
                       ("mixed_conserved", H.FP32_FP64 | H.CONSERVED), ("fp64_conserved", H.FP64 | H.CONSERVED),
                       ("mixed_characteristic", H.FP32_FP64 | H.CHARACTERISTIC),
                       ("fp64_characteristic", H.FP64 | H.CHARACTERISTIC),
                       ("fp64_gas_radiation", H.FP64 | H.GAS_RADIATION)):
        arena.copy_(U0_dev)
        b = H.Batch([H.Packet(mesh, ids, prec) for ids in P.packets])
        k = b.time_kernels(min(args.steps, 5), P.cfl, P.gamma)
        b.close()
        variants[name] = {"stage_ms_per_step": k["stage1_ms"] + k["stage2_ms"],
                          "cell_updates_per_s": cells / ((k["stage1_ms"] + k["stage2_ms"]) * 1e-3)}
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
    step_dev_ms = head["device_ms_per_step"]  # the step graph's device time over the timed region
    achieved = BYTES_PER_CELL_UPDATE * cells / (step_dev_ms * 1e-3) / 1e9
    traffic = measured_traffic(["void hyd::k_stage<3, true, 1, 1, 0, 0, 0>(hyd::StageArgs)",
                                "void hyd::k_stage<3, true, 2, 1, 0, 0, 0>(hyd::StageArgs)"]) if P.name == "sedov_noise" else None
    roofline = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_note": "HBM bytes per step (stage-1 + stage-2 launch), PMC FETCH_SIZE + WRITE_SIZE scaled by the "
                        "copy-kernel calibration, from profiles/stage_kernels_large.md (null if the kernel source "
                        "changed since)",
        "kernel": "k_stage stage-1 + stage-2 launches of one step (80 + 120 algorithmic B per interior cell); "
                  "duration = mean device time of the replayed step graph (both stage kernels and the dt update) "
                  "over the timed region, from HIP events on the mesh stream around every replay",
        "step_device_ms": step_dev_ms,
        "stage1_ms": km["stage1_ms"], "stage2_ms": km["stage2_ms"],
        "stage_ms_note": "stage1_ms / stage2_ms: mean HIP-event durations of the same kernels launched eagerly "
                         "for `steps` steps right after the timed region (the split between the two launches)",
        "algorithmic_bytes_per_step": BYTES_PER_CELL_UPDATE * cells,
        "copy_probe_gbs": probe["gbs"], "frac_of_copy_probe": achieved / probe["gbs"],
    }
    ach64 = BYTES_PER_CELL_UPDATE * cells / (results["batched_fp64"]["device_ms_per_step"] * 1e-3) / 1e9

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
        "tuning": results["batched_mixed"]["config"],
        "errors_vs_oracle": errs,
        "variants_kernel_time": variants,
    }
    if "plain_fp64" in results:
        line["speedup_vs_plain_fp64"] = head["cell_updates_per_s"] / results["plain_fp64"]["cell_updates_per_s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
