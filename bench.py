#!/usr/bin/env python3
"""Benchmark of the LJ Verlet-list path on one MI355X.

One step = one pass of the whole hot path over one synthetic system held in
HBM: validate and bin the positions into cells, sort them by cell, rebuild
the Verlet list in place, then compute forces, potential energy and virial
(lj_update_neighbors + lj_forces).  The workload is the 131,072-atom FCC
fluid at rho = 1.0, rc = 3.0, skin = 0.3 (32^3 unit cells, jitter +-0.1),
FP64, positions as padded double4 records, atoms cell-sorted (cubic cells of
side >= rc + skin, z-major; `--order lattice | permuted` for the others).

Prints ONE JSON line.  `value` = interacting pairs (r < rc, each unordered
pair once) per second of whole steps.  Extra keys: per-kernel times from HIP
events on the library's stream, the roofline of the dominant kernel, the
force-kernel-only rate (what the paper times), the variant matrix (atom order
x layout x list kind x precision) and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
FP64_VECTOR_TFLOPS = 78.6  # MI355X FP64 vector peak (fused multiply-adds counted as 2)
# Vector operations per second without fusion, FP64 or unpacked FP32: 256 CUs
# x 4 SIMDs x 16 lanes x 2.4 GHz.  The pair test forms r^2 from separately
# rounded products and sums, so no multiply-add can be fused and this is its
# ceiling.
VALU_OPS_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
TEST_OPS = 8               # per candidate pair test: 3 differences, 3 squares, 2 sums
COPY_BYTES = 256 << 20     # size of the calibration copy (read once, written once)


def algorithmic_force_bytes(n: int, entries: int) -> int:
    """Bytes the force evaluation must move once: each atom's position (32 B
    record) and force (32 B), its row bookkeeping (row atom + row length, 8 B)
    and every list entry (4 B)."""
    return n * (32 + 32 + 8) + 4 * entries


def traffic_file(kernel: str) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}_lj131k_hbm_traffic.txt")


def measured_traffic(path: str):
    """HBM bytes per force launch from the committed counter summary (two
    rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE, scaled by a plain copy),
    or None when the summary is missing or the force-kernel sources have
    changed since the counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for src in kv["source_files"].split():
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != kv["source_sha256"]:
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def ordered(s, order: str):
    """The system with its atoms cell-sorted, in lattice order or permuted."""
    from paper_1806_05713_amd import synth
    if order == "cellsorted":
        return synth.cell_sorted(s)
    if order == "permuted":
        return synth.permuted(s, synth.SEEDS["perm"])
    return s


def time_steps(torch, fn, steps: int, warmup: int):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return a.elapsed_time(b) / steps, wall / steps * 1e3


def cpu_baseline(sys_, budget_s: float = 20.0):
    """The oracle (scalar FP64 C, one thread) on the same workload: one step =
    linked-list cell search + counting sort + force loop.  Repeats whole steps
    until about budget_s of CPU time is used (at least one)."""
    from oracle.ljref import Oracle
    O = Oracle()
    rs = sys_.rc + sys_.skin
    times, nin = [], 0
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        rp, col = O.cell_pairs(sys_.pos, sys_.box, rs)
        F, E, W, nin = O.forces(sys_.pos, sys_.box, 1.0, 1.0, sys_.rc, rp, col)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(times) >= 20:
            break
    t = float(np.median(times))
    return {"value": nin / t, "unit": "pair interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(times)} whole steps (cell list build + forces, {sys_.n} atoms, "
                      f"{nin} interacting pairs), median {t:.3f} s/step, single thread, "
                      f"host {platform.processor() or platform.machine()}, "
                      f"{os.cpu_count()} logical CPUs present"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kind", choices=["full", "half"], default="full")
    ap.add_argument("--order", choices=["cellsorted", "lattice", "permuted"],
                    default="cellsorted", help="atom order of the input")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per list row (0: default)")
    ap.add_argument("--build-lanes", type=int, default=0,
                    help="lanes per row in the list build, 64, 1, 2 or 4 (0: default, 64)")
    ap.add_argument("--force-batch", type=int, default=0,
                    help="list entries in flight per lane in the force kernel, 2, 4 or 8 "
                         "(0: default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the variant matrix")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain 256 MiB device-to-device copies (a known-size "
                         "kernel that scales HBM byte counters)")
    ap.add_argument("--workload", choices=["lj131k", "lj4m", "batch512", "accuracy"],
                    default="lj131k",
                    help="lj131k (default): build + forces on the 131k-atom fluid; lj4m: "
                         "100-step NVE of the 4M-atom fluid; batch512: 100-step NVE of 512 "
                         "batched systems; accuracy: 10,000-step mixed vs FP64 run on the "
                         "500k-atom fluid (use --steps to shorten)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the "
              "library runs on a single GPU: sharding by spatial domains is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_05713_amd import lj, synth
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload != "lj131k":
        from paper_1806_05713_amd import workloads
        if args.workload == "accuracy":
            result = workloads.accuracy_lj500k(steps=args.steps)
        else:
            fn = workloads.bench_lj4m if args.workload == "lj4m" else workloads.bench_batch512
            result = fn(steps=args.steps, warmup=args.warmup, cpu=not args.no_cpu)
        print(json.dumps(result), flush=True)
        return
    ctx = lj.Context(0)
    if args.build_lanes:
        ctx.tune_set(lj.LJ_TUNE_BUILD_LANES, args.build_lanes)
    if args.force_batch:
        ctx.tune_set(lj.LJ_TUNE_FORCE_BATCH, args.force_batch)

    s = ordered(synth.lj131k(), args.order)
    kind = lj.LJ_LIST_FULL if args.kind == "full" else lj.LJ_LIST_HALF
    pos = torch.from_numpy(synth.aos4(s.pos)).to(dev)
    nl = lj.lj_build_neighbors(ctx, pos, s.box, s.rc, s.skin, kind=kind, lanes=args.lanes)
    force = torch.empty_like(pos)
    out = torch.empty(2, dtype=torch.float64, device=dev)

    def step():
        lj.lj_update_neighbors(ctx, pos, s.box, nl)
        lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_FP64, force, out)

    def force_only():
        lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_FP64, force, out)

    # ---- timed region: exactly K whole steps
    torch.cuda.synchronize()
    ms_step, wall_step = time_steps(torch, step, args.steps, args.warmup)
    ctx.sync()
    _, _, _, cnt = lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_FP64, force, out)
    torch.cuda.synchronize()
    npairs = int(cnt.item())
    desc = nl.info()
    value = npairs / (ms_step * 1e-3)

    # ---- per-kernel device times: the same K steps with HIP events around each launch
    ctx.profile_begin()
    for _ in range(args.steps):
        step()
    prof = ctx.profile_end()
    per = {k: (v[0] / max(v[1], 1) * 1e3) for k, v in prof.items()}   # us per launch
    ms_force_only, _ = time_steps(torch, force_only, args.steps, 2)

    # the same whole step with the mixed-precision force kernel (fixed-point
    # gathers, FP32 pair terms); the pair set is the FP64 one
    force_m = torch.empty_like(pos)

    def step_mixed():
        lj.lj_update_neighbors(ctx, pos, s.box, nl)
        lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_MIXED, force_m, out)

    ms_step_mixed, _ = time_steps(torch, step_mixed, args.steps, args.warmup)
    ctx.sync()

    force_us = per["force"]
    neigh_us = per["neigh"]
    default_shape = (args.order == "cellsorted" and args.lanes in (0, 8) and
                     args.build_lanes in (0, 64) and
                     args.force_batch in (0, 4))
    bytes_force = algorithmic_force_bytes(s.n, desc.entries)
    force_gbs = bytes_force / (force_us * 1e-6) / 1e9
    roofline_force = {
        "kernel": "k_force (FP64, full list)" if kind == lj.LJ_LIST_FULL
        else "k_force (FP64, half list)",
        "bound": "hbm", "achieved": round(force_gbs, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(force_gbs / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(traffic_file("k_force"))
        if (kind == lj.LJ_LIST_FULL and default_shape) else None,
        "bytes_per_launch": bytes_force, "us_per_launch": round(force_us, 3)}
    # the list build: bound by vector-ALU issue; its algorithmic work is the
    # distance test of every candidate pair it examines (8 operations, unfused:
    # FP32 first, FP64 again in the narrow band around rs; unpacked FP32 and
    # FP64 issue at the same rate)
    neigh_tflops = TEST_OPS * desc.tests / (neigh_us * 1e-6) / 1e12
    roofline_neigh = {
        "kernel": "k_neigh_rows (list build, exact pair tests: FP32 with an FP64 band)",
        "bound": "alu", "achieved": round(neigh_tflops, 3), "peak": round(VALU_OPS_PEAK_T, 2),
        "unit": "TFLOP/s", "frac": round(neigh_tflops / VALU_OPS_PEAK_T, 4),
        "traffic": measured_traffic(traffic_file("k_neigh_rows"))
        if (kind == lj.LJ_LIST_FULL and default_shape) else None,
        "candidate_tests_per_launch": int(desc.tests), "us_per_launch": round(neigh_us, 3)}
    dominant = "force" if force_us >= neigh_us else "neigh"
    roofline = roofline_force if dominant == "force" else roofline_neigh

    variants = {}
    if not args.no_variants:
        for order in ("cellsorted", "lattice", "permuted"):
            sv = ordered(synth.lj131k(), order)
            for layout_name, layout in (("aos4", 0), ("soa", 1)):
                p = torch.from_numpy(synth.aos4(sv.pos) if layout == 0 else synth.soa(sv.pos)).to(dev)
                f = torch.empty_like(p)
                for kname, kv in (("full", lj.LJ_LIST_FULL), ("half", lj.LJ_LIST_HALF)):
                    l2 = lj.lj_build_neighbors(ctx, p, sv.box, sv.rc, sv.skin, kind=kv)
                    for prec_name, prec in (("fp64", lj.LJ_FP64), ("mixed", lj.LJ_MIXED)):
                        def fo():
                            lj.lj_forces(ctx, p, sv.box, 1.0, 1.0, sv.rc, l2, prec, f, out)
                        ms, _ = time_steps(torch, fo, 50, 5)
                        variants[f"{order}/{layout_name}/{kname}/{prec_name}"] = {
                            "force_us": round(ms * 1e3, 3),
                            "pairs_per_s": round(npairs / (ms * 1e-3), 1)}
                    l2.free()

    result = {
        "metric": "pair interactions/s (FP64 vs FP32/FP64-mixed) at rho=1, rc=3; HBM GB/s",
        "value": round(value, 1),
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 6),
        "wall_ms_per_step": round(wall_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 LJ fluid, 131,072 atoms (32^3 FCC x4), rho=1.0, jitter "
                               "+-0.1 sigma, eps=sigma=1, rc=3.0, skin=0.3, atoms "
                               + {"cellsorted": "cell-sorted (cells of side >= rc + skin)",
                                  "lattice": "in lattice order",
                                  "permuted": "in random order"}[args.order]
                               + "; step = cell binning + list rebuild + forces/energy/virial",
                   "atoms": s.n, "list": args.kind, "lanes": desc.lanes, "layout": "aos4",
                   "order": args.order, "precision": "fp64",
                   "list_entries": desc.entries, "candidate_tests": int(desc.tests),
                   "interacting_pairs": npairs},
        "kernel_us": {k: round(v, 3) for k, v in per.items()},
        "dominant_kernel": dominant,
        "roofline": roofline,
        "roofline_force": roofline_force,
        "roofline_neigh": roofline_neigh,
        "mixed_step": {"ms_per_step": round(ms_step_mixed, 6),
                       "pairs_per_s": round(npairs / (ms_step_mixed * 1e-3), 1),
                       "speedup_over_fp64": round(ms_step / ms_step_mixed, 3)},
        "force_only": {"us": round(ms_force_only * 1e3, 3),
                       "pairs_per_s": round(npairs / (ms_force_only * 1e-3), 1),
                       "alg_GBps": round(bytes_force / (ms_force_only * 1e-3) / 1e9, 1)},
        "variants": variants,
    }
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(s)
        result["gpu_vs_cpu_oracle"] = round(value / result["cpu_baseline"]["value"], 1)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
