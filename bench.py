#!/usr/bin/env python3
"""Benchmark of the LJ Verlet-list path on one MI355X.

Headline (the paper's measurement, Sec. II: the time of the force
evaluations, the list built once): one step = one evaluation of forces,
potential energy and virial over the Verlet list (lj_forces: the force
kernel and the fixed-order energy/virial reduction) on the 131,072-atom FCC
fluid at rho = 1.0, rc = 3.0, skin = 0.3 (32^3 unit cells, jitter +-0.1),
FP64, full list, positions as padded double4 records, atoms cell-sorted
(`--order lattice | permuted` for the others).  `value` = interacting pairs
(r < rc, each unordered pair once) per second of such steps, timed with HIP
events on the library's stream over exactly K steps.

Prints ONE JSON line.  Besides the contract keys: the roofline of the force
kernel (its algorithmic bytes over its mean launch time, from the library's
HIP-event profiler, against 8 TB/s), its HBM traffic, L2 hit rate and VALU
issue utilisation from the committed rocprofv3 counter summary while the
kernel sources are unchanged since the counters were taken; the whole hot
path per step (cell binning + list rebuild + forces) with the list build's
own roofline; mixed precision, half list, force-shifted truncation and
64-byte records; the order x layout x list x precision matrix; the 4M-atom
NVE run and the 512-system batch (short forms); and the oracle baseline
(its force evaluation, one thread and all host cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
# The list build's pair test runs in FP32 (FMA-contracted) on unpacked
# instructions (packed FP32 is disabled in this build), so its ceiling is
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s, half the
# published packed FP32 vector peak of 157.3.
FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
TEST_FLOPS = 8             # per candidate pair test: 3 differences, 3 squares, 2 sums
COPY_BYTES = 256 << 20     # size of the calibration copy (read once, written once)
SIMDS = 256 * 4
CLOCK_GHZ = 2.4


def algorithmic_force_bytes(n: int, entries: int) -> int:
    """Bytes the force evaluation must move once: each atom's position (32 B
    record) and force (32 B), its row bookkeeping (row atom + row length, 8 B)
    and every list entry (4 B)."""
    return n * (32 + 32 + 8) + 4 * entries


def profile_summary(name: str):
    """Key/value lines of a committed rocprofv3 summary under profiles/, or
    None when it is missing or the sources it names have changed since the
    counters were taken (then its figures no longer describe the kernel)."""
    path = os.path.join(ROOT, "profiles", name)
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
    except (KeyError, OSError):
        return None
    return kv


def counters(name: str, keys):
    kv = profile_summary(name)
    if kv is None:
        return None
    out = {"source": f"profiles/{name}"}
    for k in keys:
        try:
            out[k] = float(kv[k].split()[0])
        except (KeyError, ValueError, IndexError):
            out[k] = None
    return out


def ordered(s, order: str):
    """The system with its atoms cell-sorted, in lattice order or permuted."""
    from paper_1806_05713_amd import synth
    if order == "cellsorted":
        return synth.cell_sorted(s)
    if order == "permuted":
        return synth.permuted(s, synth.SEEDS["perm"])
    return s


def time_steps(torch, fn, steps: int, warmup: int):
    """ms per call of fn over exactly `steps` calls after `warmup`, from HIP
    events on the current stream (the library's), with a synchronisation on
    both sides; also the wall-clock ms per call."""
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


def per_launch(ctx, fn, steps: int):
    """us per launch of each phase over `steps` calls of fn (the library's
    HIP-event profiler on its stream)."""
    ctx.profile_begin()
    for _ in range(steps):
        fn()
    prof = ctx.profile_end()
    return {k: (v[0] / max(v[1], 1) * 1e3) for k, v in prof.items()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(s, single_budget_s: float = 10.0, multi_budget_s: float = 6.0):
    """The oracle (scalar FP64 C, -O2 without contraction) timed on this
    host: its force evaluation over the full list (built once by its own
    cell list, not timed), as the paper times the force calls alone; one
    thread, and all host cores (an OpenMP loop over rows whose result is
    bitwise that of one thread).  Each leg repeats whole evaluations until
    its budget is used; the median is reported."""
    from oracle.ljref import Oracle
    O = Oracle()
    rp, col = O.cell_pairs(s.pos, s.box, s.rc + s.skin)
    frp, fcol = O.full_pairs(rp, col)
    legs = {}
    ref = None
    for name, threads in (("single", 1), ("all", 0)):
        was = O.set_threads(0)
        # all cores: the host's share for this process (OMP_NUM_THREADS when set)
        n_all = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
        used = O.set_threads(threads if threads else n_all)
        times = []
        t_start = time.perf_counter()
        budget = single_budget_s if threads == 1 else multi_budget_s
        while True:
            t0 = time.perf_counter()
            F, E, W, nin = O.forces_full(s.pos, s.box, 1.0, 1.0, s.rc, frp, fcol)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_start > budget or len(times) >= 200:
                break
        O.set_threads(was)
        if ref is None:
            ref = (F, E, W)
        else:
            legs["bitwise_equal_to_single_thread"] = bool(
                np.array_equal(F, ref[0]) and E == ref[1] and W == ref[2])
        t = float(np.median(times))
        legs[name] = {"threads": used, "evaluations": len(times), "s_per_eval": round(t, 5),
                      "pairs_per_s": round(nin / t, 1)}
    return {"value": legs["all"]["pairs_per_s"], "unit": "pair interactions/s",
            "cores": legs["all"]["threads"], "kind": "oracle",
            "sample": f"{legs['all']['evaluations']} force evaluations of the oracle over the "
                      f"full list ({s.n} atoms, {nin} interacting pairs; list built once, not "
                      f"timed), OpenMP over rows on {legs['all']['threads']} threads, median "
                      f"{legs['all']['s_per_eval']} s each; host {cpu_model()}, nproc "
                      f"{os.cpu_count()}",
            "single_thread": legs["single"], "all_cores": legs["all"],
            "bitwise_equal_to_single_thread": legs["bitwise_equal_to_single_thread"],
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kind", choices=["full", "half"], default="full")
    ap.add_argument("--order", choices=["cellsorted", "lattice", "permuted"],
                    default="cellsorted", help="atom order of the input")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes per list row (0: the tuned or default choice)")
    ap.add_argument("--build-lanes", type=int, default=0,
                    help="lanes per row in the list build, 64, 1, 2 or 4 (0: default, 64)")
    ap.add_argument("--force-batch", type=int, default=0,
                    help="list entries in flight per lane in the force kernel, 2, 4 or 8 "
                         "(0: default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the variant matrix and the 4M / batch workloads")
    ap.add_argument("--no-extras", action="store_true",
                    help="the headline only (no whole step, other forms, variants, 4M or "
                         "batch workloads): the command the force kernel's counters are "
                         "taken with")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain 256 MiB device-to-device copies (a known-size "
                         "kernel that scales HBM byte counters)")
    ap.add_argument("--workload", choices=["lj131k", "lj4m", "batch512", "accuracy"],
                    default="lj131k",
                    help="lj131k (default): the headline and its extras; lj4m: the 4M-atom "
                         "NVE runs alone; batch512: the batched NVE alone (--tune to retune "
                         "its launch shapes into the cache); accuracy: 10,000-step mixed vs "
                         "FP64 run on the 500k-atom fluid (use --steps to shorten)")
    ap.add_argument("--tune", action="store_true",
                    help="retune launch shapes (131k headline or batch512) and save them in "
                         "the autotuner's cache")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the "
              "library runs on a single GPU: sharding by spatial domains is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_05713_amd import autotune, lj, synth, workloads
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
        if args.workload == "accuracy":
            result = workloads.accuracy_lj500k(steps=args.steps)
        elif args.workload == "lj4m":
            result = workloads.bench_lj4m(steps=args.steps, warmup=args.warmup)
        else:
            result = workloads.bench_batch512(steps=args.steps, warmup=args.warmup,
                                              tune=args.tune)
        print(json.dumps(result), flush=True)
        return

    ctx = lj.Context(0)
    s = ordered(synth.lj131k(), args.order)
    kind = lj.LJ_LIST_FULL if args.kind == "full" else lj.LJ_LIST_HALF
    pos = torch.from_numpy(synth.aos4(s.pos)).to(dev)
    # launch shapes: given on the command line, else the autotuner's cached
    # choice for this device and workload shape, else the library's defaults
    tkey = autotune.system_key(s.n, 1.0, s.rc + s.skin, kind, lj.LJ_FP64)
    if args.tune:
        # tuned for the whole step (list build + force evaluation): the list
        # layout serves both, and the shape that gives the force kernel alone
        # its last few percent (4 lanes per row) slows the build by a third
        shape = autotune.best_config(ctx, pos, s.box, s.rc, s.skin, kind, lj.LJ_FP64, 1.0,
                                     objective="step_us", retune=True,
                                     space={"lanes": (4, 8, 16), "build_lanes": (64,),
                                            "batch": (2, 4, 8), "cell_div": (2,)},
                                     log=lambda m: print(f"[tune] {m}", file=sys.stderr))
        shape_from = "tuned now"
    else:
        shape = autotune.cached(tkey)
        shape_from = "cache" if shape else "defaults"
    shape = dict(shape or {})
    if args.lanes:
        shape["lanes"], shape_from = args.lanes, "command line"
    if args.build_lanes:
        shape["build_lanes"], shape_from = args.build_lanes, "command line"
    if args.force_batch:
        shape["batch"], shape_from = args.force_batch, "command line"
    autotune.apply(ctx, shape)
    nl = lj.lj_build_neighbors(ctx, pos, s.box, s.rc, s.skin, kind=kind,
                               lanes=shape.get("lanes", 0))
    force = torch.empty_like(pos)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)

    def step():
        lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_FP64, force, out)

    # ---- timed region: exactly K force evaluations over the list built once
    torch.cuda.synchronize()
    ms_step, wall_step = time_steps(torch, step, args.steps, args.warmup)
    ctx.sync()
    _, _, _, cnt = lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_FP64, force, out)
    torch.cuda.synchronize()
    npairs = int(cnt.item())
    desc = nl.info()
    value = npairs / (ms_step * 1e-3)

    # ---- per-kernel device times over the same K evaluations
    per = per_launch(ctx, step, args.steps)
    force_us = per["force"]
    bytes_force = algorithmic_force_bytes(s.n, desc.entries)
    force_gbs = bytes_force / (force_us * 1e-6) / 1e9
    default_shape = (args.order == "cellsorted" and kind == lj.LJ_LIST_FULL and
                     desc.lanes == 8 and shape.get("batch", 4) in (0, 4))
    cf = counters("k_force_lj131k_counters.txt",
                  ["traffic_bytes_per_launch", "l2_hit_rate", "valu_issue_utilisation",
                   "ta_busy", "vmem_instructions_per_launch", "valu_instructions_per_launch",
                   "duration_us"]) if default_shape else None
    roofline = {
        "kernel": "k_force (FP64, full list)" if kind == lj.LJ_LIST_FULL
        else "k_force (FP64, half list)",
        "bound": "hbm", "achieved": round(force_gbs, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(force_gbs / HBM_PEAK_GBS, 4),
        "traffic": int(cf["traffic_bytes_per_launch"]) if cf and cf["traffic_bytes_per_launch"]
        else None,
        "bytes_per_launch": bytes_force, "us_per_launch": round(force_us, 3),
        "pairs_per_s_kernel": round(npairs / (force_us * 1e-6), 1),
        "counters": cf}

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
                               + f", {args.kind} Verlet list built once; step = one force/"
                               "energy/virial evaluation over the list (the paper times the "
                               "force calls alone)",
                   "atoms": s.n, "list": args.kind, "lanes": desc.lanes, "layout": "aos4",
                   "order": args.order, "precision": "fp64", "launch_shapes": shape,
                   "launch_shapes_from": shape_from,
                   "list_entries": desc.entries, "interacting_pairs": npairs},
        "kernel_us": {k: round(v, 3) for k, v in per.items()},
        "roofline": roofline,
    }

    if args.no_extras:
        if not args.no_cpu:
            result["cpu_baseline"] = cpu_baseline(s)
        print(json.dumps(result), flush=True)
        return

    # ---- the whole hot path per step: bin + sort + rebuild the list in place + forces
    def whole():
        lj.lj_update_neighbors(ctx, pos, s.box, nl)
        lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_FP64, force, out)

    ms_whole, _ = time_steps(torch, whole, args.steps, args.warmup)
    ctx.sync()
    per_w = per_launch(ctx, whole, args.steps)
    desc = nl.info()
    neigh_tf = TEST_FLOPS * desc.tests / (per_w["neigh"] * 1e-6) / 1e12
    cb = counters("k_neigh_rows_lj131k_counters.txt",
                  ["traffic_bytes_per_launch", "l2_hit_rate", "valu_issue_utilisation",
                   "valu_instructions_per_launch", "duration_us"]) if default_shape else None
    result["whole_step"] = {
        "what": "cell binning and sort, list rebuild in place, forces/energy/virial (the whole "
                "hot path over one input resident in HBM)",
        "ms_per_step": round(ms_whole, 6),
        "pairs_per_s": round(npairs / (ms_whole * 1e-3), 1),
        "kernel_us": {k: round(v, 3) for k, v in per_w.items()},
        "roofline_build": {"kernel": "k_neigh_rows (list build: FP32 pair test with an FP64 "
                                     "band, FMA-contracted)",
                           "bound": "alu", "unit": "TFLOP/s",
                           "achieved": round(neigh_tf, 3),
                           "peak": round(FP32_UNPACKED_TFLOPS, 1),
                           "frac": round(neigh_tf / FP32_UNPACKED_TFLOPS, 4),
                           "frac_of_published_fp32_157": round(neigh_tf / 157.3, 4),
                           "candidate_tests_per_launch": int(desc.tests),
                           "us_per_launch": round(per_w["neigh"], 3),
                           "counters": cb}}

    # ---- the other forms of the force evaluation (same list kind and atoms)
    def rate(fn, reps=None):
        ms, _ = time_steps(torch, fn, reps or args.steps, 3)
        return {"us": round(ms * 1e3, 3), "pairs_per_s": round(npairs / (ms * 1e-3), 1),
                "speedup_over_fp64": round(ms_step / ms, 3)}

    lj.lj_update_neighbors(ctx, pos, s.box, nl)
    ctx.sync()
    force_m = torch.empty_like(pos)
    result["mixed"] = {
        "what": "fixed-point (32-bit, fraction of the box) position gathers, FP64 r^2 and "
                "exact cutoff test, FP32 pair terms, FP64 accumulation and reductions",
        **rate(lambda: lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_MIXED, force_m,
                                    out))}
    result["force_shifted"] = rate(lambda: lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl,
                                                        lj.LJ_FP64, force_m, out, trunc=1))
    nl_h = lj.lj_build_neighbors(ctx, pos, s.box, s.rc, s.skin, kind=lj.LJ_LIST_HALF)
    result["half_list"] = rate(lambda: lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl_h,
                                                    lj.LJ_FP64, force_m, out), 20)
    result["half_list"]["entries"] = nl_h.info().entries
    nl_h.free()
    rec = np.zeros((s.n, 8))
    rec[:, :3] = s.pos
    pos8 = torch.from_numpy(rec).to(dev)
    nl8 = lj.lj_build_neighbors(ctx, pos8, s.box, s.rc, s.skin, kind=kind,
                                lanes=shape.get("lanes", 0))
    result["aos8_records"] = rate(lambda: lj.lj_forces(ctx, pos8, s.box, 1.0, 1.0, s.rc, nl8,
                                                       lj.LJ_FP64, force_m, out))
    nl8.free()
    del pos8

    if not args.no_variants:
        variants = {}
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
                        ms, _ = time_steps(torch, fo, 20, 3)
                        variants[f"{order}/{layout_name}/{kname}/{prec_name}"] = {
                            "force_us": round(ms * 1e3, 3),
                            "pairs_per_s": round(npairs / (ms * 1e-3), 1)}
                    l2.free()
        result["variants"] = variants
        nl.free()
        ctx.close()
        del pos, force, force_m
        torch.cuda.empty_cache()
        result["lj4m_nve"] = workloads.bench_lj4m(steps=100, warmup=10)
        torch.cuda.empty_cache()
        result["batch512_nve"] = workloads.bench_batch512(steps=100, warmup=10)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(s)
        result["gpu_vs_cpu_oracle_all_cores"] = round(value / result["cpu_baseline"]["value"], 1)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
