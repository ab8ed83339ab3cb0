"""Measured workloads beyond the 131k-atom force benchmark: the 4M-atom NVE
run, the 512-system batched NVE run and the 10,000-step mixed-precision
accuracy run.  Each returns a result dictionary (pair interactions per
second of whole MD steps, with per-phase kernel times from HIP events on the
library's stream).

An MD step here is: drift, the in-place list rebuild (every 10th step, or
when an atom has moved more than skin/2), forces, kick, and the per-step
log; runs are captured as HIP-graph cycles of 10 steps.
"""
from __future__ import annotations

import sys
import time

import numpy as np

from . import lj, synth

HBM_PEAK_GBS = 8000.0


def _note(msg: str) -> None:
    print(f"[workload] {msg}", file=sys.stderr, flush=True)


def _sync(ctx) -> bool:
    """lj_sync; True if it reported a fixed rebuild cadence whose list went
    stale (some atom moved more than skin/2 between builds)."""
    try:
        ctx.sync()
    except lj.LJError as e:
        if e.status != lj.LJ_E_STALE:
            raise
        return True
    return False


def _state(pos0: np.ndarray, vel0: np.ndarray, layout: int, dev):
    """Device arrays (pos, vel, force) for a run in `layout`: AoS4 records,
    or LJ_AOS8 position-velocity records (vel is then None; forces AoS4)."""
    import torch
    if layout == lj.LJ_AOS8:
        rec = np.zeros((pos0.shape[0], 8))
        rec[:, :3] = pos0
        rec[:, 4:7] = vel0
        pos = torch.from_numpy(rec).to(dev)
        return pos, None, torch.zeros((pos0.shape[0], 4), dtype=torch.float64, device=dev)
    pos = torch.from_numpy(synth.aos4(pos0)).to(dev)
    vel = torch.from_numpy(synth.aos4(vel0)).to(dev)
    return pos, vel, torch.zeros_like(pos)


def nve_measure(ctx, pos0, vel0, box, rc, steps: int, precision: int, every: int = 10,
                layout: int = lj.LJ_AOS4, batch_n=None, lanes: int = 0, warmup: int = 10,
                profile_steps: int = 20) -> dict:
    """One NVE measurement (eps = sigma = 1, dt = 0.005, full list): `steps`
    HIP-graph steps timed with HIP events on the context's stream after
    `warmup` untimed ones (rounded up to whole cycles of 10: the first cycle
    captures the graph), then the per-phase device time of `profile_steps`
    eager steps from the library's profiler.  batch_n: the atom counts of a
    batch (box and rc per system), else one system."""
    import torch
    dev = torch.device("cuda:0")
    batch = batch_n is not None
    ones = np.ones(len(batch_n)) if batch else 1.0
    res = {}
    with torch.cuda.stream(ctx.stream):
        pos, vel, force = _state(pos0, vel0, layout, dev)
        torch.cuda.synchronize()
        if batch:
            nl = lj.lj_build_neighbors_batch(ctx, pos, batch_n, box, rc, 0.3,
                                             kind=lj.LJ_LIST_FULL, lanes=lanes)
        else:
            nl = lj.lj_build_neighbors(ctx, pos, box, rc, 0.3, kind=lj.LJ_LIST_FULL, lanes=lanes)
        entries = nl.info().entries
        warm = -(-max(int(warmup), 0) // 10) * 10
        nve = lj.NVE(ctx, pos, vel, force, box, ones, ones, rc, nl, 0.005, every, precision,
                     log_rows=warm + steps + 1, batch=batch)
        nve.init()
        if warm:
            nve.run(warm, use_graph=True)
        stale = _sync(ctx)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(ctx.stream)
        nve.run(steps, use_graph=True)
        ev1.record(ctx.stream)
        stale = _sync(ctx) or stale
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        log = nve.log.cpu().numpy().copy()
        nve.free()
        # per-phase device times of eager steps (a fresh integrator, same state)
        nve = lj.NVE(ctx, pos, vel, force, box, ones, ones, rc, nl, 0.005, every, precision,
                     log_rows=0, batch=batch)
        nve.init()
        ctx.profile_begin()
        nve.run(profile_steps, use_graph=False)
        prof = ctx.profile_end()
        stale = _sync(ctx) or stale
        nve.free()
        nl.free()
    if log.ndim == 2:
        log = log[:, None, :]
    timed = log[warm + 1:]
    pairs = float(timed[:, :, 4].sum(axis=1).mean())
    between = timed[:, :, 5] == 0.0
    res = {"ms_per_step": round(ms / steps, 4),
           "pairs_per_s": round(pairs / (ms / steps * 1e-3), 1),
           "phase_us_per_step": {k: round(v[0] * 1e3 / profile_steps, 3)
                                 for k, v in prof.items()},
           "energy_drift_per_1000_steps": _drift(log, 0.005),
           "list_entries": int(entries),
           "rebuilds": int(timed[:, 0, 5].sum()),
           "max_displacement_between_builds": float(timed[:, :, 3].max()),
           "list_stale": bool(stale)}
    res["force_pairs_per_s"] = round(pairs / (res["phase_us_per_step"]["force"] * 1e-6), 1)
    return res


def _drift(log, dt, e_index=None):
    """Total-energy drift per 1,000 steps: slope of a linear fit of
    (E(t) - E(0)) / |E(0)| against the step number, times 1,000."""
    et = log[..., 0] + log[..., 1]
    if et.ndim == 2:
        et = et.sum(axis=1)
    x = np.arange(et.shape[0], dtype=np.float64)
    y = (et - et[0]) / abs(et[0])
    return float(np.polyfit(x, y, 1)[0] * 1000.0)


def bench_lj4m(steps: int = 100, warmup: int = 10, variants: bool = True) -> dict:
    """The 4,000,000-atom fluid (100^3 FCC cells, rho = 0.85, Maxwell T = 1.0,
    rc = 2.5, skin 0.3, dt = 0.005), 100 velocity-Verlet steps in HIP-graph
    cycles, full list: FP64 and mixed with the configured rebuild every 10
    steps (whether the list went stale is reported); with `variants` also
    FP64 with the displacement rule (rebuild_every = 0: the list stays
    exact), with the kicks in separate kernels instead of folded into the
    force pass, and with (x, y, z, pad, vx, vy, vz, pad) records."""
    import torch
    s = synth.lj4m()
    ctx = lj.Context(0, stream=torch.cuda.Stream())
    out = {}
    runs = [("fp64", lj.LJ_FP64, 10, lj.LJ_AOS4, 0), ("mixed", lj.LJ_MIXED, 10, lj.LJ_AOS4, 0)]
    if variants:
        runs += [("fp64_displacement_rule", lj.LJ_FP64, 0, lj.LJ_AOS4, 0),
                 ("fp64_separate_kicks", lj.LJ_FP64, 10, lj.LJ_AOS4, 2),
                 ("fp64_aos8_records", lj.LJ_FP64, 10, lj.LJ_AOS8, 0)]
    for name, prec, every, layout, kick in runs:
        ctx.tune_set(lj.LJ_TUNE_KICK, kick)
        out[name] = nve_measure(ctx, s.pos, s.vel, s.box, s.rc, steps, prec, every, layout,
                                warmup=warmup)
        ctx.tune_set(lj.LJ_TUNE_KICK, 0)
        _note(f"lj4m: {name} done")
    f64 = out["fp64"]
    force_bytes = s.n * (32 + 32 + 8) + 4 * f64["list_entries"]
    fus = f64["phase_us_per_step"]["force"]
    out["force_roofline"] = {"kernel": "k_force (FP64, full list, kicks folded in)",
                             "bound": "hbm", "bytes_per_launch": force_bytes,
                             "us_per_launch": fus,
                             "achieved": round(force_bytes / (fus * 1e-6) / 1e9, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(force_bytes / (fus * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    out["mixed_speedup_force"] = round(fus / out["mixed"]["phase_us_per_step"]["force"], 3)
    out["mixed_speedup_step"] = round(f64["ms_per_step"] / out["mixed"]["ms_per_step"], 3)
    out["workload"] = ("FP64 and mixed LJ fluid, 4,000,000 atoms (100^3 FCC x4), rho=0.85, "
                       "Maxwell T=1.0, rc=2.5, skin=0.3, dt=0.005, velocity-Verlet steps in "
                       f"HIP-graph cycles of 10, {steps} steps timed after "
                       f"{-(-max(warmup, 0) // 10) * 10} untimed")
    ctx.close()
    return out


def bench_batch512(steps: int = 100, warmup: int = 10, tune: bool = False) -> dict:
    """512 independent systems (about 4.3M atoms): 100 NVE steps in HIP-graph
    cycles with one launch per phase for every system, FP64 and mixed, launch
    shapes from the autotuner's cache (or tuned here with tune=True); the
    batching gain of one batched force launch over a loop of 512 per-system
    launches."""
    import torch
    dev = torch.device("cuda:0")
    systems = synth.batch512()
    n = np.array([x.n for x in systems])
    box = np.array([x.box for x in systems])
    rc = np.array([x.rc for x in systems])
    ones = np.ones(len(systems))
    pos0 = np.concatenate([x.pos for x in systems])
    vel0 = np.concatenate([x.vel for x in systems])
    ctx = lj.Context(0, stream=torch.cuda.Stream())
    from . import autotune
    key = autotune.batch_key("batch512", lj.LJ_LIST_FULL, lj.LJ_FP64)
    cache = autotune.load_cache()
    tuned = None
    if tune or key not in cache:
        with torch.cuda.stream(ctx.stream):
            p = torch.from_numpy(synth.aos4(pos0)).to(dev)
            torch.cuda.synchronize()
            tuned = autotune.tune_batch(ctx, p, n, box, rc, 0.3, objective="nve_us",
                                        space={"lanes": (4, 8), "build_lanes": (64, 4),
                                               "batch": (2, 4), "cell_div": (2,)}, reps=5)
            del p
        best = tuned["best"]
        cache[key] = best
        if tune:
            autotune.save_cache(cache)
    else:
        best = cache[key]
    autotune.apply(ctx, best)
    _note(f"batch512: launch shapes {best}")
    out = {}
    for name, prec in (("fp64", lj.LJ_FP64), ("mixed", lj.LJ_MIXED)):
        out[name] = nve_measure(ctx, pos0, vel0, box, rc, steps, prec, 10, lj.LJ_AOS4,
                                batch_n=n, lanes=best["lanes"], warmup=warmup)
        _note(f"batch512: {name} done")
    # batching gain: one batched force launch vs one launch per system
    with torch.cuda.stream(ctx.stream):
        pos = torch.from_numpy(synth.aos4(pos0)).to(dev)
        torch.cuda.synchronize()
        nl = lj.lj_build_neighbors_batch(ctx, pos, n, box, rc, 0.3, kind=lj.LJ_LIST_FULL,
                                         lanes=best["lanes"])
        F = torch.empty_like(pos)
        lj.lj_forces_batch(ctx, pos, nl, ones, ones, rc, force=F)
        ctx.sync()
        t0 = time.perf_counter()
        for _ in range(10):
            lj.lj_forces_batch(ctx, pos, nl, ones, ones, rc, force=F)
        ctx.sync()
        t_batched = (time.perf_counter() - t0) / 10
        nl.free()
        off = np.concatenate([[0], np.cumsum(n)])
        singles = []
        for k, x in enumerate(systems):
            p = pos[off[k]:off[k + 1]].contiguous()
            singles.append((p, lj.lj_build_neighbors(ctx, p, x.box, x.rc, 0.3,
                                                     kind=lj.LJ_LIST_FULL,
                                                     lanes=best["lanes"]), x))
        outs = [(torch.empty_like(p), torch.empty(2, dtype=torch.float64, device=dev))
                for p, _, _ in singles]
        ctx.sync()
        t0 = time.perf_counter()
        for _ in range(3):
            for (p, l1, x), (f1, o1) in zip(singles, outs):
                lj.lj_forces(ctx, p, x.box, 1.0, 1.0, x.rc, l1, lj.LJ_FP64, f1, o1)
        ctx.sync()
        t_loop = (time.perf_counter() - t0) / 3
        for _, l1, _ in singles:
            l1.free()
    ctx.close()
    res = {"workload": "512 independent LJ systems, N ~ U{256..16384} (total "
                       f"{int(n.sum())} atoms), rho ~ U[0.7, 1.1], rc ~ U[2.5, 3.0], skin 0.3, "
                       "jittered FCC, T=1.0; one launch per phase for all systems, NVE in "
                       f"HIP-graph cycles of 10, {steps} steps timed",
           "systems": len(systems), "atoms": int(n.sum()),
           "launch_shapes": best, "launch_shapes_from": "tuned now" if tuned else "cache",
           **out,
           "mixed_speedup_step": round(out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"],
                                       3),
           "force_batched_ms": round(t_batched * 1e3, 3),
           "force_per_system_launch_loop_ms": round(t_loop * 1e3, 3),
           "batching_gain_force": round(t_loop / t_batched, 2)}
    if tuned:
        res["autotune_results"] = tuned["results"]
    return res


def accuracy_lj500k(steps: int = 10000, rebuild_every: int = 0):
    """Mixed-precision accuracy run on the 500,000-atom fluid (rho = 1.0,
    T = 0.7, rc = 3.0, skin = 0.3, dt = 0.005), FP64 and mixed trajectories
    from the same initial state.

    rebuild_every = 0 (the default) rebuilds the list when some atom has moved
    more than skin/2 since the last build, so both trajectories use exact
    lists.  Per step of the mixed trajectory, the FP64 kernel re-evaluates the forces
    on the same positions with the same list; the error is
    max_i |F_mixed_i - F_fp64_i| / max_i |F_fp64_i| (norms per component).
    Step 0 is the perfect lattice, where every force vanishes by symmetry and
    both kernels return rounding residues, so the relative statistics cover
    steps 1..N and step 0 is reported as absolute values.  Energy drift per
    1,000 steps is the slope of a linear fit of (E_tot(t) - E_tot(0)) /
    |E_tot(0)| for each trajectory."""
    import torch
    dev = torch.device("cuda:0")
    s = synth.lj500k()
    ctx = lj.Context(0, stream=torch.cuda.Stream())
    res = {}
    with torch.cuda.stream(ctx.stream):
        for prec_name, prec in (("fp64", lj.LJ_FP64), ("mixed", lj.LJ_MIXED)):
            pos = torch.from_numpy(synth.aos4(s.pos)).to(dev)
            vel = torch.from_numpy(synth.aos4(s.vel)).to(dev)
            force = torch.zeros_like(pos)
            nl = lj.lj_build_neighbors(ctx, pos, s.box, s.rc, s.skin, kind=lj.LJ_LIST_FULL)
            nve = lj.NVE(ctx, pos, vel, force, s.box, 1.0, 1.0, s.rc, nl, 0.005, rebuild_every,
                         prec, log_rows=steps + 1)
            nve.init()
            t0 = time.perf_counter()
            if prec == lj.LJ_FP64:
                nve.run(steps, use_graph=True)
                _sync(ctx)
            else:
                f64 = torch.empty_like(pos)
                out = torch.empty(2, dtype=torch.float64, device=dev)
                err = torch.empty(steps + 1, dtype=torch.float64, device=dev)
                fmax = torch.empty(steps + 1, dtype=torch.float64, device=dev)
                e_f = torch.empty(steps + 1, dtype=torch.float64, device=dev)
                for k in range(steps + 1):
                    if k:
                        nve.run(1, use_graph=False)
                    if k % 1000 == 0:
                        _note(f"accuracy: mixed step {k}")
                    lj.lj_forces(ctx, pos, s.box, 1.0, 1.0, s.rc, nl, lj.LJ_FP64, f64, out)
                    err[k] = (force[:, :3] - f64[:, :3]).abs().amax()
                    fmax[k] = f64[:, :3].abs().amax()
                    e_f[k] = out[0]
                _sync(ctx)
            wall = time.perf_counter() - t0
            log = nve.log.cpu().numpy().copy()
            nve.free()
            nl.free()
            _note(f"accuracy: {prec_name} trajectory done in {wall:.1f} s")
            r = {"wall_s": round(wall, 2),
                 "energy_drift_per_1000_steps": _drift(log, 0.005),
                 "E0": float(log[0, 0] + log[0, 1]),
                 "E_end": float(log[-1, 0] + log[-1, 1]),
                 "max_abs_rel_dE": float(np.max(np.abs((log[:, 0] + log[:, 1]) /
                                                       (log[0, 0] + log[0, 1]) - 1.0))),
                 "T_end": float(2.0 * log[-1, 1] / (3 * s.n - 3)),
                 "rebuilds": int(log[1:, 5].sum()),
                 "max_displacement_between_builds": float(log[:, 3].max())}
            if prec == lj.LJ_MIXED:
                d = err.cpu().numpy()
                fm = fmax.cpu().numpy()
                e = d[1:] / fm[1:]
                pe_mixed = log[:, 0]
                pe_f64 = e_f.cpu().numpy()
                r.update({"force_rel_err_max": float(e.max()),
                          "force_rel_err_mean": float(e.mean()),
                          "force_rel_err_p99": float(np.quantile(e, 0.99)),
                          "force_rel_err_argmax_step": int(e.argmax()) + 1,
                          "step0_abs_err": float(d[0]), "step0_max_abs_f64": float(fm[0]),
                          "max_abs_f64_min_over_steps": float(fm[1:].min()),
                          "pe_rel_err_max": float(np.max(np.abs(pe_mixed / pe_f64 - 1.0)))})
            res[prec_name] = r
    rule = (f"list rebuilt every {rebuild_every} steps" if rebuild_every else
            "list rebuilt when an atom has moved more than skin/2 since the last build")
    return {"workload": "mixed-precision accuracy run: 500,000 atoms (50^3 FCC x4), rho=1.0, "
                        f"Maxwell T=0.7, rc=3.0, skin=0.3, dt=0.005, {rule}, {steps} "
                        "velocity-Verlet steps, full list",
            "atoms": s.n, "steps": steps, **res}
