"""Autotuner for the launch shapes of the LJ library.

The knobs change speed only -- every setting yields the same list (as a set)
and the same forces -- so tuning is a search over timings:
  lanes        lanes of a 64-wide wavefront per row of the list layout (force kernel)
  build_lanes  lanes per row in the list-build kernel (LJ_TUNE_BUILD_LANES)
  batch        list entries each lane keeps in flight in the force kernel
               (LJ_TUNE_FORCE_BATCH)
  cell_div     list-build cells of side (rc + skin) / cell_div (LJ_TUNE_CELL_DIV)

Each candidate is timed with the library's own HIP-event profiler on the
context's stream (device time of the list-build and force kernels) and
ranked by one objective: build_us, force_us, step_us (a rebuild and a force
evaluation, the default) or nve_us (the force evaluation plus a tenth of the
rebuild: a step of the integrator at its default rebuild cadence).  Results
are cached as JSON keyed by device name, CU count, atom-count bucket,
density, search length, list kind and precision.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from typing import Dict, Iterable, Optional

from . import lj

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")

SPACE = {
    "lanes": (4, 8, 16),
    "build_lanes": (64, 4, 2),
    "batch": (2, 4, 8),
    "cell_div": (1, 2, 3),
}


def key(device_name: str, cus: int, n: int, rho: float, rs: float, kind: int,
        precision: int) -> str:
    nb = int(round(math.log2(max(n, 1))))
    return f"{device_name}/{cus}cu/n2^{nb}/rho{rho:.2f}/rs{rs:.2f}/k{kind}/p{precision}"


def device_tag() -> str:
    """Architecture and compute-unit count of cuda:0 (part of every cache key)."""
    import torch
    props = torch.cuda.get_device_properties(0)
    name = getattr(props, "gcnArchName", props.name).split(":")[0]
    return f"{name}/{props.multi_processor_count}cu"


def system_key(n: int, rho: float, rs: float, kind: int, precision: int) -> str:
    arch, cus = device_tag().split("/")
    return key(arch, int(cus[:-2]), n, rho, rs, kind, precision)


def batch_key(name: str, kind: int, precision: int) -> str:
    """Cache key of a named batch workload."""
    return f"{device_tag()}/batch:{name}/k{kind}/p{precision}"


def cached(k: str, path: str = CACHE) -> Optional[dict]:
    """The cached configuration under key k, or None."""
    return load_cache(path).get(k)


def load_cache(path: str = CACHE) -> Dict[str, dict]:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(cache: Dict[str, dict], path: str = CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(ctx: "lj.Context", cfg: dict) -> None:
    ctx.tune_set(lj.LJ_TUNE_BUILD_LANES, cfg.get("build_lanes", 0))
    ctx.tune_set(lj.LJ_TUNE_FORCE_BATCH, cfg.get("batch", 0))
    ctx.tune_set(lj.LJ_TUNE_CELL_DIV, cfg.get("cell_div", 0))


# An NVE step of the library's integrator rebuilds the list every
# NVE_REBUILD_EVERY steps (its default cadence).
NVE_REBUILD_EVERY = 10


def timings(per: dict) -> dict:
    """Objectives from per-phase device times (us): build_us (cells + list),
    force_us, step_us (one rebuild and one force evaluation) and nve_us (an
    integrator step: the force evaluation plus the rebuild's share)."""
    build = per["cells"] + per["neigh"]
    force = per["force"] + per["other"]
    return {"build_us": build, "force_us": per["force"],
            "step_us": build + force,
            "nve_us": force + build / NVE_REBUILD_EVERY}


def measure(ctx, pos, box, rc, skin, kind, precision, cfg, reps: int = 20) -> dict:
    """Device time (us) of one list rebuild and one force evaluation with cfg."""
    import torch
    apply(ctx, cfg)
    nl = lj.lj_build_neighbors(ctx, pos, box, rc, skin, kind=kind, lanes=cfg["lanes"])
    force = torch.empty_like(pos)
    out = torch.empty(2, dtype=torch.float64, device=pos.device)
    for _ in range(3):
        lj.lj_update_neighbors(ctx, pos, box, nl)
        lj.lj_forces(ctx, pos, box, 1.0, 1.0, rc, nl, precision, force, out)
    ctx.profile_begin()
    for _ in range(reps):
        lj.lj_update_neighbors(ctx, pos, box, nl)
        lj.lj_forces(ctx, pos, box, 1.0, 1.0, rc, nl, precision, force, out)
    prof = ctx.profile_end()
    ctx.sync()
    nl.free()
    per = {k: v[0] * 1e3 / max(v[1], 1) for k, v in prof.items()}
    return timings(per)


def tune(ctx, pos, box, rc, skin, kind=lj.LJ_LIST_FULL, precision=lj.LJ_FP64,
         objective: str = "step_us", space: Optional[dict] = None, reps: int = 20,
         log=None) -> dict:
    """Search `space` (default SPACE); returns {"best": cfg, "results": [...]}."""
    space = dict(SPACE if space is None else space)
    results = []
    names = list(space)
    for vals in itertools.product(*(space[k] for k in names)):
        cfg = dict(zip(names, vals))
        if cfg["build_lanes"] != 64 and cfg["build_lanes"] > cfg["lanes"]:
            continue
        t = measure(ctx, pos, box, rc, skin, kind, precision, cfg, reps)
        results.append({**cfg, **t})
        if log:
            log(json.dumps(results[-1]))
    best = min(results, key=lambda r: r[objective])
    return {"best": {k: best[k] for k in names}, "objective": objective, "results": results}


def measure_batch(ctx, pos, n, box, rc, skin, kind, precision, cfg, reps: int = 10) -> dict:
    """Device time (us) of one batched list rebuild and one batched force
    evaluation with cfg (eps = sigma = 1 for every system)."""
    import numpy as np
    import torch
    apply(ctx, cfg)
    nl = lj.lj_build_neighbors_batch(ctx, pos, n, box, rc, skin, kind=kind, lanes=cfg["lanes"])
    ones = np.ones(len(n))
    force = torch.empty_like(pos)
    for _ in range(2):
        lj.lj_update_neighbors(ctx, pos, None, nl)
        lj.lj_forces_batch(ctx, pos, nl, ones, ones, rc, precision, force)
    ctx.profile_begin()
    for _ in range(reps):
        lj.lj_update_neighbors(ctx, pos, None, nl)
        lj.lj_forces_batch(ctx, pos, nl, ones, ones, rc, precision, force)
    prof = ctx.profile_end()
    ctx.sync()
    nl.free()
    per = {k: v[0] * 1e3 / max(v[1], 1) for k, v in prof.items()}
    return timings(per)


def tune_batch(ctx, pos, n, box, rc, skin, kind=lj.LJ_LIST_FULL, precision=lj.LJ_FP64,
               objective: str = "step_us", space: Optional[dict] = None, reps: int = 10,
               log=None) -> dict:
    """tune() for a batch of systems (lj_build_neighbors_batch / lj_forces_batch)."""
    space = dict(SPACE if space is None else space)
    results = []
    names = list(space)
    for vals in itertools.product(*(space[k] for k in names)):
        cfg = dict(zip(names, vals))
        if cfg.get("build_lanes", 1) != 64 and cfg.get("build_lanes", 1) > cfg["lanes"]:
            continue
        t = measure_batch(ctx, pos, n, box, rc, skin, kind, precision, cfg, reps)
        results.append({**cfg, **t})
        if log:
            log(json.dumps(results[-1]))
    best = min(results, key=lambda r: r[objective])
    return {"best": {k: best[k] for k in names}, "objective": objective, "results": results}


def best_config(ctx, pos, box, rc, skin, kind, precision, rho: float,
                objective: str = "force_us", space: Optional[dict] = None,
                cache_path: str = CACHE, retune: bool = False, log=None) -> dict:
    """Cached tuned configuration for this device and workload shape (tuned
    and cached when missing or when retune is set)."""
    n = int(pos.shape[0] if pos.dim() == 2 and pos.shape[1] in (4, 8) else pos.shape[1])
    k = system_key(n, rho, rc + skin, kind, precision)
    cache = load_cache(cache_path)
    if k in cache and not retune:
        return cache[k]
    res = tune(ctx, pos, box, rc, skin, kind, precision, objective=objective, space=space,
               log=log)
    cache[k] = res["best"]
    save_cache(cache, cache_path)
    return res["best"]
