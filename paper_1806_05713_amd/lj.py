"""Python binding of the gfx950 LJ library (include/lj.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Device arrays are torch tensors on a ROCm device; the library reads and
writes them in place through their data pointers, on torch's current stream
(or a stream given to `Context`).  The functions carry the C names.

The binding loads paper_1806_05713_amd/liblj.so and raises ImportError-like
errors if it is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblj.so")

LJ_OK = 0
LJ_E_INVALID, LJ_E_BOX, LJ_E_POSITION, LJ_E_CAPACITY = -1, -2, -3, -4
LJ_E_STALE, LJ_E_NOMEM, LJ_E_HIP, LJ_E_NODEVICE = -5, -6, -7, -8
STATUS_NAMES = {0: "LJ_OK", -1: "LJ_E_INVALID", -2: "LJ_E_BOX", -3: "LJ_E_POSITION",
                -4: "LJ_E_CAPACITY", -5: "LJ_E_STALE", -6: "LJ_E_NOMEM", -7: "LJ_E_HIP",
                -8: "LJ_E_NODEVICE"}
LJ_LIST_HALF, LJ_LIST_FULL = 0, 1
LJ_FP64, LJ_MIXED = 0, 1
LJ_AOS4, LJ_SOA, LJ_AOS8 = 0, 1, 2
LJ_TRUNC_SHIFT, LJ_TRUNC_FORCE_SHIFT = 0, 1
LOG_COLS = 6   # integrator log: PE, KE, W, max displacement, pairs, rebuilt

# every entry point declared in include/lj.h
EXPORTS = ["lj_create", "lj_destroy", "lj_set_stream", "lj_sync", "lj_build_cells",
           "lj_cells_info", "lj_cells_export", "lj_cells_free", "lj_build_neighbors",
           "lj_update_neighbors", "lj_list_info", "lj_list_pairs", "lj_list_free",
           "lj_list_device_view", "lj_forces", "lj_nve_create", "lj_nve_init", "lj_nve_run",
           "lj_nve_steps", "lj_nve_free", "lj_build_neighbors_batch", "lj_forces_batch",
           "lj_list_sys_info", "lj_nve_create_batch",
           "lj_profile_begin", "lj_profile_end", "lj_tune_set", "lj_tune_get", "lj_last_error",
           "lj_forces_noalloc"]
LJ_TUNE_BUILD_LANES, LJ_TUNE_FORCE_BATCH, LJ_TUNE_CELL_DIV, LJ_TUNE_KICK, LJ_TUNE_N = 0, 1, 2, 3, 4
LJ_PROF_CELLS, LJ_PROF_NEIGH, LJ_PROF_FORCE, LJ_PROF_OTHER, LJ_PROF_INTEGRATE = 0, 1, 2, 3, 4
LJ_PROF_N = 5
PROF_PHASES = ("cells", "neigh", "force", "other", "integrate")


class LJError(RuntimeError):
    def __init__(self, status: int, what: str, text: str):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {text}")


class ListView(ctypes.Structure):
    _fields_ = [("col", ctypes.c_void_p), ("row_atom", ctypes.c_void_p),
                ("row_len", ctypes.c_void_p), ("slice_iters", ctypes.c_void_p),
                ("nslices", ctypes.c_int64), ("lanes", ctypes.c_int32), ("cap", ctypes.c_int32)]


class ListDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("kind", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("cap", ctypes.c_int32), ("max_row", ctypes.c_int32),
                ("entries", ctypes.c_int64), ("slots", ctypes.c_int64),
                ("rc", ctypes.c_double), ("skin", ctypes.c_double),
                ("box", ctypes.c_double * 3), ("nc", ctypes.c_int32 * 3), ("nsys", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("tests", ctypes.c_int64)]


_lib = None
_VP = ctypes.c_void_p
_D3 = ctypes.c_double * 3


def load(path: str = LIB_PATH):
    """Load liblj.so and declare the C signatures (no device is touched)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_1806_05713_amd.build`")
    L = ctypes.CDLL(path)
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    PP = ctypes.POINTER(_VP)
    sig = {
        "lj_create": ([ctypes.c_int, _VP, PP]),
        "lj_destroy": ([_VP]),
        "lj_set_stream": ([_VP, _VP]),
        "lj_sync": ([_VP]),
        "lj_build_cells": ([_VP, _VP, i64, i32, _D3, dbl, PP]),
        "lj_cells_info": ([_VP, ctypes.POINTER(i32), ctypes.POINTER(i64)]),
        "lj_cells_export": ([_VP, _VP, _VP, _VP]),
        "lj_cells_free": ([_VP]),
        "lj_build_neighbors": ([_VP, _VP, i64, i32, _D3, dbl, dbl, i32, i32, _VP, PP]),
        "lj_update_neighbors": ([_VP, _VP, i64, i32, ctypes.POINTER(ctypes.c_double), _VP]),
        "lj_list_info": ([_VP, ctypes.POINTER(ListDesc)]),
        "lj_profile_begin": ([_VP]),
        "lj_profile_end": ([_VP, _VP, _VP]),
        "lj_tune_set": ([_VP, i32, i32]),
        "lj_tune_get": ([_VP, i32, ctypes.POINTER(i32)]),
        "lj_list_pairs": ([_VP, _VP, i64, _VP, ctypes.POINTER(i64)]),
        "lj_list_free": ([_VP]),
        "lj_list_device_view": ([_VP, ctypes.POINTER(ListView)]),
        "lj_forces": ([_VP, _VP, i64, i32, _D3, dbl, dbl, dbl, _VP, i32, i32, _VP, _VP, _VP,
                       _VP]),
        "lj_forces_noalloc": ([_VP, _VP, i64, i32, _D3, dbl, dbl, dbl, _VP, i32, i32, _VP, _VP,
                               _VP, _VP]),
        "lj_nve_create": ([_VP, _VP, _VP, _VP, i64, i32, _D3, dbl, dbl, dbl, i32, i32, _VP, dbl,
                           i32, _VP, i64, PP]),
        "lj_nve_create_batch": ([_VP, _VP, _VP, _VP, i32, _VP, _VP, _VP, i32, i32, _VP, dbl,
                                 i32, _VP, i64, PP]),
        "lj_build_neighbors_batch": ([_VP, _VP, i32, i32, _VP, _VP, _VP, dbl, i32, i32, PP]),
        "lj_forces_batch": ([_VP, _VP, i32, _VP, _VP, _VP, _VP, i32, i32, _VP, _VP, _VP, _VP]),
        "lj_list_sys_info": ([_VP, i32, ctypes.POINTER(i64), ctypes.POINTER(i32),
                              ctypes.POINTER(i64), ctypes.POINTER(i32)]),
        "lj_nve_init": ([_VP]),
        "lj_nve_run": ([_VP, i32, i32]),
        "lj_nve_steps": ([_VP, ctypes.POINTER(i64)]),
        "lj_nve_free": ([_VP]),
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.lj_last_error.argtypes = []
    L.lj_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st: int, what: str):
    if st != LJ_OK:
        raise LJError(st, what, load().lj_last_error().decode())


def _box(box) -> ctypes.Array:
    b = np.asarray(box, dtype=np.float64).reshape(3)
    return _D3(*[float(x) for x in b])


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError("expected a tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _pos_layout(pos) -> Tuple[int, int]:
    """(n, layout) from a tensor's shape: (n, 4) -> AOS4, (n, 8) -> AOS8
    (position and velocity records), (3, n) -> SOA."""
    import torch
    if pos.dtype != torch.float64:
        raise TypeError("positions must be float64")
    if pos.dim() == 2 and pos.shape[1] == 4:
        return int(pos.shape[0]), LJ_AOS4
    if pos.dim() == 2 and pos.shape[1] == 8:
        return int(pos.shape[0]), LJ_AOS8
    if pos.dim() == 2 and pos.shape[0] == 3:
        return int(pos.shape[1]), LJ_SOA
    raise ValueError("positions must be (n, 4) [AOS4], (n, 8) [AOS8] or (3, n) [SOA]")


def _force_like(pos, layout):
    """A force array for positions in `layout` (AOS8 positions give AOS4 forces)."""
    import torch
    if layout == LJ_AOS8:
        return torch.empty((pos.shape[0], 4), dtype=pos.dtype, device=pos.device)
    return torch.empty_like(pos)


class Context:
    """lj_create / lj_destroy; binds torch's current stream unless one is given."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        L = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = _VP()
        _check(L.lj_create(device, _VP(stream.cuda_stream), ctypes.byref(h)), "lj_create")
        self.h = h

    def set_stream(self, stream):
        self.stream = stream
        _check(load().lj_set_stream(self.h, _VP(stream.cuda_stream)), "lj_set_stream")

    def sync(self):
        _check(load().lj_sync(self.h), "lj_sync")

    def tune_set(self, knob: int, value: int):
        _check(load().lj_tune_set(self.h, int(knob), int(value)), "lj_tune_set")

    def tune_get(self, knob: int) -> int:
        v = ctypes.c_int32()
        _check(load().lj_tune_get(self.h, int(knob), ctypes.byref(v)), "lj_tune_get")
        return v.value

    def profile_begin(self):
        _check(load().lj_profile_begin(self.h), "lj_profile_begin")

    def profile_end(self):
        """{phase: (ms, launches)} since profile_begin."""
        ms = np.zeros(LJ_PROF_N, dtype=np.float64)
        cnt = np.zeros(LJ_PROF_N, dtype=np.int64)
        _check(load().lj_profile_end(self.h, ms.ctypes.data, cnt.ctypes.data), "lj_profile_end")
        return {name: (float(ms[k]), int(cnt[k])) for k, name in enumerate(PROF_PHASES)}

    def close(self):
        if getattr(self, "h", None):
            load().lj_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cells:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def info(self):
        nc = (ctypes.c_int32 * 3)()
        n = ctypes.c_int64()
        _check(load().lj_cells_info(self.h, nc, ctypes.byref(n)), "lj_cells_info")
        return tuple(nc), n.value

    def export(self):
        nc, n = self.info()
        ncell = nc[0] * nc[1] * nc[2]
        cs = np.zeros(ncell + 1, dtype=np.int32)
        order = np.zeros(n, dtype=np.int32)
        _check(load().lj_cells_export(self.ctx.h, self.h, cs.ctypes.data, order.ctypes.data),
               "lj_cells_export")
        return cs, order

    def free(self):
        if self.h:
            load().lj_cells_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class NeighborList:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def info(self) -> ListDesc:
        d = ListDesc()
        _check(load().lj_list_info(self.h, ctypes.byref(d)), "lj_list_info")
        return d

    def device_view(self) -> ListView:
        v = ListView()
        _check(load().lj_list_device_view(self.h, ctypes.byref(v)), "lj_list_device_view")
        return v

    def sys_info(self, s: int):
        """(n, max_row, entries, cap) of system s."""
        n, mr, e, cap = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(load().lj_list_sys_info(self.h, int(s), ctypes.byref(n), ctypes.byref(mr),
                                       ctypes.byref(e), ctypes.byref(cap)), "lj_list_sys_info")
        return n.value, mr.value, e.value, cap.value

    def pairs(self) -> np.ndarray:
        """(entries, 2) int32 array of the stored (i, j) entries."""
        d = self.info()
        ij = np.zeros((max(d.entries, 1), 2), dtype=np.int32)
        n = ctypes.c_int64()
        _check(load().lj_list_pairs(self.ctx.h, self.h, d.entries, ij.ctypes.data,
                                    ctypes.byref(n)), "lj_list_pairs")
        return ij[: n.value]

    def free(self):
        if self.h:
            load().lj_list_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lj_build_cells(ctx: Context, pos, box, min_cell: float) -> Cells:
    n, layout = _pos_layout(pos)
    h = _VP()
    _check(load().lj_build_cells(ctx.h, _ptr(pos), n, layout, _box(box), float(min_cell),
                                 ctypes.byref(h)), "lj_build_cells")
    return Cells(ctx, h)


def lj_build_neighbors(ctx: Context, pos, box, rc: float, skin: float,
                       kind: int = LJ_LIST_HALF, lanes: int = 0,
                       cells: Optional[Cells] = None) -> NeighborList:
    n, layout = _pos_layout(pos)
    h = _VP()
    _check(load().lj_build_neighbors(ctx.h, _ptr(pos), n, layout, _box(box), float(rc),
                                     float(skin), int(kind), int(lanes),
                                     cells.h if cells is not None else None, ctypes.byref(h)),
           "lj_build_neighbors")
    return NeighborList(ctx, h)


def lj_update_neighbors(ctx: Context, pos, box, nlist: NeighborList) -> NeighborList:
    """Rebuild nlist in place for new positions (asynchronous).  box may be
    None for a batch list (each system keeps its own box)."""
    n, layout = _pos_layout(pos)
    _check(load().lj_update_neighbors(ctx.h, _ptr(pos), n, layout,
                                      None if box is None else _box(box), nlist.h),
           "lj_update_neighbors")
    return nlist


def lj_forces(ctx: Context, pos, box, eps: float, sigma: float, rc: float,
              nlist: NeighborList, precision: int = LJ_FP64, force=None, out=None,
              trunc: int = LJ_TRUNC_SHIFT):
    """Launch the force kernel (asynchronous).  force: tensor shaped like pos
    ((n, 4) for AOS8 positions; allocated if None); out: float64 device tensor
    of 2 receiving energy and virial (allocated if None).  Returns (force,
    energy, virial, npairs) as device tensors."""
    import torch
    n, layout = _pos_layout(pos)
    if force is None:
        force = _force_like(pos, layout)
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=pos.device)
    cnt = torch.empty(1, dtype=torch.int64, device=pos.device)
    _check(load().lj_forces(ctx.h, _ptr(pos), n, layout, _box(box), float(eps), float(sigma),
                            float(rc), nlist.h, int(precision), int(trunc), _ptr(force),
                            _ptr(out), out.data_ptr() + 8, _ptr(cnt)), "lj_forces")
    return force, out[0:1], out[1:2], cnt


def lj_forces_noalloc(ctx: Context, pos, box, eps: float, sigma: float, rc: float,
                      nlist: NeighborList, precision: int, force, energy, virial, npairs,
                      trunc: int = LJ_TRUNC_SHIFT):
    """lj_forces with the library's static block partials: every output is a
    caller-allocated device tensor (force like pos, energy / virial float64
    of 1, npairs int64 of 1); nothing is allocated here."""
    n, layout = _pos_layout(pos)
    _check(load().lj_forces_noalloc(ctx.h, _ptr(pos), n, layout, _box(box), float(eps),
                                    float(sigma), float(rc), nlist.h, int(precision), int(trunc),
                                    _ptr(force), _ptr(energy), _ptr(virial), _ptr(npairs)),
           "lj_forces_noalloc")


def _harr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _pos_layout_total(pos) -> Tuple[int, int]:
    return _pos_layout(pos)


def lj_build_neighbors_batch(ctx: Context, pos, n, box, rc, skin: float,
                             kind: int = LJ_LIST_FULL, lanes: int = 0) -> NeighborList:
    """Batch list: n[s] atoms per system, box (nsys, 3), rc (nsys,), concatenated pos."""
    _, layout = _pos_layout(pos)
    n = _harr(n, np.int64)
    box = _harr(box, np.float64).reshape(-1, 3)
    rc = _harr(rc, np.float64)
    h = _VP()
    _check(load().lj_build_neighbors_batch(ctx.h, _ptr(pos), layout, int(n.size), n.ctypes.data,
                                           box.ctypes.data, rc.ctypes.data, float(skin),
                                           int(kind), int(lanes), ctypes.byref(h)),
           "lj_build_neighbors_batch")
    nl = NeighborList(ctx, h)
    nl._keep = (n, box, rc)
    return nl


def lj_forces_batch(ctx: Context, pos, nlist: NeighborList, eps, sigma, rc,
                    precision: int = LJ_FP64, force=None, trunc: int = LJ_TRUNC_SHIFT):
    """(force, energy[nsys], virial[nsys], npairs[nsys]) as device tensors."""
    import torch
    _, layout = _pos_layout(pos)
    eps, sigma, rc = _harr(eps, np.float64), _harr(sigma, np.float64), _harr(rc, np.float64)
    ns = int(eps.size)
    if force is None:
        force = _force_like(pos, layout)
    e = torch.empty(ns, dtype=torch.float64, device=pos.device)
    w = torch.empty(ns, dtype=torch.float64, device=pos.device)
    c = torch.empty(ns, dtype=torch.int64, device=pos.device)
    _check(load().lj_forces_batch(ctx.h, _ptr(pos), layout, nlist.h, eps.ctypes.data,
                                  sigma.ctypes.data, rc.ctypes.data, int(precision), int(trunc),
                                  _ptr(force), _ptr(e), _ptr(w), _ptr(c)), "lj_forces_batch")
    return force, e, w, c


class NVE:
    """Velocity-Verlet integrator bound to device arrays pos, vel, force (same
    layout; with (n, 8) AOS8 position-velocity records vel is ignored: the
    velocities are the second half of each record, and force is (n, 4)) and a
    device log of log_rows x 6 doubles (lj_nve_create).  rebuild_every = 0
    rebuilds the list when an atom has moved more than skin/2."""

    def __init__(self, ctx: Context, pos, vel, force, box, eps, sigma, rc,
                 nlist: NeighborList, dt: float, rebuild_every: int = 10,
                 precision: int = LJ_FP64, log_rows: int = 0, batch: bool = False,
                 trunc: int = LJ_TRUNC_SHIFT):
        """Single system: box (3,), scalar eps, sigma, rc; log (log_rows, 6).
        batch=True: per-system arrays eps, sigma, rc; log (log_rows, nsys, 6)."""
        import torch
        n, layout = _pos_layout(pos)
        if layout == LJ_AOS8:
            if force.shape != (n, 4) or force.dtype != pos.dtype:
                raise ValueError("AOS8 records need an (n, 4) float64 force array")
            vel_ptr = pos.data_ptr() + 32
        else:
            for t in (vel, force):
                if t.shape != pos.shape or t.dtype != pos.dtype:
                    raise ValueError("vel and force must match pos in shape and dtype")
            vel_ptr = _ptr(vel)
        self.ctx, self.pos, self.vel, self.force, self.nlist = ctx, pos, vel, force, nlist
        h = _VP()
        if batch:
            eps, sigma, rc = _harr(eps, np.float64), _harr(sigma, np.float64), _harr(rc, np.float64)
            ns = int(eps.size)
            self.log = torch.zeros((max(log_rows, 1), ns, LOG_COLS), dtype=torch.float64,
                                   device=pos.device)
            _check(load().lj_nve_create_batch(ctx.h, _ptr(pos), vel_ptr, _ptr(force), layout,
                                              eps.ctypes.data, sigma.ctypes.data, rc.ctypes.data,
                                              int(precision), int(trunc), nlist.h, float(dt),
                                              int(rebuild_every), _ptr(self.log), int(log_rows),
                                              ctypes.byref(h)), "lj_nve_create_batch")
        else:
            self.log = torch.zeros((max(log_rows, 1), LOG_COLS), dtype=torch.float64,
                                   device=pos.device)
            _check(load().lj_nve_create(ctx.h, _ptr(pos), vel_ptr, _ptr(force), n, layout,
                                        _box(box), float(eps), float(sigma), float(rc),
                                        int(precision), int(trunc), nlist.h, float(dt),
                                        int(rebuild_every), _ptr(self.log), int(log_rows),
                                        ctypes.byref(h)), "lj_nve_create")
        self.h = h

    def init(self):
        _check(load().lj_nve_init(self.h), "lj_nve_init")

    def run(self, nsteps: int, use_graph: bool = False):
        _check(load().lj_nve_run(self.h, int(nsteps), int(bool(use_graph))), "lj_nve_run")

    @property
    def steps(self) -> int:
        v = ctypes.c_int64()
        _check(load().lj_nve_steps(self.h, ctypes.byref(v)), "lj_nve_steps")
        return v.value

    def free(self):
        if getattr(self, "h", None):
            load().lj_nve_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lj_last_error() -> str:
    return load().lj_last_error().decode()
