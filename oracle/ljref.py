"""ctypes wrapper of the CPU oracle (oracle/ljref.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library or its binding.

`build()` compiles libljref.so with gcc -O2 -ffp-contract=off -fopenmp.
`lib()` loads the built library, building it first only if it is absent.
All arrays are numpy float64 / int64 / int32 on the host.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ljref.c")
SO = os.path.join(HERE, "libljref.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wextra"]

_lib = None

# truncation of the potential at rc (oracle/ljref.h)
TRUNC_SHIFT = 0          # V(r) - V(rc): the paper's simple truncation
TRUNC_FORCE_SHIFT = 1    # V(r) - V(rc) + (r - rc) Fc: force and energy vanish at rc

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)


def build(src: str = SRC, out: str = SO, extra=()) -> str:
    """Compile the oracle (or a variant of its source) into a shared library."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, out)
    return out


def _bind(so: str):
    L = ctypes.CDLL(so)
    L.ljref_brute_pairs.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_double, ctypes.c_int64,
                                    _I64, _I32, _I64]
    L.ljref_cell_pairs.argtypes = L.ljref_brute_pairs.argtypes
    L.ljref_forces.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, _I64, _I32, _D, _D, _D, _I64]
    L.ljref_forces_full.argtypes = L.ljref_forces.argtypes
    L.ljref_full_pairs.argtypes = [ctypes.c_int64, _I64, _I32, _I64, _I32]
    L.ljref_set_threads.argtypes = [ctypes.c_int]
    L.ljref_sample.argtypes = [ctypes.c_int64, _D, _D, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                               _I64, _D, _D, _D, _I64, _I32, ctypes.c_int64]
    L.ljref_nve.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                            ctypes.c_int32, ctypes.c_int32, _D, _D]
    for f in (L.ljref_brute_pairs, L.ljref_cell_pairs, L.ljref_forces, L.ljref_forces_full,
              L.ljref_full_pairs, L.ljref_set_threads, L.ljref_sample, L.ljref_nve):
        f.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            build()
        _lib = _bind(SO)
    return _lib


class Oracle:
    """The oracle's calls on numpy arrays; `so` selects a library file
    (the default is the built oracle; tests may load a variant)."""

    def __init__(self, so: Optional[str] = None):
        self.L = lib() if so is None else _bind(so)

    @staticmethod
    def _p(a, t):
        return a.ctypes.data_as(t)

    def _pos(self, pos):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        assert pos.ndim == 2 and pos.shape[1] == 3
        return pos

    def _pairs(self, fn, pos, box, rs) -> Tuple[np.ndarray, np.ndarray]:
        pos = self._pos(pos)
        box = np.ascontiguousarray(box, dtype=np.float64)
        n = pos.shape[0]
        row_ptr = np.zeros(n + 1, dtype=np.int64)
        np_ = ctypes.c_int64(0)
        cap = max(16, int(n * 96))
        col = np.zeros(cap, dtype=np.int32)
        st = fn(n, self._p(pos, _D), self._p(box, _D), rs, cap, self._p(row_ptr, _I64),
                self._p(col, _I32), ctypes.byref(np_))
        if st == -4:
            cap = int(np_.value)
            col = np.zeros(max(cap, 1), dtype=np.int32)
            st = fn(n, self._p(pos, _D), self._p(box, _D), rs, cap, self._p(row_ptr, _I64),
                    self._p(col, _I32), ctypes.byref(np_))
        if st != 0:
            raise RuntimeError(f"oracle pair build failed: status {st}")
        return row_ptr, col[: np_.value].copy()

    def brute_pairs(self, pos, box, rs):
        """Half list (CSR, i < j, rows and columns ascending) by O(N^2) search."""
        return self._pairs(self.L.ljref_brute_pairs, pos, box, rs)

    def cell_pairs(self, pos, box, rs):
        """The same half list via the linked-list cell method + counting sort."""
        return self._pairs(self.L.ljref_cell_pairs, pos, box, rs)

    def forces(self, pos, box, eps, sigma, rc, row_ptr, col, trunc: int = TRUNC_SHIFT):
        """(F (n,3), E, W, n_in) over a half list."""
        return self._forces(self.L.ljref_forces, pos, box, eps, sigma, rc, row_ptr, col, trunc)

    def forces_full(self, pos, box, eps, sigma, rc, row_ptr, col, trunc: int = TRUNC_SHIFT):
        """(F (n,3), E, W, n_in) over a full list (rows independent, OpenMP)."""
        return self._forces(self.L.ljref_forces_full, pos, box, eps, sigma, rc, row_ptr, col,
                            trunc)

    def _forces(self, fn, pos, box, eps, sigma, rc, row_ptr, col, trunc):
        pos = self._pos(pos)
        box = np.ascontiguousarray(box, dtype=np.float64)
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        if col.size == 0:
            col = np.zeros(1, dtype=np.int32)
        n = pos.shape[0]
        F = np.zeros((n, 3), dtype=np.float64)
        E = ctypes.c_double(0.0)
        W = ctypes.c_double(0.0)
        nin = ctypes.c_int64(0)
        st = fn(n, self._p(pos, _D), self._p(box, _D), eps, sigma, rc, int(trunc),
                self._p(row_ptr, _I64), self._p(col, _I32), self._p(F, _D),
                ctypes.byref(E), ctypes.byref(W), ctypes.byref(nin))
        if st != 0:
            raise RuntimeError(f"oracle forces failed: status {st}")
        return F, E.value, W.value, nin.value

    def full_pairs(self, row_ptr, col):
        """The full list (CSR, rows and columns ascending) of a half list."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        n = row_ptr.shape[0] - 1
        frp = np.zeros(n + 1, dtype=np.int64)
        fcol = np.zeros(max(2 * col.size, 1), dtype=np.int32)
        colp = col if col.size else np.zeros(1, dtype=np.int32)
        st = self.L.ljref_full_pairs(n, self._p(row_ptr, _I64), self._p(colp, _I32),
                                     self._p(frp, _I64), self._p(fcol, _I32))
        if st != 0:
            raise RuntimeError(f"oracle full list failed: status {st}")
        return frp, fcol[: 2 * col.size].copy()

    def set_threads(self, nthreads: int = 0) -> int:
        """Threads of the oracle's OpenMP loops (0: leave as is); returns the count."""
        return int(self.L.ljref_set_threads(int(nthreads)))

    def sample(self, pos, box, eps, sigma, rc, rs, idx, rowcap: int = 0,
               trunc: int = TRUNC_SHIFT):
        """Per-atom (F (ns,3), e (ns), w (ns), nrs (ns), rows (ns,rowcap) or None)."""
        pos = self._pos(pos)
        box = np.ascontiguousarray(box, dtype=np.float64)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        ns = idx.shape[0]
        f = np.zeros((ns, 3), dtype=np.float64)
        e = np.zeros(ns, dtype=np.float64)
        w = np.zeros(ns, dtype=np.float64)
        nrs = np.zeros(ns, dtype=np.int64)
        rows = np.full((ns, rowcap), -1, dtype=np.int32) if rowcap > 0 else None
        st = self.L.ljref_sample(pos.shape[0], self._p(pos, _D), self._p(box, _D), eps, sigma,
                                 rc, int(trunc), rs, ns, self._p(idx, _I64), self._p(f, _D),
                                 self._p(e, _D), self._p(w, _D), self._p(nrs, _I64),
                                 self._p(rows, _I32) if rows is not None else None, rowcap)
        if st != 0:
            raise RuntimeError(f"oracle sample failed: status {st}")
        return f, e, w, nrs, rows

    def nve(self, pos, vel, box, eps, sigma, rc, skin, dt, nsteps, rebuild_every,
            trunc: int = TRUNC_SHIFT):
        """Velocity Verlet; returns (pos, vel, force, log (nsteps+1, 6)).
        rebuild_every = 0 rebuilds when a displacement exceeds skin/2."""
        pos = self._pos(pos).copy()
        vel = np.ascontiguousarray(vel, dtype=np.float64).copy()
        box = np.ascontiguousarray(box, dtype=np.float64)
        n = pos.shape[0]
        F = np.zeros((n, 3), dtype=np.float64)
        log = np.zeros((nsteps + 1, 6), dtype=np.float64)
        st = self.L.ljref_nve(n, self._p(pos, _D), self._p(vel, _D), self._p(box, _D), eps, sigma,
                              rc, int(trunc), skin, dt, nsteps, rebuild_every, self._p(log, _D),
                              self._p(F, _D))
        if st != 0:
            raise RuntimeError(f"oracle nve failed: status {st}")
        return pos, vel, F, log


def half_pairs_set(row_ptr: np.ndarray, col: np.ndarray) -> np.ndarray:
    """CSR -> (npairs, 2) int64 array of (i, j), sorted lexicographically."""
    n = row_ptr.shape[0] - 1
    i = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    ij = np.stack([i, col.astype(np.int64)], axis=1)
    key = ij[:, 0] * (n + 1) + ij[:, 1]
    return ij[np.argsort(key, kind="stable")]
