"""CPU oracle for the oMAP maze planner -- TEST INFRASTRUCTURE ONLY.

Plain loops in C (``oracle.c``) restating the paper's network and path
reconstruction.  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package; the GPU library never
uses it.

Every function returns numpy arrays:
  layers(occ, sources, L)        literal network output A_L (int64) and L used
  bfs(occ, sources)              8-neighbour BFS step distances (int32, -1 = none)
  activity_from_bfs(dist, L)     closed form max(0, L+1-d) (int64)
  walk(O, sources, targets)      simple path reconstruction -> (len, offsets, cells)
  walk_euclidean(O, sources, targets)  Euclidean path reconstruction
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O3 for x86-64-v3, i.e. AVX2, which every
    host of this build has; OpenMP over rows for the timed runs)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _rc(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1, 2))


class Oracle:
    """ctypes view of one build of oracle.c (the default build, or a test's
    deliberately altered copy)."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.oracle_layers.argtypes = [i32, i32, P, P, i32, i64, P, i32]
        L.oracle_layers.restype = i64
        L.oracle_bfs.argtypes = [i32, i32, P, P, i32, P]
        L.oracle_bfs.restype = i64
        L.oracle_activity_from_bfs.argtypes = [i64, P, i64, P]
        L.oracle_activity_from_bfs.restype = None
        for fn in (L.oracle_walk, L.oracle_walk_euclidean):
            fn.argtypes = [i32, i32, P, P, i32, P, i32, P, P, P, i64]
            fn.restype = i64
        L.oracle_walk_random.argtypes = [i32, i32, P, P, i32, P, i32, ctypes.c_uint64, P, P, P, i64]
        L.oracle_walk_random.restype = i64
        L.oracle_tie_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_tie_hash.restype = ctypes.c_uint64
        self.lib = L
        self.path = path

    def layers(self, occ, sources, L: int, threads: int = 1):
        """Output of the L-layer network (L < 0: run-time determination of L).
        Returns (A int64 (H, W), layers_used)."""
        occ = np.ascontiguousarray(occ, dtype=np.uint8)
        H, W = occ.shape
        src = _rc(sources)
        out = np.empty((H, W), dtype=np.int64)
        n = self.lib.oracle_layers(H, W, _p(occ), _p(src), len(src), int(L), _p(out), int(threads))
        if n < 0:
            raise MemoryError("oracle_layers: allocation failed")
        return out, int(n)

    def bfs(self, occ, sources):
        """Multi-source 8-neighbour BFS. Returns (dist int32 (H, W), eccentricity)."""
        occ = np.ascontiguousarray(occ, dtype=np.uint8)
        H, W = occ.shape
        src = _rc(sources)
        dist = np.empty((H, W), dtype=np.int32)
        ecc = self.lib.oracle_bfs(H, W, _p(occ), _p(src), len(src), _p(dist))
        if ecc < 0:
            raise MemoryError("oracle_bfs: allocation failed")
        return dist, int(ecc)

    def activity_from_bfs(self, dist, L: int):
        dist = np.ascontiguousarray(dist, dtype=np.int32)
        out = np.empty(dist.shape, dtype=np.int64)
        self.lib.oracle_activity_from_bfs(dist.size, _p(dist), int(L), _p(out))
        return out

    def _walk(self, fn, O, sources, targets, capacity=None):
        O = np.ascontiguousarray(O, dtype=np.int64)
        H, W = O.shape
        src = _rc(sources)
        tgt = _rc(targets)
        nt = len(tgt)
        if capacity is None:
            capacity = int(nt * (H + W) * 4 + 16)
        while True:
            ln = np.empty(nt, dtype=np.int32)
            off = np.empty(nt + 1, dtype=np.int64)
            cells = np.empty(max(capacity, 1), dtype=np.int32)
            tot = fn(H, W, _p(O), _p(src), len(src), _p(tgt), nt, _p(ln), _p(off), _p(cells),
                     capacity)
            if tot == -1:
                capacity *= 4
                continue
            if tot < 0:
                raise RuntimeError(f"oracle walk failed ({tot})")
            return ln, off, cells[:tot].copy()

    def walk(self, O, sources, targets, capacity=None):
        """Simple path reconstruction on activity map O. Returns (len, offsets, cells)."""
        return self._walk(self.lib.oracle_walk, O, sources, targets, capacity)

    def walk_euclidean(self, O, sources, targets, capacity=None):
        """Euclidean path reconstruction on activity map O. Returns (len, offsets, cells)."""
        return self._walk(self.lib.oracle_walk_euclidean, O, sources, targets, capacity)

    def walk_random(self, O, sources, targets, seed: int, capacity=None):
        """Simple path reconstruction with seeded random ties. Returns (len, offsets, cells)."""
        fn = lambda H, W, o, s, ns, t, nt, ln, off, cells, cap: self.lib.oracle_walk_random(  # noqa: E731
            H, W, o, s, ns, t, nt, int(seed) & 0xFFFFFFFFFFFFFFFF, ln, off, cells, cap)
        return self._walk(fn, O, sources, targets, capacity)

    def tie_hash(self, seed: int, target: int, step: int) -> int:
        return int(self.lib.oracle_tie_hash(seed & 0xFFFFFFFFFFFFFFFF, target, step))


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(_SO):
            build()
        _default = Oracle(_SO)
    return _default


def layers(occ, sources, L: int, threads: int = 1):
    return default().layers(occ, sources, L, threads)


def bfs(occ, sources):
    return default().bfs(occ, sources)


def activity_from_bfs(dist, L: int):
    return default().activity_from_bfs(dist, L)


def walk(O, sources, targets, capacity=None):
    return default().walk(O, sources, targets, capacity)


def walk_euclidean(O, sources, targets, capacity=None):
    return default().walk_euclidean(O, sources, targets, capacity)


def walk_random(O, sources, targets, seed: int, capacity=None):
    return default().walk_random(O, sources, targets, seed, capacity)
