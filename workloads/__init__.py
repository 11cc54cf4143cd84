"""Seeded synthetic workloads for the oMAP maze planner.

Input preparation only: occupancy grids, source lists and target lists.  No
activity, distance or path arithmetic lives here, so this module can feed both
the CPU oracle and the GPU library without tying them together.

The five workload families follow the configurations the paper's method is
measured on here (the paper's own maps are not available, so seeded synthetic
mazes of the same kind stand in for them):

  config1  64x64, Bernoulli(0.30) obstacles, 1 source, 4 reachable targets
  config2  4096x4096 randomised-DFS maze + 2% extra wall removals, 1 source,
           256 targets
  config3  23170x23170, Bernoulli(0.40) + 50,000 filled rectangles (sides
           U{2..200}), 16 sources + 4096 targets on the largest 8-connected
           free component
  config4  512 mazes, sides log-uniform in [128, 2048], Bernoulli(p),
           p ~ U[0.2, 0.45], 1-8 sources, 16-512 targets (largest component)
  serve_query(i)  side log-uniform in [256, 8192], DFS (2% removals) or
           Bernoulli(0.35) by a fair coin, 1-16 sources, 8-2048 targets

Occupancy: uint8 (H, W), 1 = obstacle.  Coordinates: int32 (n, 2) arrays of
(row, col).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libomapgen.so")
_SRC = os.path.join(_HERE, "gen.c")

# stream tags: one independent random stream per purpose
S_OBST, S_RECT, S_SRC, S_TGT, S_DFS, S_PARAM, S_ARRIVAL = 1, 2, 3, 4, 5, 6, 7


def build(force: bool = False) -> str:
    """Compile gen.c into libomapgen.so (gcc, -O2)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.gen_uniform.argtypes = [u64, u64, i64, P]
        L.gen_below.argtypes = [u64, u64, u64, i64, P]
        L.gen_bernoulli.argtypes = [i32, i32, f64, u64, u64, P]
        L.gen_rectangles.argtypes = [i32, i32, i32, i32, i32, u64, u64, P]
        L.gen_dfs_maze.argtypes = [i32, i32, f64, u64, u64, P]
        L.gen_dfs_maze.restype = i64
        L.gen_components.argtypes = [i32, i32, P, P, P, P]
        L.gen_components.restype = i64
        L.gen_sample_cells.argtypes = [i32, i32, P, i32, i32, i32, i64, u64, u64, P]
        L.gen_sample_cells.restype = i32
        L.gen_fnv1a.argtypes = [P, i64]
        L.gen_fnv1a.restype = u64
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---- primitive generators ---------------------------------------------------

def uniform(seed: int, stream: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().gen_uniform(seed, stream, n, _ptr(out))
    return out


def below(seed: int, stream: int, bound: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    lib().gen_below(seed, stream, bound, n, _ptr(out))
    return out


def bernoulli(H: int, W: int, p: float, seed: int, stream: int = S_OBST) -> np.ndarray:
    occ = np.empty((H, W), dtype=np.uint8)
    lib().gen_bernoulli(H, W, p, seed, stream, _ptr(occ))
    return occ


def add_rectangles(occ: np.ndarray, n: int, side_min: int, side_max: int, seed: int,
                   stream: int = S_RECT) -> np.ndarray:
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous
    H, W = occ.shape
    lib().gen_rectangles(H, W, n, side_min, side_max, seed, stream, _ptr(occ))
    return occ


def dfs_maze(H: int, W: int, removal_frac: float, seed: int, stream: int = S_DFS):
    """Returns (occ, n_removed)."""
    occ = np.empty((H, W), dtype=np.uint8)
    m = lib().gen_dfs_maze(H, W, removal_frac, seed, stream, _ptr(occ))
    if m < 0:
        raise MemoryError("gen_dfs_maze: allocation failed")
    return occ, int(m)


def components(occ: np.ndarray):
    """8-connected free components: (labels int32, n_components, largest_label, largest_size)."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    H, W = occ.shape
    lab = np.empty((H, W), dtype=np.int32)
    ll = ctypes.c_int32(0)
    ls = ctypes.c_int64(0)
    n = lib().gen_components(H, W, _ptr(occ), _ptr(lab), ctypes.byref(ll), ctypes.byref(ls))
    if n < 0:
        raise MemoryError("gen_components: allocation failed")
    return lab, int(n), int(ll.value), int(ls.value)


def sample_cells(labels: np.ndarray, want: int, k: int, distinct: bool, population: int,
                 seed: int, stream: int) -> np.ndarray:
    """k cells uniform on {label == want} (want=-2: any free cell), as (k, 2) int32."""
    H, W = labels.shape
    out = np.empty((max(k, 0), 2), dtype=np.int32)
    got = lib().gen_sample_cells(H, W, _ptr(labels), want, k, int(distinct), population,
                                 seed, stream, _ptr(out))
    if got != k:
        raise ValueError(f"sample_cells: population {population} too small for {k} cells")
    return out


def content_hash(*arrays: np.ndarray) -> int:
    h = 0
    for a in arrays:
        a = np.ascontiguousarray(a)
        h ^= int(lib().gen_fnv1a(_ptr(a.view(np.uint8)), a.nbytes))
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


# ---- maze instances -----------------------------------------------------------

@dataclass
class Maze:
    occ: np.ndarray                      # uint8 (H, W), 1 = obstacle
    sources: np.ndarray                  # int32 (s, 2) (row, col)
    targets: np.ndarray                  # int32 (t, 2) (row, col)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def H(self) -> int:
        return int(self.occ.shape[0])

    @property
    def W(self) -> int:
        return int(self.occ.shape[1])


def _on_largest_component(occ, n_src, n_tgt, seed, name, meta=None):
    lab, ncomp, ll, ls = components(occ)
    cells = sample_cells(lab, ll, n_src + n_tgt, True, ls, seed, S_SRC)
    m = dict(meta or {})
    m.update(n_components=ncomp, largest_component=ls)
    return Maze(occ, cells[:n_src].copy(), cells[n_src:].copy(), name, m)


def config1() -> Maze:
    """64x64 Bernoulli(0.30), seed 0; 1 source uniform on free cells; 4 targets
    uniform on free cells, each redrawn until reachable (i.e. uniform on the
    source's component)."""
    seed = 0
    occ = bernoulli(64, 64, 0.30, seed)
    lab, ncomp, ll, ls = components(occ)
    free = int((occ == 0).sum())
    src = sample_cells(lab, -2, 1, True, free, seed, S_SRC)
    comp = int(lab[src[0, 0], src[0, 1]])
    size = int((lab == comp).sum())
    tgt = sample_cells(lab, comp, 4, False, size, seed, S_TGT)
    return Maze(occ, src, tgt, "config1_64x64_bernoulli0.30",
                dict(n_components=ncomp, source_component=size))


def config2(side: int = 4096) -> Maze:
    """side x side randomised-DFS maze on a (side/2)^2 lattice + 2% removals, seed 1;
    1 source and 256 targets uniform on the free cells (all connected)."""
    seed = 1
    occ, removed = dfs_maze(side, side, 0.02, seed)
    lab, ncomp, ll, ls = components(occ)
    src = sample_cells(lab, ll, 1, True, ls, seed, S_SRC)
    tgt = sample_cells(lab, ll, 256, True, ls, seed, S_TGT)
    return Maze(occ, src, tgt, f"config2_{side}x{side}_dfs_maze",
                dict(walls_removed=removed, n_components=ncomp, largest_component=ls))


def config3(side: int = 23170, n_rects: int = 50000) -> Maze:
    """side^2 Bernoulli(0.40) overlaid with n_rects filled rectangles (sides
    U{2..200}), seed 2; 16 sources + 4096 targets, distinct, uniform on the
    largest 8-connected free component."""
    seed = 2
    occ = bernoulli(side, side, 0.40, seed)
    add_rectangles(occ, n_rects, 2, 200, seed)
    return _on_largest_component(occ, 16, 4096, seed, f"config3_{side}x{side}_rect_overlay")


def config4_params(n_mazes: int = 512, seed: int = 3):
    """Per-maze (H, W, p, n_src, n_tgt) for the batched workload."""
    u = uniform(seed, S_PARAM, 5 * n_mazes).reshape(n_mazes, 5)
    lo, hi = math.log(128), math.log(2048)
    out = []
    for i in range(n_mazes):
        H = int(round(math.exp(lo + (hi - lo) * u[i, 0])))
        W = int(round(math.exp(lo + (hi - lo) * u[i, 1])))
        p = 0.2 + 0.25 * u[i, 2]
        ns = 1 + int(u[i, 3] * 8)
        nt = 16 + int(u[i, 4] * 497)
        out.append((H, W, p, ns, nt))
    return out


def config4_maze(i: int, params=None, seed: int = 3) -> Maze:
    params = params or config4_params(seed=seed)
    H, W, p, ns, nt = params[i]
    sub = seed * 1000003 + 17 * i + 1
    occ = bernoulli(H, W, p, sub)
    return _on_largest_component(occ, ns, nt, sub, f"config4_{i}_{H}x{W}_p{p:.3f}", dict(p=p))


def config4(n_mazes: int = 512, seed: int = 3):
    params = config4_params(n_mazes, seed)
    return [config4_maze(i, params, seed) for i in range(n_mazes)]


def serve_query(i: int, seed: int = 4, side_lo: int = 256, side_hi: int = 8192) -> Maze:
    """Query i of the serving stream: square side log-uniform in [side_lo, side_hi],
    DFS maze (2% removals) or Bernoulli(0.35) by a fair coin, 1-16 sources,
    8-2048 targets, on the largest component."""
    u = uniform(seed * 7919 + i, S_PARAM, 4)
    s = int(round(math.exp(math.log(side_lo) + (math.log(side_hi) - math.log(side_lo)) * u[0])))
    sub = seed * 1000003 + 31 * i + 7
    if u[1] < 0.5:
        occ, _ = dfs_maze(s, s, 0.02, sub)
        kind = "dfs"
    else:
        occ = bernoulli(s, s, 0.35, sub)
        kind = "bernoulli0.35"
    ns = 1 + int(u[2] * 16)
    nt = 8 + int(u[3] * 2041)
    return _on_largest_component(occ, ns, nt, sub, f"serve_{i}_{s}_{kind}", dict(kind=kind))


def serve_arrivals(n: int, rate_per_s: float, seed: int = 4) -> np.ndarray:
    """Poisson arrival times (seconds from 0) at rate_per_s: exponential gaps."""
    u = uniform(seed, S_ARRIVAL, n)
    gaps = -np.log1p(-u) / rate_per_s
    return np.cumsum(gaps)


def random_maze(H: int, W: int, p: float, n_src: int, n_tgt: int, seed: int,
                targets_anywhere: bool = True) -> Maze:
    """Small test maze: Bernoulli(p); n_src distinct sources uniform on free cells
    (any component); targets uniform over all cells (obstacles and unreachable
    cells included) when targets_anywhere, else uniform on free cells."""
    occ = bernoulli(H, W, p, seed)
    lab, ncomp, ll, ls = components(occ)
    free = int((occ == 0).sum())
    if free == 0:
        occ[0, 0] = 0
        lab, ncomp, ll, ls = components(occ)
        free = 1
    ns = min(n_src, free)
    src = sample_cells(lab, -2, ns, True, free, seed, S_SRC)
    if targets_anywhere:
        rc = below(seed, S_TGT, H * W, n_tgt)
        tgt = np.stack([rc // W, rc % W], axis=1).astype(np.int32) if n_tgt else np.zeros((0, 2), np.int32)
    else:
        tgt = sample_cells(lab, -2, n_tgt, False, free, seed, S_TGT)
    return Maze(occ, src, tgt, f"random_{H}x{W}_p{p}_s{seed}")
