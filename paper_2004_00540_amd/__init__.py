"""Python binding of the gfx950 oMAP maze planner (libomap.so, include/omap.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and the current HIP stream.
If the library has not been built the import still succeeds, but every call
raises -- there is no CPU fallback.

    import torch, paper_2004_00540_amd as omap
    occ = torch.from_numpy(grid).cuda()                 # uint8 (H, W), 1 = obstacle
    with omap.Plan(occ, sources, targets) as plan:      # (row, col) int arrays
        info = plan.propagate()                         # run-time determined L
        O = plan.activity()                             # int32 (H, W) on the GPU
        lengths, offsets, cells = plan.paths()
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OMAP_LIBRARY may name another build of the same library (e.g. for A/B timing)
LIB_PATH = os.environ.get("OMAP_LIBRARY") or os.path.join(_HERE, "libomap.so")

AUTO = -1
SCHEDULE_DEFAULT = 0
SCHEDULE_ACTIVE = 1
SCHEDULE_DENSE = 2
SCHEDULE_BITS = 3
QUERY_QUEUED, QUERY_RUNNING, QUERY_DONE, QUERY_FAILED = 0, 1, 2, 3
QUERY_KEEP_ACTIVITY = 1

STATUS = {
    0: "OMAP_OK", 1: "OMAP_ERR_INVALID_ARG", 2: "OMAP_ERR_TOO_LARGE",
    3: "OMAP_ERR_SOURCE_OUT_OF_BOUNDS", 4: "OMAP_ERR_SOURCE_ON_OBSTACLE", 5: "OMAP_ERR_NO_SOURCES",
    6: "OMAP_ERR_TARGET_OUT_OF_BOUNDS", 7: "OMAP_ERR_NOT_PROPAGATED", 8: "OMAP_ERR_BUFFER_TOO_SMALL",
    9: "OMAP_ERR_OUT_OF_MEMORY", 10: "OMAP_ERR_HIP", 11: "OMAP_ERR_NOT_FOUND", 12: "OMAP_ERR_BUSY",
}
OK, ERR_BUFFER_TOO_SMALL, ERR_BUSY = 0, 8, 12


class OmapError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Options(ctypes.Structure):
    _fields_ = [("temporal_depth", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("check_interval", ctypes.c_int32),
                ("lane_columns", ctypes.c_int32), ("round_launch", ctypes.c_int32)]


class PropagateInfo(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int64), ("sweeps_executed", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("tile_visits", ctypes.c_int64),
                ("reached_cells", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


WALK_FIRST_MAX, WALK_RANDOM_TIES, WALK_EUCLIDEAN = 0, 1, 2


class WalkOptions(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class MazeDesc(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("occupancy_dev", ctypes.c_void_p),
                ("sources_host", ctypes.c_void_p), ("n_sources", ctypes.c_int32),
                ("targets_host", ctypes.c_void_p), ("n_targets", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libomap.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "omap_plan_create": [PP, i32, i32, P, P, i32, P, i32, P, P],
        "omap_plan_load": [P, P, P, i32, P, i32],
        "omap_propagate": [P, i64, P],
        "omap_get_activity": [P, P, i64],
        "omap_extract_paths": [P, P, P, P, i64, P],
        "omap_extract_paths_ex": [P, P, P, P, P, i64, P, P],
        "omap_extract_paths_noalloc": [P, P, P, P, i64, P],
        "omap_batch_extract_paths_ex": [P, P, P, P, P, i64, P, P],
        "omap_plan_destroy": [P],
        "omap_batch_create": [PP, P, i32, P, P],
        "omap_batch_propagate": [P, P, P],
        "omap_batch_get_activity": [P, i32, P, i64],
        "omap_batch_extract_paths": [P, P, P, P, i64, P],
        "omap_batch_destroy": [P],
        "omap_engine_create": [PP, i64, i32, P, P],
        "omap_engine_submit": [P, i32, i32, P, P, i32, P, i32, i64, P],
        "omap_engine_submit_ex": [P, i32, i32, P, P, i32, P, i32, i64, ctypes.c_uint32, P],
        "omap_engine_fetch_activity": [P, i64, P, i64],
        "omap_engine_step": [P, i32, P, P],
        "omap_engine_poll": [P, i64, P],
        "omap_engine_completed": [P, P, i32, P],
        "omap_engine_fetch": [P, i64, P, P, P, i64, P, P],
        "omap_engine_destroy": [P],
        "omap_profile_enable": [P, i32, i32],
        "omap_profile_read": [P, i32, P, P, P],
        "omap_selftest": [P],
        "omap_resolve_options": [P, P],
        "omap_tune": [P, i32, i32, P, P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name in ("omap_last_error", "omap_version"):
        getattr(L, name).restype = ctypes.c_char_p
        getattr(L, name).argtypes = []
    L.omap_status_string.restype = ctypes.c_char_p
    L.omap_status_string.argtypes = [ctypes.c_int]
    _lib = L
    return L


def _check(status: int):
    if status != OK:
        raise OmapError(status, lib().omap_last_error().decode())


def _rc(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1, 2))


def _host_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def _stream(stream=None) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


LAUNCH_PER_ROUND, LAUNCH_GRAPH = 0, 1
USE_PLAN, USE_BATCH, USE_ENGINE = 0, 1, 2


class TuneResult(ctypes.Structure):
    _fields_ = [("options", Options), ("candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


def _options(temporal_depth=0, tile_rows=0, schedule=SCHEDULE_DEFAULT, check_interval=0,
             lane_columns=0, round_launch=LAUNCH_PER_ROUND):
    return Options(temporal_depth, tile_rows, schedule, check_interval, lane_columns, round_launch)


def _descs(mazes):
    """MazeDesc array (and the host arrays it points into) for (occupancy,
    sources, targets) triples."""
    keep, descs = [], []
    for occ, src, tgt in mazes:
        occ = _device_u8(occ)
        s = _rc(src)
        t = _rc(tgt if tgt is not None else np.zeros((0, 2), np.int32))
        keep += [occ, s, t]
        descs.append(MazeDesc(int(occ.shape[0]), int(occ.shape[1]), occ.data_ptr(),
                              s.ctypes.data, len(s), t.ctypes.data if len(t) else None, len(t)))
    return (MazeDesc * len(descs))(*descs), keep


def tune(mazes, use: int = USE_BATCH, stream=None) -> dict:
    """omap_tune on (occupancy CUDA tensor, sources, targets) triples: the
    fastest options for a workload like them (every candidate's maps checked
    against the defaults'), read from OMAP_TUNE_CACHE when present.  Returns
    {"options": keyword options for Plan / Batch / Engine, "candidates",
    "from_cache", "best_ms", "default_ms"}."""
    arr, keep = _descs(mazes)
    res = TuneResult()
    _check(lib().omap_tune(arr, len(arr), int(use), ctypes.byref(res), ctypes.c_void_p(_stream(stream))))
    del keep
    return {"options": {f: getattr(res.options, f) for f, _ in Options._fields_},
            "candidates": res.candidates, "from_cache": res.from_cache,
            "best_ms": res.best_ms, "default_ms": res.default_ms}


def resolve_options(**options) -> dict:
    """The options a plan / batch / engine created with these keyword options
    runs with (defaults filled in); host only."""
    out = Options()
    _check(lib().omap_resolve_options(ctypes.byref(_options(**options)), ctypes.byref(out)))
    return {f: getattr(out, f) for f, _ in Options._fields_}


def _device_u8(occ):
    import torch
    if not isinstance(occ, torch.Tensor) or not occ.is_cuda:
        raise TypeError("occupancy must be a CUDA (HIP) uint8 tensor")
    if occ.dtype != torch.uint8 or occ.dim() != 2 or not occ.is_contiguous():
        raise TypeError("occupancy must be a contiguous uint8 (H, W) tensor")
    return occ


def version() -> str:
    return lib().omap_version().decode()


def selftest(stream=None) -> None:
    """Device checks of the cross-lane moves and saturating arithmetic."""
    _check(lib().omap_selftest(ctypes.c_void_p(_stream(stream))))


def _paths(extract, n_targets: int, device, walk=None, source_index=False):
    """Two-phase path extraction through an omap_*_extract_paths_ex entry point.
    Returns (lengths, offsets, cells) or, with source_index, also the index of
    the source each path ends on."""
    import torch
    lengths = torch.empty(max(n_targets, 1), dtype=torch.int32, device=device)
    offsets = torch.empty(n_targets + 1, dtype=torch.int64, device=device)
    src = torch.empty(max(n_targets, 1), dtype=torch.int32, device=device) if source_index else None
    wopt = ctypes.byref(walk) if walk is not None else None
    sptr = src.data_ptr() if src is not None else None
    needed = ctypes.c_int64(0)
    st = extract(wopt, lengths.data_ptr(), offsets.data_ptr(), None, 0, ctypes.byref(needed), sptr)
    if st not in (OK, ERR_BUFFER_TOO_SMALL):
        _check(st)
    cells = torch.empty(max(int(needed.value), 1), dtype=torch.int32, device=device)
    _check(extract(wopt, lengths.data_ptr(), offsets.data_ptr(), cells.data_ptr(), cells.numel(),
                   ctypes.byref(needed), sptr))
    out = (lengths[:n_targets], offsets, cells[: int(needed.value)])
    return out + (src[:n_targets],) if source_index else out


def _walk_options(mode, seed):
    if mode is None:
        return None
    m = {"first_max": WALK_FIRST_MAX, "random": WALK_RANDOM_TIES, "euclidean": WALK_EUCLIDEAN}.get(mode, mode)
    return WalkOptions(int(m), 0, int(seed) & 0xFFFFFFFFFFFFFFFF)


class Plan:
    """One maze: omap_plan_create / omap_propagate / omap_get_activity /
    omap_extract_paths / omap_plan_destroy."""

    def __init__(self, occupancy, sources, targets=None, stream=None, **options):
        occ = _device_u8(occupancy)
        self.H, self.W = int(occ.shape[0]), int(occ.shape[1])
        self.device = occ.device
        src = _rc(sources)
        tgt = _rc(targets if targets is not None else np.zeros((0, 2), np.int32))
        self.n_targets = len(tgt)
        self._opts = _options(**options)
        self._stream = _stream(stream)
        h = ctypes.c_void_p()
        _check(lib().omap_plan_create(ctypes.byref(h), self.H, self.W, occ.data_ptr(),
                                      _host_ptr(src), len(src), _host_ptr(tgt), len(tgt),
                                      ctypes.byref(self._opts), ctypes.c_void_p(self._stream)))
        self.handle = h

    def load(self, occupancy, sources, targets=None):
        occ = _device_u8(occupancy)
        assert tuple(occ.shape) == (self.H, self.W)
        src = _rc(sources)
        tgt = _rc(targets if targets is not None else np.zeros((0, 2), np.int32))
        _check(lib().omap_plan_load(self.handle, occ.data_ptr(), _host_ptr(src), len(src),
                                    _host_ptr(tgt), len(tgt)))
        self.n_targets = len(tgt)

    def propagate(self, layers: int = AUTO, sync: bool = True):
        """Run the network; returns the info dict (sync) or None (async)."""
        if sync:
            info = PropagateInfo()
            _check(lib().omap_propagate(self.handle, int(layers), ctypes.byref(info)))
            return info.as_dict()
        _check(lib().omap_propagate(self.handle, int(layers), None))
        return None

    def activity(self, out=None):
        import torch
        if out is None:
            out = torch.empty((self.H, self.W), dtype=torch.int32, device=self.device)
        _check(lib().omap_get_activity(self.handle, out.data_ptr(), int(out.stride(0))))
        return out

    def paths(self, mode=None, seed: int = 0, source_index: bool = False):
        """(lengths int32 [t], offsets int64 [t+1], cells int32) on the GPU
        (+ source index per target).  mode: None / "first_max", "random",
        "euclidean"."""
        ex = lambda *a: lib().omap_extract_paths_ex(self.handle, *a)  # noqa: E731
        return _paths(ex, self.n_targets, self.device, _walk_options(mode, seed), source_index)

    def extract_into(self, lengths, offsets, cells):
        needed = ctypes.c_int64(0)
        _check(lib().omap_extract_paths(self.handle, lengths.data_ptr(), offsets.data_ptr(),
                                        cells.data_ptr(), cells.numel(), ctypes.byref(needed)))
        return int(needed.value)

    def profile(self, enable: bool):
        _check(lib().omap_profile_enable(self.handle, 0, int(enable)))

    def profile_read(self):
        n, ms, cu = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().omap_profile_read(self.handle, 0, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(cu)))
        return {"launches": n.value, "ms": ms.value, "cell_updates": cu.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().omap_plan_destroy(self.handle)
            self.handle = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many mazes advanced by the same launches: omap_batch_*."""

    def __init__(self, mazes, stream=None, **options):
        """mazes: iterable of (occupancy uint8 CUDA tensor, sources, targets)."""
        self._keep = []
        descs = []
        self.n_targets = []
        self.shapes = []
        device = None
        for occ, src, tgt in mazes:
            occ = _device_u8(occ)
            device = occ.device
            s = _rc(src)
            t = _rc(tgt if tgt is not None else np.zeros((0, 2), np.int32))
            self._keep += [occ, s, t]
            descs.append(MazeDesc(int(occ.shape[0]), int(occ.shape[1]), occ.data_ptr(),
                                  s.ctypes.data, len(s), t.ctypes.data if len(t) else None, len(t)))
            self.n_targets.append(len(t))
            self.shapes.append((int(occ.shape[0]), int(occ.shape[1])))
        self.device = device
        arr = (MazeDesc * len(descs))(*descs)
        self._opts = _options(**options)
        h = ctypes.c_void_p()
        _check(lib().omap_batch_create(ctypes.byref(h), arr, len(descs), ctypes.byref(self._opts),
                                       ctypes.c_void_p(_stream(stream))))
        self.handle = h
        self._keep = []   # inputs were copied / packed synchronously

    def __len__(self):
        return len(self.shapes)

    def propagate(self, layers=None, sync: bool = True):
        n = len(self.shapes)
        L = None
        if layers is not None:
            arr = np.broadcast_to(np.asarray(layers, dtype=np.int64), (n,)).copy()
            L = arr.ctypes.data_as(ctypes.c_void_p)
        if sync:
            infos = (PropagateInfo * n)()
            _check(lib().omap_batch_propagate(self.handle, L, infos))
            return [i.as_dict() for i in infos]
        _check(lib().omap_batch_propagate(self.handle, L, None))
        return None

    def activity(self, index: int, out=None):
        import torch
        H, W = self.shapes[index]
        if out is None:
            out = torch.empty((H, W), dtype=torch.int32, device=self.device)
        _check(lib().omap_batch_get_activity(self.handle, int(index), out.data_ptr(), int(out.stride(0))))
        return out

    def paths(self, mode=None, seed: int = 0, source_index: bool = False):
        ex = lambda *a: lib().omap_batch_extract_paths_ex(self.handle, *a)  # noqa: E731
        return _paths(ex, sum(self.n_targets), self.device, _walk_options(mode, seed), source_index)

    def profile(self, enable: bool):
        _check(lib().omap_profile_enable(self.handle, 1, int(enable)))

    def profile_read(self):
        n, ms, cu = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().omap_profile_read(self.handle, 1, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(cu)))
        return {"launches": n.value, "ms": ms.value, "cell_updates": cu.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().omap_batch_destroy(self.handle)
            self.handle = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


@dataclass
class QueryResult:
    lengths: np.ndarray
    offsets: np.ndarray
    cells: np.ndarray
    info: dict


class Engine:
    """Serving loop with continuous batching: omap_engine_*."""

    def __init__(self, memory_budget_bytes: int, max_slots: int = 64, stream=None, **options):
        self._opts = _options(**options)
        h = ctypes.c_void_p()
        _check(lib().omap_engine_create(ctypes.byref(h), int(memory_budget_bytes), int(max_slots),
                                        ctypes.byref(self._opts), ctypes.c_void_p(_stream(stream))))
        self.handle = h
        self._nt = {}
        self._shape = {}

    def submit(self, occupancy: np.ndarray, sources, targets, layers: int = AUTO,
               keep_activity: bool = False) -> int:
        """Queue a query (omap_engine_submit_ex); keep_activity keeps its
        activity map for activity()."""
        occ = np.ascontiguousarray(occupancy, dtype=np.uint8)
        src = _rc(sources)
        tgt = _rc(targets if targets is not None else np.zeros((0, 2), np.int32))
        qid = ctypes.c_int64()
        _check(lib().omap_engine_submit_ex(self.handle, occ.shape[0], occ.shape[1], _host_ptr(occ),
                                           _host_ptr(src), len(src), _host_ptr(tgt), len(tgt),
                                           int(layers), QUERY_KEEP_ACTIVITY if keep_activity else 0,
                                           ctypes.byref(qid)))
        self._nt[qid.value] = len(tgt)
        self._shape[qid.value] = (int(occ.shape[0]), int(occ.shape[1]))
        return qid.value

    def activity(self, qid: int) -> np.ndarray:
        """Activity map (int32 (H, W), host) of a finished query submitted with
        keep_activity; call before fetch()."""
        H, W = self._shape[qid]
        out = np.empty((H, W), np.int32)
        _check(lib().omap_engine_fetch_activity(self.handle, int(qid), out.ctypes.data_as(ctypes.c_void_p), W))
        return out

    def step(self, rounds: int = 4):
        res, done = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().omap_engine_step(self.handle, int(rounds), ctypes.byref(res), ctypes.byref(done)))
        return res.value, done.value

    def completed(self, capacity: int = 4096) -> list:
        """Ids of the queries that finished (DONE or FAILED) since the last call."""
        out = []
        buf = np.empty(capacity, np.int64)
        n = ctypes.c_int32()
        while True:
            _check(lib().omap_engine_completed(self.handle, buf.ctypes.data_as(ctypes.c_void_p), capacity,
                                               ctypes.byref(n)))
            out += buf[: n.value].tolist()
            if n.value < capacity:
                return out

    def poll(self, qid: int) -> int:
        st = ctypes.c_int32()
        _check(lib().omap_engine_poll(self.handle, int(qid), ctypes.byref(st)))
        return st.value

    def fetch(self, qid: int) -> QueryResult:
        nt = self._nt[qid]
        ln = np.empty(max(nt, 1), np.int32)
        off = np.empty(nt + 1, np.int64)
        needed = ctypes.c_int64()
        info = PropagateInfo()
        st = lib().omap_engine_fetch(self.handle, int(qid), ln.ctypes.data_as(ctypes.c_void_p),
                                     off.ctypes.data_as(ctypes.c_void_p), None, 0,
                                     ctypes.byref(needed), ctypes.byref(info))
        if st == OK:     # no target has a path: the query is complete already
            del self._nt[qid]
            self._shape.pop(qid, None)
            return QueryResult(ln[:nt], off, np.zeros(0, np.int32), info.as_dict())
        if st != ERR_BUFFER_TOO_SMALL:
            _check(st)
        cells = np.empty(max(int(needed.value), 1), np.int32)
        _check(lib().omap_engine_fetch(self.handle, int(qid), ln.ctypes.data_as(ctypes.c_void_p),
                                       off.ctypes.data_as(ctypes.c_void_p),
                                       cells.ctypes.data_as(ctypes.c_void_p), cells.size,
                                       ctypes.byref(needed), ctypes.byref(info)))
        del self._nt[qid]
        self._shape.pop(qid, None)
        return QueryResult(ln[:nt], off, cells[: int(needed.value)], info.as_dict())

    def close(self):
        if getattr(self, "handle", None):
            lib().omap_engine_destroy(self.handle)
            self.handle = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
