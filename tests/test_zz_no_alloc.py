"""The allocation-free path extraction (omap_extract_paths_noalloc) against
omap_extract_paths on the same plans, called through the C ABI: two calls in
a row, the second on a smaller input, plus its two-phase sizing and its limit."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _extract(L, fn, plan, n_targets, device):
    import torch
    ln = torch.full((max(n_targets, 1),), -7, dtype=torch.int32, device=device)
    off = torch.full((n_targets + 1,), -7, dtype=torch.int64, device=device)
    need = ctypes.c_int64(-1)
    st = fn(plan, ctypes.c_void_p(ln.data_ptr()), ctypes.c_void_p(off.data_ptr()), None, 0, ctypes.byref(need))
    if need.value > 0:
        assert st == 8, L.omap_last_error()            # BUFFER_TOO_SMALL, needed written
    else:
        assert st == 0, L.omap_last_error()
    cells = torch.full((max(int(need.value), 1),), -7, dtype=torch.int32, device=device)
    st = fn(plan, ctypes.c_void_p(ln.data_ptr()), ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(cells.data_ptr()),
            cells.numel(), ctypes.byref(need))
    assert st == 0, L.omap_last_error()
    return ln[:n_targets].cpu().numpy(), off.cpu().numpy(), cells[: int(need.value)].cpu().numpy()


def _plan(L, m, stream):
    h = ctypes.c_void_p()
    occ = to_dev(m.occ)
    src = np.ascontiguousarray(m.sources, np.int32)
    tgt = np.ascontiguousarray(m.targets, np.int32)
    st = L.omap_plan_create(ctypes.byref(h), m.H, m.W, ctypes.c_void_p(occ.data_ptr()), src.ctypes.data, len(src),
                            tgt.ctypes.data if len(tgt) else None, len(tgt), None, stream)
    assert st == 0, L.omap_last_error()
    return h, occ


def test_noalloc_matches_extract_paths_twice_then_smaller():
    import torch
    import paper_2004_00540_amd as omap
    L = omap.lib()
    dev = torch.device("cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = workloads.random_maze(300, 410, 0.3, 3, 700, seed=71)
    small = workloads.random_maze(300, 410, 0.35, 2, 37, seed=72)     # same size, fewer targets
    plan, occ = _plan(L, big, stream)
    try:
        for m in (big, small):
            if m is small:
                occ = to_dev(m.occ)
                src = np.ascontiguousarray(m.sources, np.int32)
                tgt = np.ascontiguousarray(m.targets, np.int32)
                assert L.omap_plan_load(plan, ctypes.c_void_p(occ.data_ptr()), src.ctypes.data, len(src),
                                        tgt.ctypes.data, len(tgt)) == 0, L.omap_last_error()
            assert L.omap_propagate(plan, -1, None) == 0, L.omap_last_error()
            want = _extract(L, L.omap_extract_paths, plan, len(m.targets), dev)
            got = _extract(L, L.omap_extract_paths_noalloc, plan, len(m.targets), dev)
            for a, b in zip(got, want):
                assert np.array_equal(a, b)
            A, _ = oracle.layers(m.occ, m.sources, -1)
            rl, ro, rc = oracle.walk(A, m.sources, m.targets)
            assert np.array_equal(got[0], rl) and np.array_equal(got[1], ro) and np.array_equal(got[2], rc)
    finally:
        L.omap_plan_destroy(plan)


def test_noalloc_limit_and_not_propagated():
    import torch
    import paper_2004_00540_amd as omap
    L = omap.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n = (1 << 18) + 1
    m = workloads.random_maze(8, 8, 0.0, 1, 0, seed=5)
    m.targets = np.zeros((n, 2), np.int32)
    plan, occ = _plan(L, m, stream)
    try:
        ln = torch.empty(n, dtype=torch.int32, device="cuda")
        off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        need = ctypes.c_int64(-1)
        st = L.omap_extract_paths_noalloc(plan, ctypes.c_void_p(ln.data_ptr()), ctypes.c_void_p(off.data_ptr()),
                                          None, 0, ctypes.byref(need))
        assert omap.STATUS[st] == "OMAP_ERR_NOT_PROPAGATED"
        assert L.omap_propagate(plan, -1, None) == 0
        st = L.omap_extract_paths_noalloc(plan, ctypes.c_void_p(ln.data_ptr()), ctypes.c_void_p(off.data_ptr()),
                                          None, 0, ctypes.byref(need))
        assert omap.STATUS[st] == "OMAP_ERR_TOO_LARGE"
        assert b"at most 262144" in L.omap_last_error()
    finally:
        L.omap_plan_destroy(plan)
