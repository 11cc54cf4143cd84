"""Status codes, two-phase extraction, plan reuse and stream ordering of the
C ABI on the GPU."""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_helpers import oracle_solution, run_plan, to_dev, assert_same

pytestmark = pytest.mark.gpu


def test_source_on_obstacle_rejected():
    import paper_2004_00540_amd as omap
    m = workloads.random_maze(20, 30, 0.3, 1, 3, 1)
    occ = m.occ.copy()
    occ[m.sources[0, 0], m.sources[0, 1]] = 1
    with pytest.raises(omap.OmapError) as e:
        omap.Plan(to_dev(occ), m.sources, m.targets)
    assert e.value.name == "OMAP_ERR_SOURCE_ON_OBSTACLE"


def test_not_propagated_and_two_phase_extraction():
    import torch
    import paper_2004_00540_amd as omap
    m = workloads.random_maze(40, 50, 0.2, 2, 9, 2)
    L = omap.lib()
    with omap.Plan(to_dev(m.occ), m.sources, m.targets) as plan:
        out = torch.empty((40, 50), dtype=torch.int32, device="cuda")
        assert omap.STATUS[L.omap_get_activity(plan.handle, out.data_ptr(), 50)] == "OMAP_ERR_NOT_PROPAGATED"
        lens = torch.empty(9, dtype=torch.int32, device="cuda")
        offs = torch.empty(10, dtype=torch.int64, device="cuda")
        need = ctypes.c_int64(-1)
        st = L.omap_extract_paths(plan.handle, lens.data_ptr(), offs.data_ptr(), None, 0, ctypes.byref(need))
        assert omap.STATUS[st] == "OMAP_ERR_NOT_PROPAGATED"
        plan.propagate()
        assert omap.STATUS[L.omap_get_activity(plan.handle, out.data_ptr(), 49)] == "OMAP_ERR_INVALID_ARG"
        st = L.omap_extract_paths(plan.handle, lens.data_ptr(), offs.data_ptr(), None, 0, ctypes.byref(need))
        assert omap.STATUS[st] == "OMAP_ERR_BUFFER_TOO_SMALL"
        A, Ls, rl, ro, rc = oracle_solution(m, -1)
        assert need.value == len(rc)
        cells = torch.empty(need.value, dtype=torch.int32, device="cuda")
        st = L.omap_extract_paths(plan.handle, lens.data_ptr(), offs.data_ptr(), cells.data_ptr(),
                                  need.value - 1, ctypes.byref(need))
        assert omap.STATUS[st] == "OMAP_ERR_BUFFER_TOO_SMALL" and need.value == len(rc)
        assert plan.extract_into(lens, offs, cells) == len(rc)
        assert np.array_equal(cells.cpu().numpy(), rc)
        # pitched destination
        wide = torch.full((40, 64), -5, dtype=torch.int32, device="cuda")
        plan.activity(out=wide[:, :50])
        w = wide.cpu().numpy()
        assert np.array_equal(w[:, :50], A) and (w[:, 50:] == -5).all()


def test_bad_layer_counts():
    import paper_2004_00540_amd as omap
    m = workloads.random_maze(10, 10, 0.1, 1, 1, 3)
    with omap.Plan(to_dev(m.occ), m.sources, m.targets) as plan:
        with pytest.raises(omap.OmapError) as e:
            plan.propagate(-2)
        assert e.value.name == "OMAP_ERR_INVALID_ARG"
        with pytest.raises(omap.OmapError) as e:
            plan.propagate(2**31 - 1)
        assert e.value.name == "OMAP_ERR_TOO_LARGE"


def test_plan_reuse_and_repeated_propagate():
    import paper_2004_00540_amd as omap
    a = workloads.random_maze(123, 321, 0.3, 2, 20, 10)
    b = workloads.random_maze(123, 321, 0.4, 4, 30, 11)
    with omap.Plan(to_dev(a.occ), a.sources, a.targets, temporal_depth=12, tile_rows=24) as plan:
        for m in (a, b, a):
            plan.load(to_dev(m.occ), m.sources, m.targets)
            for L in (-1, 9, -1):
                info = plan.propagate(L)
                act = plan.activity().cpu().numpy()
                ln, off, cells = (t.cpu().numpy() for t in plan.paths())
                assert_same(m, (act, ln, off, cells, info), oracle_solution(m, L), f"{m.name} L={L}")


def test_side_stream_ordering():
    import torch
    import paper_2004_00540_amd as omap
    m = workloads.random_maze(700, 900, 0.3, 3, 64, 12)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        occ = to_dev(m.occ)
        with omap.Plan(occ, m.sources, m.targets, stream=s) as plan:
            plan.propagate(-1, sync=False)
            out = torch.empty((700, 900), dtype=torch.int32, device="cuda")
            plan.activity(out=out)
            host = out.to("cpu", non_blocking=False)
    A, L, *_ = oracle_solution(m, -1)
    assert np.array_equal(host.numpy(), A)


def test_no_paths_needs_no_cell_buffer():
    import torch
    import paper_2004_00540_amd as omap
    occ = np.zeros((8, 8), np.uint8)
    occ[3, :] = 1
    src = np.array([[0, 0]], np.int32)
    tgt = np.array([[7, 7], [3, 3]], np.int32)     # unreachable, obstacle
    L = omap.lib()
    with omap.Plan(to_dev(occ), src, tgt) as plan:
        plan.propagate()
        lens = torch.empty(2, dtype=torch.int32, device="cuda")
        offs = torch.empty(3, dtype=torch.int64, device="cuda")
        need = ctypes.c_int64(-1)
        st = L.omap_extract_paths(plan.handle, lens.data_ptr(), offs.data_ptr(), None, 0, ctypes.byref(need))
        assert st == 0 and need.value == 0
        assert lens.cpu().tolist() == [-1, -1] and offs.cpu().tolist() == [0, 0, 0]
