"""Parity of the HIP path with the CPU oracle, bit for bit, through the C ABI.

Activity maps are compared with the oracle's literal network (small inputs)
or with its BFS closed form (large inputs, pinned to the literal network by
the CPU tests); paths are compared with the oracle's walk on the same map."""
import numpy as np
import pytest

import workloads
from gpu_helpers import assert_same, oracle_solution, run_plan, to_dev

pytestmark = pytest.mark.gpu

ALL_T = (4, 8, 12, 16)
ACTIVE, DENSE, BITS = 1, 2, 3      # OMAP_SCHEDULE_*


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available()
    import paper_2004_00540_amd as omap
    omap.selftest()


def test_selftest():
    import paper_2004_00540_amd as omap
    omap.selftest()


VARIANTS = [(T, 4) for T in ALL_T] + [(T, 2) for T in (4, 8, 12, 16, 24, 32)] + [(T, 1) for T in ALL_T]


@pytest.mark.parametrize("T,C", VARIANTS)
@pytest.mark.parametrize("tile_rows", [32, 64])
def test_random_mazes_all_variants(T, C, tile_rows):
    rng = np.random.default_rng(100 + T + tile_rows + C)
    for i in range(10):
        H, W = int(rng.integers(1, 300)), int(rng.integers(1, 700))
        m = workloads.random_maze(H, W, float(rng.uniform(0, 0.45)), int(rng.integers(1, 6)),
                                  int(rng.integers(0, 40)), 7000 + 31 * T + 7 * C + i)
        for L in (-1, int(rng.integers(0, 50))):
            got = run_plan(m, L, temporal_depth=T, tile_rows=tile_rows, lane_columns=C)
            assert_same(m, got, oracle_solution(m, L), f"{m.name} L={L} T={T} C={C} TH={tile_rows}")


@pytest.mark.parametrize("T,C", VARIANTS)
def test_minimum_tile_rows(T, C):
    m = workloads.random_maze(211, 389, 0.3, 3, 25, 555 + T + C)
    for L in (-1, 17):
        got = run_plan(m, L, temporal_depth=T, tile_rows=T, lane_columns=C)
        assert_same(m, got, oracle_solution(m, L), f"T={T} C={C} TH=T L={L}")


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (2, 1), (1, 1000), (1000, 1), (3, 257), (257, 3),
                                   (33, 31), (64, 64), (65, 225), (17, 224), (17, 226), (130, 449)])
def test_edge_shapes(shape):
    H, W = shape
    for seed in range(3):
        m = workloads.random_maze(H, W, 0.25, 2, 10, 9000 + seed * 7 + H)
        for L in (-1, 0, 1, 5):
            for T, C in ((4, 4), (16, 4), (8, 2), (32, 2)):
                got = run_plan(m, L, temporal_depth=T, tile_rows=max(T, 8), lane_columns=C)
                assert_same(m, got, oracle_solution(m, L), f"{shape} L={L} T={T} C={C}")


@pytest.mark.parametrize("shape", [(1, 1), (1, 1000), (1000, 1), (15, 40), (17, 33), (33, 31), (56, 100),
                                   (57, 100), (72, 65), (73, 97), (130, 449)])
def test_edge_shapes_two_wave_visits(shape):
    # the single-maze defaults (one column per lane, 16 layers, 16-row tiles)
    # visit each tile with two waves; near the top and bottom edges wave A
    # clamps rows and wave B drops rows cut by the edge
    H, W = shape
    for seed in range(3):
        m = workloads.random_maze(H, W, 0.25, 2, 10, 9100 + seed * 7 + H)
        for L in (-1, 0, 1, 5, 40):
            assert_same(m, run_plan(m, L), oracle_solution(m, L), f"{shape} L={L} default options")


def test_sources_on_borders_and_corners():
    H, W = 97, 301
    occ = workloads.bernoulli(H, W, 0.2, 55)
    srcs = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (0, 150), (48, 0), (48, W - 1), (H - 1, 77)]
    for s in srcs:
        occ[s] = 0
    tg = workloads.below(55, 9, H * W, 64)
    tg = np.stack([tg // W, tg % W], 1).astype(np.int32)
    for k in range(1, len(srcs) + 1):
        m = workloads.Maze(occ, np.array(srcs[:k], np.int32), tg, f"borders{k}")
        for L in (-1, 3, 40):
            assert_same(m, run_plan(m, L), oracle_solution(m, L), f"{m.name} L={L}")


def test_pockets_duplicates_and_special_targets():
    H, W = 80, 90
    occ = np.zeros((H, W), np.uint8)
    occ[20:40, 30] = 1
    occ[20:40, 50] = 1
    occ[20, 30:51] = 1
    occ[40, 30:51] = 1          # walled pocket (unreachable free cells inside)
    occ[60:70, 10:20] = 1
    src = np.array([[5, 5], [5, 5], [70, 80]], np.int32)          # duplicate source
    tgt = np.array([[30, 40], [65, 15], [5, 5], [70, 80], [0, 0], [79, 89], [30, 40]], np.int32)
    m = workloads.Maze(occ, src, tgt, "pockets")
    for L in (-1, 0, 1, 2, 30, 200):
        for T, C in VARIANTS:
            assert_same(m, run_plan(m, L, temporal_depth=T, tile_rows=max(16, T), lane_columns=C),
                        oracle_solution(m, L), f"pockets L={L} T={T} C={C}")


def test_isolated_source_and_all_obstacles():
    occ = np.ones((40, 40), np.uint8)
    occ[10, 10] = 0
    m = workloads.Maze(occ, np.array([[10, 10]], np.int32), np.array([[10, 10], [0, 0]], np.int32), "iso")
    for L in (-1, 0, 9):
        got = run_plan(m, L)
        assert_same(m, got, oracle_solution(m, L), f"iso L={L}")


def test_large_layer_count():
    m = workloads.random_maze(50, 70, 0.3, 1, 20, 4242)
    L = 2**31 - 2
    got = run_plan(m, L)
    act, ln, off, cells, info = got
    d, ecc = __import__("oracle").bfs(m.occ, m.sources)
    want = np.where(d >= 0, (L + 1) - d.astype(np.int64), 0)
    assert np.array_equal(act.astype(np.int64), want)
    assert info["layers"] == L


def test_schedules_and_options_identical_bits():
    m = workloads.random_maze(333, 517, 0.35, 3, 50, 31337)
    ref = oracle_solution(m, -1)
    for T, C in VARIANTS:
        for th in sorted({T, 2 * T + 2, 64, 256}):
            for sched in (ACTIVE, DENSE):
                for chk in (0, 1, 5):
                    got = run_plan(m, -1, temporal_depth=T, tile_rows=th, schedule=sched, check_interval=chk,
                                   lane_columns=C)
                    assert_same(m, got, ref, f"T={T} C={C} th={th} sched={sched} chk={chk}")


def test_config1():
    m = workloads.config1()
    for L in (-1, 0, 10, 58, 100):
        assert_same(m, run_plan(m, L), oracle_solution(m, L), f"config1 L={L}")


def test_config2_full_size():
    m = workloads.config2()
    got = run_plan(m, -1)
    assert_same(m, got, oracle_solution(m, -1, closed_form=True), "config2")
    got = run_plan(m, 1000, schedule=DENSE)
    assert_same(m, got, oracle_solution(m, 1000, closed_form=True), "config2 L=1000 dense")


@pytest.mark.parametrize("launch", [0, 1])
def test_launch_modes_identical_bits(launch):
    for i, (T, C) in enumerate([(16, 2), (16, 4), (8, 2), (32, 2)]):
        m = workloads.random_maze(400, 700, 0.33, 2 + i, 30, 6060 + i)
        for sched in (ACTIVE, DENSE):
            for L in (-1, 40):
                print(f"launch={launch} T={T} C={C} sched={sched} L={L}", flush=True)
                got = run_plan(m, L, temporal_depth=T, lane_columns=C, schedule=sched, round_launch=launch)
                assert_same(m, got, oracle_solution(m, L), f"launch={launch} T={T} C={C} sched={sched} L={L}")


def test_graph_replays_across_propagations():
    """Rounds replayed from captured HIP graphs: one plan propagated again and
    again with other layer counts and other mazes of the same size (the graph
    is captured again when its arguments change), every result against the
    oracle, for the integer and the bit-sliced schedules."""
    import paper_2004_00540_amd as omap
    ms = [workloads.random_maze(700, 300, p, 3, 25, 6100 + k) for k, p in enumerate((0.3, 0.1, 0.38))]
    for sched, T, C in ((ACTIVE, 16, 1), (ACTIVE, 12, 2), (BITS, 16, 0), (DENSE, 8, 4)):
        with omap.Plan(to_dev(ms[0].occ), ms[0].sources, ms[0].targets, temporal_depth=T, lane_columns=C,
                       schedule=sched, round_launch=omap.LAUNCH_GRAPH) as plan:
            for k, L in enumerate((-1, 37, -1, 200, 5, -1)):
                m = ms[k % len(ms)]
                plan.load(to_dev(m.occ), m.sources, m.targets)
                info = plan.propagate(L)
                act = plan.activity().cpu().numpy()
                ln, off, cells = (t.cpu().numpy() for t in plan.paths())
                assert_same(m, (act, ln, off, cells, info), oracle_solution(m, L), f"graph sched={sched} T={T} L={L}")
