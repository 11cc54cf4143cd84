"""Path reconstruction variants on the GPU against the oracle: the paper's
random tie-break (seeded, counter-based), Euclidean reconstruction (Eq. 1 and
straightening), and the index of the source each path ends on."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _source_index(cells, off, ln, sources, W):
    first = {}
    for j, (r, c) in enumerate(np.asarray(sources).reshape(-1, 2)):
        first.setdefault(int(r) * W + int(c), j)
    return np.array([first[int(cells[off[k + 1] - 1])] if ln[k] >= 0 else -1 for k in range(len(ln))],
                    np.int32)


def _cases():
    rng = np.random.default_rng(808)
    out = [workloads.config1()]
    for i in range(14):
        H, W = int(rng.integers(1, 200)), int(rng.integers(1, 300))
        out.append(workloads.random_maze(H, W, float(rng.uniform(0, 0.45)), int(rng.integers(1, 5)),
                                         int(rng.integers(0, 40)), 8080 + i))
    occ = np.zeros((90, 130), np.uint8)
    out.append(workloads.Maze(occ, np.array([[0, 0], [45, 65]], np.int32),
                              np.argwhere(np.ones((90, 130)))[::97].astype(np.int32), "empty_90x130"))
    return out


@pytest.mark.parametrize("mode", ["random", "euclidean", "first_max"])
def test_walk_modes_match_oracle(mode):
    import paper_2004_00540_amd as omap
    for m in _cases():
        A, L = oracle.layers(m.occ, m.sources, -1)
        for seed in ((0, 7, 2**63 + 5) if mode == "random" else (0,)):
            if mode == "random":
                rl, ro, rc = oracle.walk_random(A, m.sources, m.targets, seed)
            elif mode == "euclidean":
                rl, ro, rc = oracle.walk_euclidean(A, m.sources, m.targets)
            else:
                rl, ro, rc = oracle.walk(A, m.sources, m.targets)
            with omap.Plan(to_dev(m.occ), m.sources, m.targets) as plan:
                plan.propagate()
                ln, off, cells, src = (t.cpu().numpy() for t in plan.paths(mode, seed, source_index=True))
            assert np.array_equal(ln, rl), (m.name, mode, seed)
            assert np.array_equal(off, ro), (m.name, mode, seed)
            assert np.array_equal(cells, rc), (m.name, mode, seed)
            assert np.array_equal(src, _source_index(rc, ro, rl, m.sources, m.W)), (m.name, mode)


def test_random_ties_fixed_layers_and_config2():
    import paper_2004_00540_amd as omap
    m = workloads.config2()
    d, ecc = oracle.bfs(m.occ, m.sources)
    for L in (-1, 3000):
        A = oracle.activity_from_bfs(d, ecc if L < 0 else L)
        with omap.Plan(to_dev(m.occ), m.sources, m.targets) as plan:
            plan.propagate(L)
            for mode in ("random", "euclidean"):
                got = [t.cpu().numpy() for t in plan.paths(mode, 99)]
                ref = oracle.walk_random(A, m.sources, m.targets, 99) if mode == "random" else \
                    oracle.walk_euclidean(A, m.sources, m.targets)
                for g, r in zip(got, ref):
                    assert np.array_equal(g, r), (mode, L)


def test_batch_walk_modes_per_maze():
    import paper_2004_00540_amd as omap
    ms = _cases()[1:9]
    with omap.Batch([(to_dev(m.occ), m.sources, m.targets) for m in ms]) as b:
        b.propagate()
        for mode in ("random", "euclidean"):
            ln, off, cells, src = (t.cpu().numpy() for t in b.paths(mode, 4242, source_index=True))
            t0 = 0
            for m in ms:
                A, _ = oracle.layers(m.occ, m.sources, -1)
                rl, ro, rc = (oracle.walk_random(A, m.sources, m.targets, 4242) if mode == "random"
                              else oracle.walk_euclidean(A, m.sources, m.targets))
                n = len(m.targets)
                assert np.array_equal(ln[t0:t0 + n], rl)
                o = off[t0:t0 + n + 1] - off[t0]
                assert np.array_equal(o, ro)
                assert np.array_equal(cells[off[t0]:off[t0 + n]], rc)
                assert np.array_equal(src[t0:t0 + n], _source_index(rc, ro, rl, m.sources, m.W))
                t0 += n


def test_bad_walk_mode():
    import paper_2004_00540_amd as omap
    m = workloads.random_maze(10, 10, 0.1, 1, 2, 1)
    with omap.Plan(to_dev(m.occ), m.sources, m.targets) as plan:
        plan.propagate()
        with pytest.raises(omap.OmapError) as e:
            plan.paths(7)
        assert e.value.name == "OMAP_ERR_INVALID_ARG"


def _comb(H, W, vertical=False):
    """A serpentine maze: walls on every other row (column), each with one gap,
    alternating between the two ends, so the path from the corner source winds
    through the whole grid."""
    occ = np.zeros((H, W), np.uint8)
    for k, r in enumerate(range(1, H - 1, 2)):
        occ[r, :] = 1
        occ[r, W - 1 if k % 2 == 0 else 0] = 0
    if vertical:
        occ = np.ascontiguousarray(occ.T)
    return occ


def test_walk_winding_paths_and_short_tails():
    """Walks whose many three-step iterations stay inside one LDS window (the
    window is left because its log is full, not because the path leaves it),
    windows at the grid's edges and corners, and paths of every length modulo
    three (the last one or two steps of a path), against the oracle."""
    from gpu_helpers import assert_same, oracle_solution, run_plan
    cases = []
    # (a 20 x 30 comb lies inside the first window of a path from its far end,
    # so its ~300-step paths fill the 64-entry log before leaving the window)
    for H, W, vert in ((20, 30, False), (30, 20, True), (39, 57, False), (57, 39, True), (121, 203, False),
                       (203, 121, True), (5, 300, False)):
        occ = _comb(H, W, vert)
        free = np.argwhere(occ == 0).astype(np.int32)
        for src in ([[0, 0]], [[occ.shape[0] - 1, occ.shape[1] - 1]], [[0, 0], [occ.shape[0] // 2, 0]]):
            src = np.array(src, np.int32)
            src = src[occ[src[:, 0], src[:, 1]] == 0]
            cases.append(workloads.Maze(occ, src, free[::5].copy(), f"comb_{H}x{W}_{len(src)}"))
    # short paths: targets 0..8 cells from a source in an open grid, at the edges
    occ = np.zeros((9, 11), np.uint8)
    cases.append(workloads.Maze(occ, np.array([[4, 5]], np.int32), np.argwhere(occ == 0).astype(np.int32), "open_9x11"))
    cases.append(workloads.Maze(occ, np.array([[0, 0]], np.int32), np.argwhere(occ == 0).astype(np.int32),
                                "open_9x11_corner"))
    for m in cases:
        assert len(m.sources) > 0
        assert_same(m, run_plan(m, -1), oracle_solution(m, -1), m.name)
