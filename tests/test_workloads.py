"""Seeded input generators: determinism (content hashes pinned here), the
structure each workload family promises, and source/target placement."""
import math

import numpy as np
import pytest

import workloads as w
from pins import flood_reachable

# FNV-1a content hashes of (occupancy, sources, targets); they change only if
# the generators change.
HASH_CONFIG1 = 1796992504980525774
HASH_CONFIG2 = 8250361588706676807
HASH_CONFIG4_MAZE0 = 9882790751897786604
HASH_CONFIG3_FULL = 3616199043951189294


def test_config1_pinned_and_valid():
    m = w.config1()
    assert w.content_hash(m.occ, m.sources, m.targets) == HASH_CONFIG1
    assert m.occ.shape == (64, 64)
    assert abs(m.occ.mean() - 0.30) < 0.03
    assert m.sources.shape == (1, 2) and m.targets.shape == (4, 2)
    reach = flood_reachable(m.occ, m.sources)
    assert all(tuple(t) in reach for t in m.targets)


def test_config2_pinned_and_structure():
    m = w.config2()
    assert w.content_hash(m.occ, m.sources, m.targets) == HASH_CONFIG2
    assert m.meta["walls_removed"] == 83804          # 2% of 4,190,209 remaining walls
    assert m.meta["n_components"] == 1
    assert abs((1 - m.occ.mean()) - 0.505) < 0.002
    assert len(m.targets) == 256 and len({tuple(t) for t in m.targets}) == 256
    occ = m.occ
    assert occ[1::2, 1::2].all()                     # pillars stay wall
    assert occ[-1, :].all() and occ[:, -1].all()      # last row / column stay wall


@pytest.mark.parametrize("side", [9, 16, 33, 64])
def test_dfs_maze_is_spanning_tree_before_removals(side):
    occ, removed = w.dfs_maze(side, side, 0.0, 12345)
    assert removed == 0
    kr, kc = (side + 1) // 2, (side + 1) // 2
    passages = int((occ[0::2, 1::2] == 0).sum() + (occ[1::2, 0::2] == 0).sum())
    assert passages == kr * kc - 1                    # a tree on kr*kc lattice cells
    lab, ncomp, _, _ = w.components(occ)
    assert ncomp == 1


def test_dfs_removal_count():
    occ0, _ = w.dfs_maze(200, 200, 0.0, 99)
    walls = int((occ0[0::2, 1::2][:, :99] == 1).sum() + (occ0[1::2, 0::2][:99, :] == 1).sum())
    occ1, removed = w.dfs_maze(200, 200, 0.02, 99)
    assert removed == round(0.02 * walls)
    assert int((occ0 != occ1).sum()) == removed


def test_rect_overlay_and_largest_component():
    m = w.config3(side=2048, n_rects=50000 * 2048 * 2048 // (23170 * 23170))
    lab, ncomp, ll, ls = w.components(m.occ)
    assert len(m.sources) == 16 and len(m.targets) == 4096
    cells = np.concatenate([m.sources, m.targets])
    assert len({tuple(c) for c in cells}) == len(cells)
    assert (lab[cells[:, 0], cells[:, 1]] == ll).all()
    sizes = np.bincount(lab[lab >= 0].ravel())
    assert sizes.max() == ls


def test_components_match_flood_fill():
    for seed in range(20):
        m = w.random_maze(13, 17, 0.45, 1, 0, seed)
        lab, _, _, _ = w.components(m.occ)
        reach = flood_reachable(m.occ, m.sources)
        s = tuple(m.sources[0])
        same = {tuple(x) for x in np.argwhere(lab == lab[s])}
        assert same == reach


def test_config4_params_ranges():
    p = w.config4_params()
    assert len(p) == 512
    for H, W, prob, ns, nt in p:
        assert 128 <= H <= 2048 and 128 <= W <= 2048
        assert 0.2 <= prob <= 0.45
        assert 1 <= ns <= 8 and 16 <= nt <= 512
    total = sum(H * W for H, W, *_ in p)
    assert 2.0e8 < total < 3.0e8
    logs = np.log([H for H, *_ in p])
    assert abs(logs.mean() - (math.log(128) + math.log(2048)) / 2) < 0.15


def test_config4_maze_pinned():
    m = w.config4_maze(0)
    assert w.content_hash(m.occ, m.sources, m.targets) == HASH_CONFIG4_MAZE0
    lab, _, ll, _ = w.components(m.occ)
    cells = np.concatenate([m.sources, m.targets])
    assert (lab[cells[:, 0], cells[:, 1]] == ll).all()


def test_serve_queries():
    kinds = set()
    for i in range(6):
        u = w.uniform(4 * 7919 + i, w.S_PARAM, 4)
        s = int(round(math.exp(math.log(256) + (math.log(8192) - math.log(256)) * u[0])))
        kinds.add("dfs" if u[1] < 0.5 else "bernoulli")
        assert 256 <= s <= 8192
    q = w.serve_query(1)
    assert q.occ.shape[0] == q.occ.shape[1]
    assert 1 <= len(q.sources) <= 16 and 8 <= len(q.targets) <= 2048
    t = w.serve_arrivals(1000, 50.0)
    assert (np.diff(t) > 0).all()
    assert abs(1000 / t[-1] - 50.0) < 5.0


def test_determinism_and_seed_sensitivity():
    a = w.bernoulli(100, 120, 0.3, 5)
    b = w.bernoulli(100, 120, 0.3, 5)
    c = w.bernoulli(100, 120, 0.3, 6)
    assert (a == b).all() and (a != c).any()


@pytest.mark.slow
def test_config3_full_pinned():
    m = w.config3()
    assert w.content_hash(m.occ, m.sources, m.targets) == HASH_CONFIG3_FULL
