"""The bit-sliced reached-set schedule (OMAP_SCHEDULE_BITS): same activity
maps and paths as the oracle's literal layers, for both layer depths per
visit, fixed and run-time L, single-tile and multi-tile shapes (a bit tile is
1984 columns wide), batches and the serving engine."""
import numpy as np
import pytest

import workloads
from gpu_helpers import assert_same, oracle_solution, run_plan, to_dev

pytestmark = pytest.mark.gpu

BITS = 3   # OMAP_SCHEDULE_BITS


@pytest.mark.parametrize("T", [8, 16])
def test_bits_matches_oracle(T):
    shapes = [(37, 83, 0.3), (1, 700, 0.0), (300, 1, 0.1), (129, 2100, 0.35), (64, 4100, 0.2), (257, 1985, 0.3)]
    for k, (H, W, p) in enumerate(shapes):
        m = workloads.random_maze(H, W, p, 1 + k % 4, 25, 7700 + 13 * T + k)
        for L in (-1, 0, 1, T - 1, T, 3 * T + 5):
            print(f"bits T={T} {H}x{W} L={L}", flush=True)
            got = run_plan(m, L, schedule=BITS, temporal_depth=T)
            assert_same(m, got, oracle_solution(m, L), f"bits T={T} {H}x{W} L={L}")


def test_bits_tile_rows_and_empty_map():
    m = workloads.random_maze(400, 3000, 0.3, 3, 30, 7801)
    ref = oracle_solution(m, -1)
    for TH in (16, 18, 64):
        assert_same(m, run_plan(m, -1, schedule=BITS, temporal_depth=16, tile_rows=TH), ref, f"TH={TH}")
    e = workloads.random_maze(500, 2500, 0.0, 1, 10, 7802)
    assert_same(e, run_plan(e, 100, schedule=BITS), oracle_solution(e, 100), "empty, L=100")


def test_bits_config2_full_size():
    m = workloads.config2()
    got = run_plan(m, -1, schedule=BITS)
    assert_same(m, got, oracle_solution(m, -1, closed_form=True), "config2 bits")


def test_bits_batch_and_engine():
    import paper_2004_00540_amd as omap
    rng = np.random.default_rng(5)
    ms = [workloads.random_maze(int(rng.integers(1, 300)), int(rng.integers(1, 2500)),
                                float(rng.uniform(0.05, 0.4)), int(rng.integers(1, 5)), 12, 7900 + i)
          for i in range(12)]
    layers = [-1 if i % 3 else 20 + i for i in range(len(ms))]
    with omap.Batch([(to_dev(m.occ), m.sources, m.targets) for m in ms], schedule=BITS) as b:
        infos = b.propagate(layers)
        acts = [b.activity(i).cpu().numpy() for i in range(len(ms))]
    for i, m in enumerate(ms):
        A, L, _, _, _ = oracle_solution(m, layers[i])
        assert infos[i]["layers"] == L, i
        assert np.array_equal(acts[i], A), i
    with omap.Engine(1 << 30, max_slots=4, schedule=BITS) as eng:
        ids = {eng.submit(m.occ, m.sources, m.targets): k for k, m in enumerate(ms[:6])}
        res = {}
        n = 0
        while len(res) < len(ids):
            eng.step(rounds=2)
            for qid, k in list(ids.items()):
                if k not in res and eng.poll(qid) == omap.QUERY_DONE:
                    res[k] = eng.fetch(qid)
            n += 1
            assert n < 100000
    for k, r in res.items():
        A, L, rl, ro, rc = oracle_solution(ms[k], -1)
        assert r.info["layers"] == L
        assert np.array_equal(r.lengths, rl) and np.array_equal(r.cells, rc), k
