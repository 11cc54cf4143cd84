"""Batched and serving forms: every maze's results are bit-identical to the
oracle and to solving the maze alone, whatever else shares the launches."""
import numpy as np
import pytest

import workloads
from gpu_helpers import oracle_solution, run_plan, to_dev

pytestmark = pytest.mark.gpu


def _split(ln, off, cells, counts):
    out, t = [], 0
    for n in counts:
        l = ln[t:t + n]
        o = off[t:t + n + 1]
        c = cells[o[0]:o[-1]]
        out.append((l, o - o[0], c))
        t += n
    return out


def _batch_mazes(n, seed, hmax=300):
    rng = np.random.default_rng(seed)
    ms = []
    for i in range(n):
        H, W = int(rng.integers(1, hmax)), int(rng.integers(1, hmax * 2))
        ms.append(workloads.random_maze(H, W, float(rng.uniform(0.05, 0.45)), int(rng.integers(1, 6)),
                                        int(rng.integers(0, 30)), seed * 1000 + i))
    return ms


@pytest.mark.parametrize("T,tile_rows,schedule,launch", [(16, 64, 1, 0), (8, 16, 1, 0), (4, 8, 2, 0), (12, 24, 1, 0),
                                                        (16, 16, 1, 1), (8, 8, 2, 1), (16, 16, 3, 1), (8, 16, 3, 0)])
def test_batch_matches_oracle(T, tile_rows, schedule, launch):
    import paper_2004_00540_amd as omap
    ms = _batch_mazes(24, 50 + T + launch)
    rng = np.random.default_rng(T)
    layers = [int(x) if x >= 0 else -1 for x in rng.integers(-20, 60, len(ms))]
    with omap.Batch([(to_dev(m.occ), m.sources, m.targets) for m in ms], temporal_depth=T,
                    tile_rows=tile_rows, schedule=schedule, round_launch=launch) as b:
        infos = b.propagate(layers)
        acts = [b.activity(i).cpu().numpy() for i in range(len(ms))]
        ln, off, cells = (t.cpu().numpy() for t in b.paths())
    per = _split(ln, off, cells, [len(m.targets) for m in ms])
    for i, m in enumerate(ms):
        A, L, rl, ro, rc = oracle_solution(m, layers[i])
        assert infos[i]["layers"] == L, (i, infos[i], L)
        assert np.array_equal(acts[i], A), (i, m.name)
        assert np.array_equal(per[i][0], rl) and np.array_equal(per[i][1], ro), i
        assert np.array_equal(per[i][2], rc), i


def test_batch_equals_alone_and_auto_default():
    import paper_2004_00540_amd as omap
    ms = _batch_mazes(10, 77, hmax=500)
    with omap.Batch([(to_dev(m.occ), m.sources, m.targets) for m in ms]) as b:
        infos = b.propagate()
        acts = [b.activity(i).cpu().numpy() for i in range(len(ms))]
        ln, off, cells = (t.cpu().numpy() for t in b.paths())
    per = _split(ln, off, cells, [len(m.targets) for m in ms])
    for i, m in enumerate(ms):
        act, l1, o1, c1, info = run_plan(m, -1)
        assert infos[i]["layers"] == info["layers"]
        assert infos[i]["reached_cells"] == info["reached_cells"]
        assert np.array_equal(acts[i], act)
        assert np.array_equal(per[i][0], l1) and np.array_equal(per[i][1], o1)
        assert np.array_equal(per[i][2], c1)


def test_config4_subset_batched():
    import paper_2004_00540_amd as omap
    params = workloads.config4_params()
    idx = [0, 1, 2, 3, 100, 511]
    ms = [workloads.config4_maze(i, params) for i in idx]
    with omap.Batch([(to_dev(m.occ), m.sources, m.targets) for m in ms]) as b:
        infos = b.propagate()
        ln, off, cells = (t.cpu().numpy() for t in b.paths())
        acts = [b.activity(i).cpu().numpy() for i in range(len(ms))]
    per = _split(ln, off, cells, [len(m.targets) for m in ms])
    for i, m in enumerate(ms):
        A, L, rl, ro, rc = oracle_solution(m, -1, closed_form=True)
        assert infos[i]["layers"] == L
        assert np.array_equal(acts[i], A)
        assert np.array_equal(per[i][0], rl) and np.array_equal(per[i][2], rc)


def test_engine_results_alone_equal_mixed():
    import paper_2004_00540_amd as omap
    ms = _batch_mazes(30, 91, hmax=400)
    layers = [-1 if i % 3 else 25 for i in range(len(ms))]
    alone = {}
    for i, m in enumerate(ms):
        act, ln, off, cells, info = run_plan(m, layers[i])
        alone[i] = (ln, off, cells, info, act)
    with omap.Engine(256 << 20, max_slots=7, temporal_depth=8, tile_rows=32) as eng:
        ids = {}
        pending = list(range(len(ms)))
        done, acts = {}, {}
        step = 0
        while len(done) < len(ms):
            # staggered arrivals: a few new queries every step while others run
            for _ in range(3):
                if pending:
                    i = pending.pop(0)
                    ids[eng.submit(ms[i].occ, ms[i].sources, ms[i].targets, layers[i],
                                   keep_activity=i % 2 == 0)] = i
            eng.step(rounds=1 + step % 3)
            step += 1
            for q, i in list(ids.items()):
                if eng.poll(q) == omap.QUERY_DONE:
                    if i % 2 == 0:
                        acts[i] = eng.activity(q)
                    else:
                        with pytest.raises(omap.OmapError) as e:
                            eng.activity(q)
                        assert e.value.name == "OMAP_ERR_INVALID_ARG"
                    done[i] = eng.fetch(q)
                    del ids[q]
            assert step < 100000
    for i in range(len(ms)):
        ln, off, cells, info, act = alone[i]
        if i % 2 == 0:
            assert np.array_equal(acts[i], act), i
        r = done[i]
        assert np.array_equal(r.lengths, ln), i
        assert np.array_equal(r.offsets, off), i
        assert np.array_equal(r.cells, cells), i
        assert r.info["layers"] == info["layers"] and r.info["reached_cells"] == info["reached_cells"], i


def test_engine_completed_ids():
    """omap_engine_completed hands out every finished query once, failed ones
    included, in the order they finished."""
    import paper_2004_00540_amd as omap
    ms = _batch_mazes(9, 404, hmax=200)
    bad = ms[4].occ.copy()
    bad[ms[4].sources[0, 0], ms[4].sources[0, 1]] = 1
    with omap.Engine(128 << 20, max_slots=3) as eng:
        ids = [eng.submit(bad if i == 4 else m.occ, m.sources, m.targets) for i, m in enumerate(ms)]
        seen = []
        n = 0
        while len(seen) < len(ms):
            eng.step(rounds=2)
            got = eng.completed()
            for q in got:
                assert eng.poll(q) in (omap.QUERY_DONE, omap.QUERY_FAILED)
            seen += got
            n += 1
            assert n < 100000
        assert sorted(seen) == sorted(ids) and len(set(seen)) == len(seen)
        assert eng.completed() == []
        assert eng.poll(ids[4]) == omap.QUERY_FAILED
        for i, q in enumerate(ids):
            if i == 4:
                with pytest.raises(omap.OmapError):
                    eng.fetch(q)
            else:
                r = eng.fetch(q)
                assert r.info["layers"] == run_plan(ms[i], -1)[4]["layers"], i


def test_engine_memory_admission_and_errors():
    import paper_2004_00540_amd as omap
    big = workloads.random_maze(1500, 1500, 0.3, 1, 5, 5)
    small = workloads.random_maze(60, 60, 0.3, 1, 5, 6)
    with omap.Engine(32 << 20, max_slots=4) as eng:     # room for one big maze at a time
        qa = eng.submit(big.occ, big.sources, big.targets)
        qb = eng.submit(big.occ, big.sources, big.targets)
        qc = eng.submit(small.occ, small.sources, small.targets)
        eng.step(rounds=1)
        assert eng.poll(qa) == omap.QUERY_RUNNING
        assert eng.poll(qb) == omap.QUERY_QUEUED       # waits for memory (FIFO)
        with pytest.raises(omap.OmapError) as e:
            eng.fetch(qb)
        assert e.value.name == "OMAP_ERR_BUSY"
        with pytest.raises(omap.OmapError) as e:
            eng.submit(np.zeros((9000, 9000), np.uint8), [[0, 0]], [])
        assert e.value.name == "OMAP_ERR_OUT_OF_MEMORY"
        bad = small.occ.copy()
        bad[0, 0] = 1
        qd = eng.submit(bad, [[0, 0]], [[1, 1]])
        n = 0
        while any(eng.poll(q) not in (omap.QUERY_DONE, omap.QUERY_FAILED) for q in (qa, qb, qc, qd)):
            eng.step(rounds=4)
            n += 1
            assert n < 100000
        assert eng.poll(qd) == omap.QUERY_FAILED
        with pytest.raises(omap.OmapError) as e:
            eng.fetch(qd)
        assert e.value.name == "OMAP_ERR_SOURCE_ON_OBSTACLE"
        ref = run_plan(big, -1)
        for q in (qa, qb):
            r = eng.fetch(q)
            assert np.array_equal(r.cells, ref[3]) and np.array_equal(r.lengths, ref[1])
        assert eng.fetch(qc).info["layers"] == run_plan(small, -1)[4]["layers"]
        with pytest.raises(omap.OmapError) as e:
            eng.poll(qa)
        assert e.value.name == "OMAP_ERR_NOT_FOUND"


def test_batch_source_on_obstacle_names_the_maze():
    import paper_2004_00540_amd as omap
    ms = _batch_mazes(5, 123, hmax=60)
    occ = ms[3].occ.copy()
    occ[ms[3].sources[0, 0], ms[3].sources[0, 1]] = 1
    items = [(to_dev(m.occ if i != 3 else occ), m.sources, m.targets) for i, m in enumerate(ms)]
    with pytest.raises(omap.OmapError) as e:
        omap.Batch(items)
    assert e.value.name == "OMAP_ERR_SOURCE_ON_OBSTACLE" and "(maze 3)" in str(e.value)
