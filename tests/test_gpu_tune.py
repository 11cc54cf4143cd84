"""The autotuner (omap_tune): it times the candidates, checks each one's maps
against the defaults', returns options that reproduce the oracle's results,
and reads a cached choice back without timing."""
import os

import numpy as np
import pytest

import workloads
from gpu_helpers import assert_same, oracle_solution, run_plan, to_dev

pytestmark = pytest.mark.gpu


def _mazes(n, seed):
    rng = np.random.default_rng(seed)
    return [workloads.random_maze(int(rng.integers(60, 400)), int(rng.integers(60, 500)),
                                  float(rng.uniform(0.2, 0.45)), int(rng.integers(1, 6)), 20, seed * 100 + i)
            for i in range(n)]


def test_tune_batch_and_cache(tmp_path, monkeypatch):
    import paper_2004_00540_amd as omap
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("OMAP_TUNE_CACHE", str(cache))
    ms = _mazes(12, 5)
    items = [(to_dev(m.occ), m.sources, m.targets) for m in ms]
    r = omap.tune(items, omap.USE_BATCH)
    assert r["from_cache"] == 0 and r["candidates"] >= 8
    assert 0 < r["best_ms"] <= r["default_ms"]
    assert cache.read_text().count("use1") == 1
    opts = r["options"]
    omap.resolve_options(**opts)                 # a valid option set
    with omap.Batch(items, **opts) as b:
        infos = b.propagate()
        acts = [b.activity(i).cpu().numpy() for i in range(len(ms))]
    for i, m in enumerate(ms):
        A, L, *_ = oracle_solution(m, -1)
        assert infos[i]["layers"] == L and np.array_equal(acts[i], A), i
    again = omap.tune(items, omap.USE_BATCH)
    assert again["from_cache"] == 1 and again["candidates"] == 0 and again["options"] == opts


def test_tune_plan_and_engine(tmp_path, monkeypatch):
    import paper_2004_00540_amd as omap
    monkeypatch.delenv("OMAP_TUNE_CACHE", raising=False)
    m = workloads.random_maze(500, 700, 0.33, 3, 40, 77)
    r = omap.tune([(to_dev(m.occ), m.sources, m.targets)], omap.USE_PLAN)
    assert r["from_cache"] == 0 and r["candidates"] >= 8
    assert_same(m, run_plan(m, -1, **r["options"]), oracle_solution(m, -1), f"tuned plan {r['options']}")
    ms = _mazes(6, 9)
    e = omap.tune([(to_dev(q.occ), q.sources, q.targets) for q in ms], omap.USE_ENGINE)
    with omap.Engine(256 << 20, max_slots=4, **e["options"]) as eng:
        ids = {eng.submit(q.occ, q.sources, q.targets): k for k, q in enumerate(ms)}
        done = {}
        n = 0
        while len(done) < len(ms):
            eng.step(rounds=4)
            for qid, k in list(ids.items()):
                if eng.poll(qid) == omap.QUERY_DONE:
                    done[k] = eng.fetch(qid)
                    del ids[qid]
            n += 1
            assert n < 100000
    for k, q in enumerate(ms):
        A, L, rl, ro, rc = oracle_solution(q, -1)
        assert done[k].info["layers"] == L and np.array_equal(done[k].cells, rc), k


def test_tune_rejects_bad_arguments():
    import paper_2004_00540_amd as omap
    m = workloads.random_maze(20, 20, 0.2, 1, 2, 3)
    items = [(to_dev(m.occ), m.sources, m.targets)] * 2
    with pytest.raises(omap.OmapError) as e:
        omap.tune(items, omap.USE_PLAN)          # a plan has one maze
    assert e.value.name == "OMAP_ERR_INVALID_ARG"
    with pytest.raises(omap.OmapError):
        omap.tune(items, 7)
