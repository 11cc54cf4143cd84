"""Parity at the full workload sizes, in the configuration bench.py times
(default options, run-time L): the 23170^2 maze, all 512 batched mazes and a
sample of serving queries.  Activity maps are compared with the oracle's BFS
closed form (pinned to the literal network by the CPU tests), paths with the
oracle's walk on that map."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_config3_full_size():
    import torch
    import paper_2004_00540_amd as omap
    m = workloads.config3()
    d, ecc = oracle.bfs(m.occ, m.sources)
    print(f"config3: ecc {ecc}", flush=True)
    with omap.Plan(to_dev(m.occ), m.sources, m.targets) as plan:
        info = plan.propagate()
        act = plan.activity()
        ln, off, cells = (t.cpu().numpy() for t in plan.paths())
        assert info["layers"] == ecc
        # compare the whole map row band by row band (int32 closed form: ecc + 1 - d)
        dd = torch.from_numpy(d)
        for r0 in range(0, m.H, 2048):
            want = torch.where(dd[r0:r0 + 2048] >= 0, ecc + 1 - dd[r0:r0 + 2048], torch.zeros((), dtype=torch.int32))
            got = act[r0:r0 + 2048].cpu()
            assert torch.equal(got, want.to(torch.int32)), f"rows {r0}.."
        assert info["reached_cells"] == int((d >= 0).sum())
    del act
    A = oracle.activity_from_bfs(d, ecc)
    rl, ro, rc = oracle.walk(A, m.sources, m.targets)
    assert np.array_equal(ln, rl) and np.array_equal(off, ro) and np.array_equal(cells, rc)


def test_config4_all_512_batched():
    import paper_2004_00540_amd as omap
    ms = workloads.config4()
    with omap.Batch([(to_dev(m.occ), m.sources, m.targets) for m in ms]) as b:
        infos = b.propagate()
        ln, off, cells = (t.cpu().numpy() for t in b.paths())
        t0 = 0
        for i, m in enumerate(ms):
            d, ecc = oracle.bfs(m.occ, m.sources)
            assert infos[i]["layers"] == ecc, i
            act = b.activity(i).cpu().numpy()   # every maze's full activity map
            assert np.array_equal(act, np.where(d >= 0, ecc + 1 - d, 0)), i
            A = oracle.activity_from_bfs(d, ecc)
            rl, ro, rc = oracle.walk(A, m.sources, m.targets)
            n = len(m.targets)
            assert np.array_equal(ln[t0:t0 + n], rl), i
            assert np.array_equal(off[t0:t0 + n + 1] - off[t0], ro), i
            assert np.array_equal(cells[off[t0]:off[t0 + n]], rc), i
            t0 += n


def test_serving_queries_sample():
    """Served queries (the serving workload's first ten): every activity map
    and every path against the oracle."""
    import paper_2004_00540_amd as omap
    import torch
    qs = [workloads.serve_query(i) for i in range(10)]
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(8 << 30, free // 2))
    print(f"free device memory {free / 2**30:.1f} GiB, engine budget {budget / 2**30:.1f} GiB", flush=True)
    with omap.Engine(budget, max_slots=16) as eng:
        ids = {eng.submit(q.occ, q.sources, q.targets, keep_activity=True): k for k, q in enumerate(qs)}
        res, act = {}, {}
        n = 0
        while len(res) < len(qs):
            eng.step(rounds=8)
            for qid, k in list(ids.items()):
                if eng.poll(qid) == omap.QUERY_DONE:
                    act[k] = eng.activity(qid)
                    res[k] = eng.fetch(qid)
                    del ids[qid]
            n += 1
            assert n < 1000000
    for k, q in enumerate(qs):
        d, ecc = oracle.bfs(q.occ, q.sources)
        A = oracle.activity_from_bfs(d, ecc)
        rl, ro, rc = oracle.walk(A, q.sources, q.targets)
        assert res[k].info["layers"] == ecc, q.name
        assert np.array_equal(act[k], A), q.name
        assert np.array_equal(res[k].lengths, rl) and np.array_equal(res[k].offsets, ro), q.name
        assert np.array_equal(res[k].cells, rc), q.name


def test_maximum_size_empty_map():
    """The largest grid the boundary accepts (46340^2 = 2,147,395,600 cells <
    2^31): an empty map with a corner source, checked against the closed form
    A(r, c) = L + 1 - max(r, c) with L = n - 1 (the Chebyshev distance; the CPU
    tests pin the layers to it), on whole rows and columns and a seeded sample,
    and paths whose shape follows from the fixed tie order."""
    import torch
    import paper_2004_00540_amd as omap
    n = 46340
    assert n * n < 2 ** 31
    occ = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    tgt = np.array([[n - 1, n - 1], [n - 1, 0], [0, n - 1], [12345, 30000], [0, 0]], np.int32)
    with omap.Plan(occ, np.array([[0, 0]], np.int32), tgt) as plan:
        info = plan.propagate()
        print(f"max size: {info}", flush=True)
        assert info["layers"] == n - 1
        assert info["reached_cells"] == n * n
        act = plan.activity()
        idx = torch.arange(n, device="cuda", dtype=torch.int64)
        assert torch.equal(act[0, :].long(), n - idx)
        assert torch.equal(act[:, 0].long(), n - idx)
        assert torch.equal(act[n - 1, :].long(), torch.ones(n, dtype=torch.int64, device="cuda"))
        assert torch.equal(act[:, n - 1].long(), torch.ones(n, dtype=torch.int64, device="cuda"))
        g = torch.Generator(device="cpu").manual_seed(46340)
        r = torch.randint(0, n, (200000,), generator=g).cuda()
        c = torch.randint(0, n, (200000,), generator=g).cuda()
        assert torch.equal(act[r, c].long(), n - torch.maximum(r, c))
        del act
        torch.cuda.empty_cache()
        ln, off, cells = (t.cpu().numpy() for t in plan.paths())
    assert list(ln) == [n - 1, n - 1, n - 1, 30000, 0]
    k = np.arange(n, dtype=np.int64)
    # (n-1, n-1): the first maximal neighbour is the up-left diagonal
    assert np.array_equal(cells[off[0]:off[1]], (n - 1 - k) * n + (n - 1 - k))
    # (n-1, 0): straight up column 0; (0, n-1): straight left along row 0
    assert np.array_equal(cells[off[1]:off[2]], (n - 1 - k) * n)
    assert np.array_equal(cells[off[2]:off[3]], n - 1 - k)
    # (12345, 30000): diagonal until row 0, then left
    d = np.arange(12346, dtype=np.int64)
    left = np.arange(1, 30000 - 12345 + 1, dtype=np.int64)
    want = np.concatenate([(12345 - d) * n + (30000 - d), 30000 - 12345 - left])
    assert np.array_equal(cells[off[3]:off[4]], want)
    assert np.array_equal(cells[off[4]:off[5]], [0])
