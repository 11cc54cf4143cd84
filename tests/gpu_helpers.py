"""Shared helpers of the GPU tests: run a maze through the library's C ABI and
compute the oracle's answer for the same seeded input."""
import numpy as np

import oracle


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_plan(m, layers, **opts):
    import paper_2004_00540_amd as omap
    with omap.Plan(to_dev(m.occ), m.sources, m.targets, **opts) as plan:
        info = plan.propagate(layers)
        act = plan.activity().cpu().numpy()
        ln, off, cells = (t.cpu().numpy() for t in plan.paths())
    return act, ln, off, cells, info


def oracle_solution(m, layers, closed_form=False):
    """Activity map and paths from the oracle.  closed_form=True uses the BFS
    closed form (pinned to the literal network) for inputs too large for it."""
    if closed_form:
        d, ecc = oracle.bfs(m.occ, m.sources)
        L = ecc if layers < 0 else layers
        A = oracle.activity_from_bfs(d, L)
    else:
        A, L = oracle.layers(m.occ, m.sources, layers)
    ln, off, cells = oracle.walk(A, m.sources, m.targets)
    return A, L, ln, off, cells


def assert_same(m, got, ref, where=""):
    act, ln, off, cells, info = got
    A, L, rl, ro, rc = ref
    assert info["layers"] == L, (where, info, L)
    if not np.array_equal(act, A):
        bad = np.argwhere(act != A)
        r, c = bad[0]
        raise AssertionError(f"{where}: activity differs at {len(bad)} cells, first ({r},{c}): "
                             f"got {act[r, c]} want {A[r, c]}")
    assert np.array_equal(ln, rl), (where, ln, rl)
    assert np.array_equal(off, ro), where
    assert np.array_equal(cells, rc), where
    assert info["reached_cells"] == int((A > 0).sum()), where
