"""Checks that pin the CPU oracle to facts outside itself.

Each ``check_*`` takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with what the paper states, with a closed form, with an
independent textbook algorithm (Floyd-Warshall), or with brute-force search.
``test_oracle_pins`` runs them on the real oracle; ``test_oracle_mutants`` runs
them on copies of the oracle with planted mistakes and expects a failure.

Nothing here calls the GPU library.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NB = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]


def paper_facts() -> dict:
    with open(os.path.join(GOLDEN, "paper_facts.json")) as f:
        return json.load(f)


# ---- independent helpers (no oracle code) ------------------------------------

def chebyshev_to_sources(H, W, sources):
    r = np.arange(H)[:, None]
    c = np.arange(W)[None, :]
    d = np.full((H, W), 1 << 30, dtype=np.int64)
    for (sr, sc) in np.asarray(sources).reshape(-1, 2):
        d = np.minimum(d, np.maximum(np.abs(r - sr), np.abs(c - sc)))
    return d


def floyd_warshall(occ_batch: np.ndarray) -> np.ndarray:
    """All-pairs 8-neighbour step distances for a batch of grids (Floyd 1962).
    occ_batch: (B, h, w) uint8, 1 = obstacle.  Returns (B, n, n) int64 with a
    large value for 'no path'; obstacle cells have no path to or from anything
    (including themselves)."""
    B, h, w = occ_batch.shape
    n = h * w
    INF = 1 << 40
    D = np.full((B, n, n), INF, dtype=np.int64)
    free = occ_batch.reshape(B, n) == 0
    idx = np.arange(n)
    D[:, idx, idx] = np.where(free, 0, INF)
    for i in range(n):
        ri, ci = divmod(i, w)
        for dr, dc in NB:
            rj, cj = ri + dr, ci + dc
            if 0 <= rj < h and 0 <= cj < w:
                j = rj * w + cj
                D[:, i, j] = np.where(free[:, i] & free[:, j], 1, INF)
    for k in range(n):
        D = np.minimum(D, D[:, :, k:k + 1] + D[:, k:k + 1, :])
    return D


def fw_source_distance(occ, sources):
    """Multi-source distance from Floyd-Warshall, -1 = no path."""
    H, W = occ.shape
    D = floyd_warshall(occ[None].astype(np.uint8))[0]
    best = np.full(H * W, 1 << 40, dtype=np.int64)
    for (sr, sc) in np.asarray(sources).reshape(-1, 2):
        best = np.minimum(best, D[sr * W + sc])
    best = np.where(best >= (1 << 40), -1, best)
    return best.reshape(H, W)


def flood_reachable(occ, sources):
    """Set of free cells 8-connected to a free source (plain flood fill)."""
    H, W = occ.shape
    seen = set()
    stack = [tuple(s) for s in np.asarray(sources).reshape(-1, 2) if not occ[s[0], s[1]]]
    seen.update(stack)
    while stack:
        r, c = stack.pop()
        for dr, dc in NB:
            rr, cc = r + dr, c + dc
            if 0 <= rr < H and 0 <= cc < W and not occ[rr, cc] and (rr, cc) not in seen:
                seen.add((rr, cc))
                stack.append((rr, cc))
    return seen


def brute_lex_shortest_path(occ, sources, t, max_steps, budget=2_000_000):
    """Iterative-deepening depth-first search over simple 8-neighbour paths from
    t to any source, neighbours tried in the fixed order; the Chebyshev distance
    to the nearest source bounds the remaining steps from below.  The first path
    found at the smallest depth is the lexicographically first shortest path.
    Returns the list of cells, None if no path within max_steps, or 'budget'."""
    H, W = occ.shape
    srcset = {tuple(s) for s in np.asarray(sources).reshape(-1, 2)}
    cheb = chebyshev_to_sources(H, W, sources)
    t = tuple(t)
    if occ[t]:
        return None
    nodes = [0]

    def dfs(p, rem, path, onpath):
        nodes[0] += 1
        if nodes[0] > budget:
            raise TimeoutError
        if rem == 0:
            return p in srcset
        if p in srcset:
            return False          # a source earlier on the path would be closer
        if cheb[p] > rem:
            return False
        for dr, dc in NB:
            q = (p[0] + dr, p[1] + dc)
            if not (0 <= q[0] < H and 0 <= q[1] < W) or occ[q] or q in onpath:
                continue
            path.append(q)
            onpath.add(q)
            if dfs(q, rem - 1, path, onpath):
                return True
            path.pop()
            onpath.discard(q)
        return False

    try:
        for k in range(0, max_steps + 1):
            path = [t]
            if dfs(t, k, path, {t}):
                return path
    except TimeoutError:
        return "budget"
    return None


def maze_cases(n, seed, hmax=24, pmax=0.7):
    rng = np.random.default_rng(seed)
    for i in range(n):
        H = int(rng.integers(1, hmax + 1))
        W = int(rng.integers(1, hmax + 1))
        p = float(rng.uniform(0.0, pmax))
        ns = int(rng.integers(1, 5))
        nt = int(rng.integers(0, 9))
        yield workloads.random_maze(H, W, p, ns, nt, seed * 100003 + i)


# ---- checks -------------------------------------------------------------------

def check_layer_one_facts(o):
    """Sec. Methods worked example: after layer 1 the source holds 2, its free
    neighbours 1, obstacles 0, all other cells 0."""
    f = paper_facts()["layer_one"]
    occ = np.zeros((9, 9), np.uint8)
    for rc in [(3, 3), (3, 4), (5, 5), (0, 0), (8, 8), (4, 6), (2, 5)]:
        occ[rc] = 1
    src = (4, 4)
    A, n = o.layers(occ, [src], 1)
    assert n == 1
    for r in range(9):
        for c in range(9):
            if (r, c) == src:
                want = f["source"]
            elif occ[r, c]:
                want = f["obstacle"]
            elif max(abs(r - 4), abs(c - 4)) == 1:
                want = f["free_neighbour"]
            else:
                want = f["elsewhere"]
            assert A[r, c] == want, (r, c, A[r, c], want)


def check_source_value(o, n_cases=12):
    """Sec. Methods: sources hold n+1 after layer n and nothing is larger;
    obstacles are 0 after the rectifier."""
    off = paper_facts()["source_value"]["offset"]
    for m in maze_cases(n_cases, 11, hmax=16):
        for n in range(0, 13):
            A, used = o.layers(m.occ, m.sources, n)
            assert used == n
            s = m.sources
            assert (A[s[:, 0], s[:, 1]] == n + off).all()
            assert A.max() == n + off
            assert (A[m.occ == 1] == 0).all()


def check_empty_chebyshev(o):
    """Sec. 'oMAP versus Dijkstra': uniform step cost gives the square pattern on
    an empty map, i.e. A_L = max(0, L+1 - Chebyshev distance to the nearest
    source); the run-time determined L is the largest such distance."""
    rng = np.random.default_rng(5)
    for _ in range(10):
        H, W = int(rng.integers(1, 20)), int(rng.integers(1, 20))
        k = int(rng.integers(1, 4))
        src = np.stack([rng.integers(0, H, k), rng.integers(0, W, k)], 1)
        occ = np.zeros((H, W), np.uint8)
        cheb = chebyshev_to_sources(H, W, src)
        for L in (0, 1, 3, 7, 20):
            A, _ = o.layers(occ, src, L)
            assert (A == np.maximum(0, L + 1 - cheb)).all(), (H, W, L)
        A, Ls = o.layers(occ, src, -1)
        assert Ls == cheb.max()
        assert (A == Ls + 1 - cheb).all()


def check_centre_half_n(o):
    """Sec. 'Run-time': with the source in the middle of an empty square, the
    longest path is half the side."""
    f = paper_facts()["centre_source_longest_path"]
    for n, want in zip(f["odd_sides"], f["expected_steps"]):
        occ = np.zeros((n, n), np.uint8)
        _, Ls = o.layers(occ, [(n // 2, n // 2)], -1)
        assert Ls == want, (n, Ls, want)


def check_bfs_floyd_warshall(o, n_cases=60):
    """BFS distances equal Floyd-Warshall shortest paths on grids of <= 64 cells."""
    rng = np.random.default_rng(7)
    for i in range(n_cases):
        H, W = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        m = workloads.random_maze(H, W, float(rng.uniform(0, 0.6)), int(rng.integers(1, 4)), 0, 900 + i)
        d, ecc = o.bfs(m.occ, m.sources)
        ref = fw_source_distance(m.occ, m.sources)
        assert (d == ref).all(), (H, W, i)
        assert ecc == max(0, int(ref.max()))


def check_bfs_exhaustive(o, four_by_four=True):
    """Every 3x3 obstacle mask with every free cell as the source, and every 4x4
    mask with its first free cell as the source: BFS == Floyd-Warshall."""
    masks3 = np.array([[(b >> i) & 1 for i in range(9)] for b in range(512)], np.uint8).reshape(512, 3, 3)
    D3 = floyd_warshall(masks3)
    for b in range(512):
        occ = masks3[b]
        for s in range(9):
            if occ.flat[s]:
                continue
            d, _ = o.bfs(occ, [divmod(s, 3)])
            ref = np.where(D3[b, s] >= (1 << 40), -1, D3[b, s]).reshape(3, 3)
            assert (d == ref).all(), (b, s)
    if not four_by_four:
        return
    masks4 = ((np.arange(1 << 16)[:, None] >> np.arange(16)[None, :]) & 1).astype(np.uint8).reshape(-1, 4, 4)
    D4 = floyd_warshall(masks4)
    for b in range(1 << 16):
        occ = masks4[b]
        free = np.flatnonzero(occ.ravel() == 0)
        if len(free) == 0:
            continue
        s = int(free[0])
        d, _ = o.bfs(occ, [divmod(s, 4)])
        ref = D4[b, s]
        ref = np.where(ref >= (1 << 40), -1, ref).reshape(4, 4)
        assert (d == ref).all(), b


def check_layers_vs_bfs(o, n_cases=80):
    """The network output equals max(0, L+1-d) with d from BFS, for fixed L below,
    at and above the eccentricity, and the run-time determined L* equals the
    eccentricity; the closed-form helper agrees."""
    for m in maze_cases(n_cases, 3):
        d, ecc = o.bfs(m.occ, m.sources)
        for L in sorted({0, 1, max(ecc - 1, 0), ecc, ecc + 5}):
            A, used = o.layers(m.occ, m.sources, L)
            ref = np.where((d >= 0) & (d <= L), L + 1 - d, 0)
            assert (A == ref).all(), (m.name, L)
            assert (o.activity_from_bfs(d, L) == ref).all()
        A, Ls = o.layers(m.occ, m.sources, -1)
        assert Ls == ecc, (m.name, Ls, ecc)
        assert (A == np.where(d >= 0, ecc + 1 - d, 0)).all()


def check_more_sources_fewer_layers(o, n_cases=30):
    """Adding sources inside the reached region never increases L*."""
    rng = np.random.default_rng(13)
    for m in maze_cases(n_cases, 17, hmax=20, pmax=0.45):
        _, L1 = o.layers(m.occ, m.sources, -1)
        reach = sorted(flood_reachable(m.occ, m.sources))
        extra = [reach[int(i)] for i in rng.integers(0, len(reach), 3)]
        _, L2 = o.layers(m.occ, np.concatenate([m.sources, np.array(extra, np.int32)]), -1)
        assert L2 <= L1, (m.name, L1, L2)


def check_walk_bruteforce(o, n_cases=200, hmax=8):
    """On grids up to 8x8 the walk returns exactly the lexicographically first
    (by neighbour order) shortest path found by exhaustive search, and -1 when
    exhaustive search finds no path.  A designed part puts one obstacle in a
    5x5 grid at every position, which creates ties between every pair of
    neighbour directions."""
    checked = 0
    for src in [(0, 0), (2, 2), (4, 1)]:
        for ob in range(25):
            occ = np.zeros((5, 5), np.uint8)
            occ.flat[ob] = 1
            if occ[src]:
                continue
            tg = np.array([divmod(i, 5) for i in range(25)], np.int32)
            A, _ = o.layers(occ, [src], -1)
            ln, off, cells = o.walk(A, [src], tg)
            for k, t in enumerate(tg):
                got = [divmod(int(x), 5) for x in cells[off[k]:off[k + 1]]]
                ref = brute_lex_shortest_path(occ, [src], t, 25)
                if ref is None:
                    assert ln[k] == -1 and got == []
                else:
                    assert got == ref, (src, ob, tuple(t), got, ref)
    rng = np.random.default_rng(23)
    for i in range(n_cases):
        H, W = int(rng.integers(1, hmax + 1)), int(rng.integers(1, hmax + 1))
        m = workloads.random_maze(H, W, float(rng.uniform(0, 0.5)), int(rng.integers(1, 3)), 6, 4000 + i)
        A, Ls = o.layers(m.occ, m.sources, -1)
        ln, off, cells = o.walk(A, m.sources, m.targets)
        reach = flood_reachable(m.occ, m.sources)
        for k, t in enumerate(m.targets):
            got = [divmod(int(x), W) for x in cells[off[k]:off[k + 1]]]
            if tuple(t) not in reach:
                assert ln[k] == -1 and got == [], (m.name, k)
                continue
            ref = brute_lex_shortest_path(m.occ, m.sources, t, H * W)
            if ref == "budget":
                continue
            assert ref is not None
            assert ln[k] == len(ref) - 1, (m.name, k, ln[k], len(ref) - 1)
            assert got == ref, (m.name, k, got, ref)
            checked += 1
    assert checked >= n_cases  # most targets were decided by brute force


def _check_path_valid(occ, sources, path, steps):
    H, W = occ.shape
    srcset = {tuple(s) for s in np.asarray(sources).reshape(-1, 2)}
    assert len(path) == steps + 1
    for (r, c) in path:
        assert 0 <= r < H and 0 <= c < W and not occ[r, c]
    for a, b in zip(path, path[1:]):
        assert max(abs(a[0] - b[0]), abs(a[1] - b[1])) == 1
    assert path[-1] in srcset
    assert all(p not in srcset for p in path[:-1])


def check_walk_invariants(o, n_cases=60):
    """Every path is obstacle-free, 8-contiguous, starts at its target, ends on a
    source, climbs the activity by exactly 1 per step, and has as many steps as
    the target's BFS distance (Sec. 'Path Reconstruction'); targets with
    activity 0 get no path."""
    for m in maze_cases(n_cases, 29, hmax=32, pmax=0.5):
        d, ecc = o.bfs(m.occ, m.sources)
        for L in (-1, max(ecc // 2, 0)):
            A, Lu = o.layers(m.occ, m.sources, L)
            ln, off, cells = o.walk(A, m.sources, m.targets)
            assert off[0] == 0 and (np.diff(off) >= 0).all()
            for k, t in enumerate(m.targets):
                tr, tc = int(t[0]), int(t[1])
                if d[tr, tc] < 0 or d[tr, tc] > Lu:
                    assert ln[k] == -1 and off[k + 1] == off[k]
                    continue
                path = [divmod(int(x), m.W) for x in cells[off[k]:off[k + 1]]]
                assert path[0] == (tr, tc)
                assert ln[k] == d[tr, tc]
                _check_path_valid(m.occ, m.sources, path, int(ln[k]))
                vals = [A[p] for p in path]
                assert all(b == a + 1 for a, b in zip(vals, vals[1:]))


def check_source_on_obstacle_plateau(o):
    """Documents the reading that rejects sources on obstacles: the literal rule
    seeds the neighbours once from the input source map and then never lifts
    them, producing a plateau of 1s instead of a gradient."""
    occ = np.zeros((7, 7), np.uint8)
    occ[3, 3] = 1
    A, _ = o.layers(occ, [(3, 3)], 6)
    assert A[3, 3] == 0
    assert A.max() == 1
    assert (A[occ == 0] == 1).all()


def check_comb_bound(o):
    """Sec. 'Limitations': on serpentine (comb) mazes the run-time determined L
    stays below the paper's longest-path formula and below the free-cell count."""
    for n in (5, 7, 9, 11, 15):
        occ = np.zeros((n, n), np.uint8)
        for r in range(1, n, 2):
            occ[r, :] = 1
            occ[r, (n - 1) if (r // 2) % 2 == 0 else 0] = 0
        _, Ls = o.layers(occ, [(0, 0)], -1)
        formula = max(n, n) * ((n + 1) // 2) + n // 2
        assert Ls <= formula
        assert Ls <= int((occ == 0).sum()) - 1
        # corridors of length n joined by one-cell gaps: at least one full corridor
        # per two rows must be traversed
        assert Ls >= ((n + 1) // 2 - 1) * (n - 2)


def _octile(a, b):
    dr, dc = abs(a[0] - b[0]), abs(a[1] - b[1])
    return max(dr, dc) - min(dr, dc) + math.sqrt(2) * min(dr, dc)


def check_euclidean_walk(o, n_cases=40):
    """Euclidean path reconstruction: on an empty map the straightened path has
    the octile (shortest Euclidean 8-move) cost; in mazes every path is a valid
    8-contiguous path to a source whose cost is at least the octile distance to
    the nearest source.  (Optimality in mazes: parity unpinned.)"""
    rng = np.random.default_rng(31)
    for _ in range(10):
        H, W = int(rng.integers(2, 24)), int(rng.integers(2, 24))
        src = [(int(rng.integers(0, H)), int(rng.integers(0, W)))]
        occ = np.zeros((H, W), np.uint8)
        A, _ = o.layers(occ, src, -1)
        tg = np.stack([rng.integers(0, H, 6), rng.integers(0, W, 6)], 1)
        ln, off, cells = o.walk_euclidean(A, src, tg)
        for k, t in enumerate(tg):
            path = [divmod(int(x), W) for x in cells[off[k]:off[k + 1]]]
            cost = sum(_octile(a, b) for a, b in zip(path, path[1:]))
            assert abs(cost - _octile(tuple(t), src[0])) < 1e-9, (H, W, t, path)
    for m in maze_cases(n_cases, 37, hmax=24, pmax=0.4):
        A, Lu = o.layers(m.occ, m.sources, -1)
        ln, off, cells = o.walk_euclidean(A, m.sources, m.targets)
        srcset = {tuple(s) for s in m.sources}
        for k, t in enumerate(m.targets):
            if A[t[0], t[1]] == 0:
                assert ln[k] == -1
                continue
            path = [divmod(int(x), m.W) for x in cells[off[k]:off[k + 1]]]
            assert path[0] == tuple(t) and path[-1] in srcset
            for a, b in zip(path, path[1:]):
                assert max(abs(a[0] - b[0]), abs(a[1] - b[1])) == 1
            for p in path:
                assert not m.occ[p]
            cost = sum(_octile(a, b) for a, b in zip(path, path[1:]))
            assert cost >= min(_octile(tuple(t), s) for s in srcset) - 1e-9


def octile_dijkstra(occ, sources):
    """Shortest Euclidean 8-move distance to the nearest source (orthogonal
    step 1, diagonal step sqrt 2, diagonal steps between two obstacles allowed
    as in the 3x3 window): Dijkstra (1959) with a binary heap."""
    import heapq
    H, W = occ.shape
    D = np.full((H, W), np.inf)
    pq = []
    for s in np.asarray(sources).reshape(-1, 2):
        s = (int(s[0]), int(s[1]))
        D[s] = 0.0
        pq.append((0.0, s))
    heapq.heapify(pq)
    while pq:
        d, (r, c) = heapq.heappop(pq)
        if d > D[r, c]:
            continue
        for dr, dc in NB:
            rr, cc = r + dr, c + dc
            if 0 <= rr < H and 0 <= cc < W and not occ[rr, cc]:
                nd = d + (math.sqrt(2) if dr and dc else 1.0)
                if nd < D[rr, cc] - 1e-12:
                    D[rr, cc] = nd
                    heapq.heappush(pq, (nd, (rr, cc)))
    return D


def check_euclidean_literal_optimal(o, n_cases=180, min_literal=80):
    """Sec. "Path Reconstruction" states that the straightened path of the
    4-neighbour climb (Eq. 1) is shortest in Euclidean distance.  Where the
    paper's rule applies as written -- every 4-neighbour move rises by one, so
    after straightening each orthogonal segment rises by 1 and each diagonal
    segment by 2 -- the oracle's path must cost exactly the octile Dijkstra
    distance and no more than the simple path of the same map.  (Paths that
    need the reading's sideways or 8-neighbour moves, where the paper's rule
    has no next cell, are only checked for validity; some of them cost more
    than the simple path.)"""
    literal = 0
    for m in maze_cases(n_cases, 1007, hmax=40, pmax=0.45):
        A, _ = o.layers(m.occ, m.sources, -1)
        D = octile_dijkstra(m.occ, m.sources)
        l1, o1, c1 = o.walk(A, m.sources, m.targets)
        l2, o2, c2 = o.walk_euclidean(A, m.sources, m.targets)
        for k, t in enumerate(m.targets):
            if l1[k] < 0:
                assert l2[k] == -1
                continue
            p1 = [divmod(int(x), m.W) for x in c1[o1[k]:o1[k + 1]]]
            p2 = [divmod(int(x), m.W) for x in c2[o2[k]:o2[k + 1]]]
            rises = [int(A[b] - A[a]) - (2 if (a[0] != b[0] and a[1] != b[1]) else 1) for a, b in zip(p2, p2[1:])]
            if any(rises):
                continue
            literal += 1
            cost = sum(_octile(a, b) for a, b in zip(p2, p2[1:]))
            simple = sum(_octile(a, b) for a, b in zip(p1, p1[1:]))
            assert abs(cost - D[t[0], t[1]]) < 1e-9, (m.name, tuple(t), cost, D[t[0], t[1]])
            assert cost <= simple + 1e-9, (m.name, tuple(t), cost, simple)
    assert literal >= min_literal, literal


def check_tie_hash_vectors(o):
    """The tie-break hash is SplitMix64's output function: from state 0 the
    published generator yields the three reference values."""
    with open(os.path.join(GOLDEN, "splitmix64.json")) as f:
        g = json.load(f)
    outs = [int(x, 16) for x in g["state0_outputs_hex"]]
    inc = int(g["increment_hex"], 16)
    state = 0
    for want in outs:
        assert o.tie_hash(state, 0, 0) == want          # output after one increment from `state`
        state = (state + inc) & 0xFFFFFFFFFFFFFFFF
    # target and step enter as (target << 32) ^ step
    assert o.tie_hash(5, 3, 7) == o.tie_hash(5 ^ (3 << 32) ^ 7, 0, 0)


def check_walk_random(o, n_cases=40):
    """Random ties (Sec. 'Path Reconstruction'): every path is a shortest path
    (valid, climbs by one per step, steps = BFS distance), the same seed gives
    the same path, and where three neighbours tie the choice is spread evenly."""
    for m in maze_cases(n_cases, 41, hmax=28, pmax=0.45):
        d, _ = o.bfs(m.occ, m.sources)
        A, _ = o.layers(m.occ, m.sources, -1)
        for seed in (0, 1, 12345):
            ln, off, cells = o.walk_random(A, m.sources, m.targets, seed)
            l2, o2, c2 = o.walk_random(A, m.sources, m.targets, seed)
            assert np.array_equal(cells, c2) and np.array_equal(ln, l2)
            for k, t in enumerate(m.targets):
                tr, tc = int(t[0]), int(t[1])
                if d[tr, tc] < 0:
                    assert ln[k] == -1
                    continue
                path = [divmod(int(x), m.W) for x in cells[off[k]:off[k + 1]]]
                assert path[0] == (tr, tc) and ln[k] == d[tr, tc]
                _check_path_valid(m.occ, m.sources, path, int(ln[k]))
                vals = [A[p] for p in path]
                assert all(b == a + 1 for a, b in zip(vals, vals[1:]))
    occ = np.zeros((9, 9), np.uint8)
    A, _ = o.layers(occ, [(0, 0)], -1)
    counts = {}
    for seed in range(300):
        ln, off, cells = o.walk_random(A, [(0, 0)], [(4, 8)], seed)
        first = divmod(int(cells[1]), 9)
        counts[first] = counts.get(first, 0) + 1
    assert set(counts) == {(3, 7), (4, 7), (5, 7)}
    assert all(60 <= c <= 140 for c in counts.values()), counts


ALL_CHECKS = [
    check_layer_one_facts,
    check_source_value,
    check_empty_chebyshev,
    check_centre_half_n,
    check_bfs_floyd_warshall,
    check_bfs_exhaustive,
    check_layers_vs_bfs,
    check_more_sources_fewer_layers,
    check_walk_bruteforce,
    check_walk_invariants,
    check_source_on_obstacle_plateau,
    check_comb_bound,
    check_euclidean_walk,
    check_euclidean_literal_optimal,
    check_tie_hash_vectors,
    check_walk_random,
]
