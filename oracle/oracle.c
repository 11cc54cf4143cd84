/*
 * CPU ORACLE for the oMAP maze planner -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct loops that restate what the paper computes.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library; the GPU library never links or calls it, and the two
 * share no code.
 *
 * Paper: Kulvicius, Herzog, Tamosiunaite, Woergoetter, "Generation of Paths in
 * a Maze using a Deep Network without Learning" (arXiv 2004.00540).
 *
 * Conventions (readings of the paper are marked READING):
 *   grid     H rows x W columns, row-major, cell (r, c) at r*W + c
 *   occ      uint8, nonzero = obstacle
 *   sources  (row, col) int32 pairs
 *   window   the 3x3 neighbourhood of a cell, clipped at the border
 *   8 neighbours in the fixed order k = 0..7:
 *            (-1,-1) (-1,0) (-1,+1) (0,-1) (0,+1) (+1,-1) (+1,0) (+1,+1)
 *
 * Functions and what pins them (the pins live in the test suite):
 *   oracle_layers          literal network; pinned by the paper's layer-1 and
 *                          source-value facts, the empty-map closed form and
 *                          the BFS distances below.
 *   oracle_bfs             textbook multi-source BFS; pinned by Floyd-Warshall
 *                          and exhaustive small masks in the tests.
 *   oracle_activity_from_bfs  the closed form max(0, L+1-d); pinned by
 *                          comparison with oracle_layers.
 *   oracle_walk            simple path reconstruction; pinned by brute-force
 *                          path enumeration on grids up to 8x8.
 *   oracle_walk_euclidean  Euclidean path reconstruction; parity unpinned by the
 *                          paper (no printed path); checked for validity and
 *                          cost against octile-distance bounds only.
 *   oracle_walk_random     simple reconstruction with the paper's random ties
 *                          (counter-based hash); pinned by path validity, step
 *                          count = BFS distance and the spread of choices.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAXINT 2147483647LL   /* "-maxint" of the environment map */

static const int NB_DR[8] = {-1, -1, -1, 0, 0, 1, 1, 1};
static const int NB_DC[8] = {-1, 0, 1, -1, 1, -1, 0, 1};

/* One network layer (Sec. Methods, "Activity Map Generation"; Fig. net):
 *   out(x) = ReLU( maxpool3x3(in)(x) + I_e(x) + I_s(x) )
 * Max pooling: 3x3 window, stride 1, zero padding, so window positions that
 * fall outside the grid contribute the value 0. */
static void layer(int32_t H, int32_t W, const int64_t *in, const int64_t *Ie, const int64_t *Is,
                  int64_t *out, int n_threads)
{
#pragma omp parallel for num_threads(n_threads) schedule(static)
    for (int32_t r = 0; r < H; ++r) {
        for (int32_t c = 0; c < W; ++c) {
            int64_t m = INT64_MIN;
            for (int dr = -1; dr <= 1; ++dr)
                for (int dc = -1; dc <= 1; ++dc) {
                    const int32_t rr = r + dr, cc = c + dc;
                    const int64_t v = (rr < 0 || rr >= H || cc < 0 || cc >= W)
                                          ? 0                       /* zero padding */
                                          : in[(int64_t)rr * W + cc];
                    if (v > m) m = v;
                }
            const int64_t x = (int64_t)r * W + c;
            const int64_t s = m + Ie[x] + Is[x];
            out[x] = s > 0 ? s : 0;                                 /* ReLU */
        }
    }
}

static int same_support(int64_t N, const int64_t *a, const int64_t *b)
{
    for (int64_t i = 0; i < N; ++i)
        if ((a[i] > 0) != (b[i] > 0)) return 0;
    return 1;
}

/* The oMAP network of L identical layers (Sec. Methods).
 *   Inputs (Sec. Methods, "Input"): I_s(x) = 1 at sources, else 0;
 *   I_e(x) = -maxint at obstacles, else 0.  The first layer pools the source
 *   map, so the activity before layer 1 is A_0 = I_s.
 *   out = A_L, in int64 (no overflow: |values| <= maxint + L + 1).
 *
 * max_layers >= 0: exactly that many layers.
 * max_layers <  0: the run-time determination of L (Sec. "Determining the
 *   number of layers L"): layers are added one at a time until the activity
 *   map stops gaining nonzero cells.  READING: the paper's rule "until no zero
 *   values remain except at obstacles" never ends when some free cell is
 *   unreachable; stopping when the set of nonzero cells no longer grows is the
 *   same rule when every free cell is reachable, and ends otherwise.  The map
 *   returned is the last one that gained cells, A_{L*}.
 *
 * Returns the number of layers applied (L or L*), or -1 on allocation failure. */
int64_t oracle_layers(int32_t H, int32_t W, const uint8_t *occ, const int32_t *src_rc,
                      int32_t n_src, int64_t max_layers, int64_t *out, int32_t n_threads)
{
    const int64_t N = (int64_t)H * W;
    if (n_threads < 1) n_threads = 1;
    int64_t *Ie = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *Is = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    if (!Ie || !Is || !tmp) { free(Ie); free(Is); free(tmp); return -1; }
    for (int64_t i = 0; i < N; ++i) Ie[i] = occ[i] ? -ORACLE_MAXINT : 0;
    for (int32_t k = 0; k < n_src; ++k) Is[(int64_t)src_rc[2 * k] * W + src_rc[2 * k + 1]] = 1;

    int64_t *a = out, *b = tmp;
    memcpy(a, Is, sizeof(int64_t) * (size_t)N);              /* A_0 = I_s */
    int64_t n = 0;
    if (max_layers >= 0) {
        for (n = 0; n < max_layers; ++n) {
            layer(H, W, a, Ie, Is, b, n_threads);
            int64_t *t = a; a = b; b = t;
        }
    } else {
        for (;;) {
            layer(H, W, a, Ie, Is, b, n_threads);
            if (same_support(N, a, b)) break;                /* A_{n+1} gained nothing */
            int64_t *t = a; a = b; b = t;
            ++n;
        }
    }
    if (a != out) memcpy(out, a, sizeof(int64_t) * (size_t)N);
    free(Ie);
    free(Is);
    free(tmp);
    return n;
}

/* Multi-source breadth-first search (Moore 1959), the algorithm the paper
 * relates the network to (Sec. "Path Reconstruction"): step distance through
 * free cells under the 8-neighbourhood, every move costing 1.  dist = -1 for
 * obstacles and unreachable cells.  Sources that sit on an obstacle are not
 * seeded (the plan API rejects them).  Returns the eccentricity (largest finite
 * distance), or -1 on allocation failure. */
int64_t oracle_bfs(int32_t H, int32_t W, const uint8_t *occ, const int32_t *src_rc, int32_t n_src,
                   int32_t *dist)
{
    const int64_t N = (int64_t)H * W;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!queue) return -1;
    for (int64_t i = 0; i < N; ++i) dist[i] = -1;
    int64_t head = 0, tail = 0;
    for (int32_t k = 0; k < n_src; ++k) {
        const int64_t x = (int64_t)src_rc[2 * k] * W + src_rc[2 * k + 1];
        if (occ[x] || dist[x] == 0) continue;
        dist[x] = 0;
        queue[tail++] = x;
    }
    int64_t ecc = 0;
    while (head < tail) {
        const int64_t x = queue[head++];
        const int32_t r = (int32_t)(x / W), c = (int32_t)(x % W);
        if (dist[x] > ecc) ecc = dist[x];
        for (int k = 0; k < 8; ++k) {
            const int32_t rr = r + NB_DR[k], cc = c + NB_DC[k];
            if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
            const int64_t y = (int64_t)rr * W + cc;
            if (occ[y] || dist[y] >= 0) continue;
            dist[y] = dist[x] + 1;
            queue[tail++] = y;
        }
    }
    free(queue);
    return ecc;
}

/* Closed form of the network output in terms of BFS distance d:
 *   A_L(x) = max(0, L + 1 - d(x)) for reachable free x, else 0.
 * (Induction over layers: each layer lifts the sources by one and spreads the
 * current values one step; the paper states both facts for its layer.)  It is
 * derived, not taken from the paper, and the tests pin it to oracle_layers.
 * Used where the literal network is too slow to run. */
void oracle_activity_from_bfs(int64_t N, const int32_t *dist, int64_t L, int64_t *out)
{
    for (int64_t i = 0; i < N; ++i) {
        const int64_t d = dist[i];
        out[i] = (d >= 0 && d <= L) ? L + 1 - d : 0;
    }
}

static int is_source(int64_t x, int32_t W, const int32_t *src_rc, int32_t n_src)
{
    for (int32_t k = 0; k < n_src; ++k)
        if ((int64_t)src_rc[2 * k] * W + src_rc[2 * k + 1] == x) return 1;
    return 0;
}

/* Simple path reconstruction (Sec. "Path Reconstruction"): from the target,
 * repeatedly move to the one of the eight neighbours with the largest activity
 * until a source is reached.
 * READING: ties are broken by the fixed neighbour order above (first maximum
 * wins) instead of at random, so the output is reproducible; the paper notes
 * every tie gives the same number of steps.
 * READING: a target whose activity is 0 (obstacle, unreachable, or farther
 * than L) has no path: len = -1 and no cells.  A target on a source gives a
 * one-cell path.
 *
 * O is the activity map (int64).  Output: len[t] (steps), offsets[t] into cells
 * (n_t + 1 entries, exclusive prefix of path cell counts), cells = linear
 * indices r*W + c from target to source inclusive.  Returns the total number of
 * cells, or -1 if cells_capacity is too small, or -2 if a walk does not end
 * within H*W steps. */
int64_t oracle_walk(int32_t H, int32_t W, const int64_t *O, const int32_t *src_rc, int32_t n_src,
                    const int32_t *tgt_rc, int32_t n_tgt, int32_t *len, int64_t *offsets,
                    int32_t *cells, int64_t cells_capacity)
{
    const int64_t N = (int64_t)H * W;
    int64_t total = 0;
    for (int32_t t = 0; t < n_tgt; ++t) {
        offsets[t] = total;
        int64_t p = (int64_t)tgt_rc[2 * t] * W + tgt_rc[2 * t + 1];
        if (O[p] <= 0) { len[t] = -1; continue; }
        int64_t steps = 0;
        if (total >= cells_capacity) return -1;
        cells[total++] = (int32_t)p;
        while (!is_source(p, W, src_rc, n_src)) {
            const int32_t r = (int32_t)(p / W), c = (int32_t)(p % W);
            int64_t best = -1, best_v = INT64_MIN;
            for (int k = 0; k < 8; ++k) {
                const int32_t rr = r + NB_DR[k], cc = c + NB_DC[k];
                if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                const int64_t y = (int64_t)rr * W + cc;
                if (O[y] > best_v) { best_v = O[y]; best = y; }
            }
            p = best;
            ++steps;
            if (steps > N) return -2;
            if (total >= cells_capacity) return -1;
            cells[total++] = (int32_t)p;
        }
        len[t] = (int32_t)steps;
    }
    offsets[n_tgt] = total;
    return total;
}

/* Euclidean path reconstruction (Sec. "Path Reconstruction", Eq. 1):
 * (1) walk from the target choosing, among the four horizontal / vertical
 *     neighbours, the one with maximal activity, until a source is reached
 *     (the chosen neighbour may have the same activity as the current cell:
 *     on open ground the walk then zig-zags along a staircase);
 * (2) straighten: remove an intermediate point P(t) when P(t-1) and P(t+1) are
 *     sqrt(2) apart, i.e. diagonal neighbours.
 * READING (ties): first maximum in the order up, left, right, down.
 * READING (cycles): the literal rule can step sideways forever (two cells of
 *     equal activity choosing each other, e.g. when the only way up is a
 *     diagonal step between two obstacles).  Here a sideways move (to a
 *     4-neighbour of equal activity) is allowed only if the previous move was
 *     not sideways; when no 4-neighbour is higher and a sideways move is not
 *     allowed, the walk takes the simple-reconstruction step (first maximal
 *     8-neighbour), which always climbs.  Activity never decreases along the
 *     walk, so no cell is visited twice and at most 2 d(t) moves are made.
 * READING (straightening order): one left-to-right pass over the current list;
 *     a removed point is gone before the next triple is examined.
 * Output layout as oracle_walk; len = number of segments of the final path.
 * Returns the total number of cells, -1 if the capacity is too small, -2 if a
 * walk does not end, -3 on allocation failure. */
int64_t oracle_walk_euclidean(int32_t H, int32_t W, const int64_t *O, const int32_t *src_rc,
                              int32_t n_src, const int32_t *tgt_rc, int32_t n_tgt, int32_t *len,
                              int64_t *offsets, int32_t *cells, int64_t cells_capacity)
{
    static const int M_DR[4] = {-1, 0, 0, 1};
    static const int M_DC[4] = {0, -1, 1, 0};
    const int64_t N = (int64_t)H * W;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * N + 2));
    if (!buf) return -3;
    int64_t total = 0;
    int64_t rc = 0;
    for (int32_t t = 0; t < n_tgt; ++t) {
        offsets[t] = total;
        int64_t p = (int64_t)tgt_rc[2 * t] * W + tgt_rc[2 * t + 1];
        if (O[p] <= 0) { len[t] = -1; continue; }
        int64_t k = 0;
        int sideways_before = 0;
        buf[k++] = (int32_t)p;
        while (!is_source(p, W, src_rc, n_src)) {
            const int32_t r = (int32_t)(p / W), c = (int32_t)(p % W);
            int64_t best = -1, best_v = INT64_MIN;
            for (int m = 0; m < 4; ++m) {
                const int32_t rr = r + M_DR[m], cc = c + M_DC[m];
                if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                const int64_t y = (int64_t)rr * W + cc;
                if (O[y] > best_v) { best_v = O[y]; best = y; }
            }
            if (best >= 0 && best_v > O[p]) {
                sideways_before = 0;                       /* climb */
            } else if (best >= 0 && best_v == O[p] && !sideways_before) {
                sideways_before = 1;                       /* sideways */
            } else {                                       /* 8-neighbour step */
                best_v = INT64_MIN;
                for (int m = 0; m < 8; ++m) {
                    const int32_t rr = r + NB_DR[m], cc = c + NB_DC[m];
                    if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                    const int64_t y = (int64_t)rr * W + cc;
                    if (O[y] > best_v) { best_v = O[y]; best = y; }
                }
                sideways_before = 0;
            }
            p = best;
            if (k > 2 * N) { rc = -2; goto done; }
            buf[k++] = (int32_t)p;
        }
        /* straightening pass over triples (last kept point, buf[i], buf[i+1]) */
        int64_t out_n = 0;
        for (int64_t i = 0; i < k; ++i) {
            if (out_n >= 1 && i + 1 < k) {
                const int64_t a = cells[total + out_n - 1];
                const int64_t b = buf[i + 1];
                const int32_t ar = (int32_t)(a / W), ac = (int32_t)(a % W);
                const int32_t br = (int32_t)(b / W), bc = (int32_t)(b % W);
                const int32_t dr = ar > br ? ar - br : br - ar, dc = ac > bc ? ac - bc : bc - ac;
                if (dr == 1 && dc == 1) continue;   /* drop buf[i] */
            }
            if (total + out_n >= cells_capacity) { rc = -1; goto done; }
            cells[total + out_n] = buf[i];
            ++out_n;
        }
        len[t] = (int32_t)(out_n - 1);
        total += out_n;
    }
    offsets[n_tgt] = total;
    rc = total;
done:
    free(buf);
    return rc;
}

/* Counter-based random numbers for the random tie-break: the SplitMix64 output
 * function (Steele, Lea, Flood 2014) applied to seed ^ (target << 32) ^ step. */
uint64_t oracle_tie_hash(uint64_t seed, uint64_t target, uint64_t step)
{
    uint64_t z = seed ^ (target << 32) ^ step;
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Simple path reconstruction with the paper's random choice among maximal
 * neighbours (Sec. "Path Reconstruction"): at move s from target t, the
 * maximal 8-neighbours are listed in the fixed order and the one at position
 * oracle_tie_hash(seed, t, s) mod (their number) is taken.  Output as
 * oracle_walk. */
int64_t oracle_walk_random(int32_t H, int32_t W, const int64_t *O, const int32_t *src_rc,
                           int32_t n_src, const int32_t *tgt_rc, int32_t n_tgt, uint64_t seed,
                           int32_t *len, int64_t *offsets, int32_t *cells, int64_t cells_capacity)
{
    const int64_t N = (int64_t)H * W;
    int64_t total = 0;
    for (int32_t t = 0; t < n_tgt; ++t) {
        offsets[t] = total;
        int64_t p = (int64_t)tgt_rc[2 * t] * W + tgt_rc[2 * t + 1];
        if (O[p] <= 0) { len[t] = -1; continue; }
        int64_t steps = 0;
        if (total >= cells_capacity) return -1;
        cells[total++] = (int32_t)p;
        while (!is_source(p, W, src_rc, n_src)) {
            const int32_t r = (int32_t)(p / W), c = (int32_t)(p % W);
            int64_t cand[8];
            int n_cand = 0;
            int64_t best_v = INT64_MIN;
            for (int k = 0; k < 8; ++k) {
                const int32_t rr = r + NB_DR[k], cc = c + NB_DC[k];
                if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                const int64_t y = (int64_t)rr * W + cc;
                if (O[y] > best_v) { best_v = O[y]; n_cand = 0; }
                if (O[y] == best_v) cand[n_cand++] = y;
            }
            p = cand[oracle_tie_hash(seed, (uint64_t)t, (uint64_t)steps) % (uint64_t)n_cand];
            ++steps;
            if (steps > N) return -2;
            if (total >= cells_capacity) return -1;
            cells[total++] = (int32_t)p;
        }
        len[t] = (int32_t)steps;
    }
    offsets[n_tgt] = total;
    return total;
}
