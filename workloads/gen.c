/*
 * Seeded synthetic maze generators for the oMAP workloads.
 *
 * Input preparation only: nothing here computes activity, distances or
 * paths.  Both the CPU oracle and the GPU library are fed from these
 * generators, and neither links this file.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood 2014) expands a 64-bit seed
 * into the 256-bit state of xoshiro256** (Blackman and Vigna 2018).  Uniform
 * doubles take the top 53 bits; bounded integers use Lemire's
 * multiply-and-reject method (Lemire 2019), which is unbiased.
 *
 * Grids are row-major uint8 occupancy, H rows by W columns, cell (r, c) at
 * r*W + c; 1 = obstacle, 0 = free.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x)
{
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed, uint64_t stream)
{
    /* Distinct streams of one seed are decorrelated by mixing the stream tag
     * through SplitMix64 before expansion. */
    uint64_t x = seed;
    uint64_t t = stream;
    x ^= splitmix64(&t);
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r)
{
    uint64_t *s = r->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

static double rng_uniform(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* Uniform integer in [0, n), n >= 1. */
static uint64_t rng_below(rng_t *r, uint64_t n)
{
    uint64_t x = rng_next(r);
    __uint128_t m = (__uint128_t)x * n;
    uint64_t l = (uint64_t)m;
    if (l < n) {
        const uint64_t t = (0 - n) % n;
        while (l < t) {
            x = rng_next(r);
            m = (__uint128_t)x * n;
            l = (uint64_t)m;
        }
    }
    return (uint64_t)(m >> 64);
}

/* ---- exported scalar helpers (used to draw per-maze parameters) -------- */

/* n draws of U[0,1) from stream `stream` of `seed`. */
void gen_uniform(uint64_t seed, uint64_t stream, int64_t n, double *out)
{
    rng_t r;
    rng_seed(&r, seed, stream);
    for (int64_t i = 0; i < n; ++i) out[i] = rng_uniform(&r);
}

/* n draws of U{0..bound-1}. */
void gen_below(uint64_t seed, uint64_t stream, uint64_t bound, int64_t n, int64_t *out)
{
    rng_t r;
    rng_seed(&r, seed, stream);
    for (int64_t i = 0; i < n; ++i) out[i] = (int64_t)rng_below(&r, bound);
}

/* ---- obstacle fields ----------------------------------------------------- */

/* i.i.d. Bernoulli(p) obstacles, one uniform draw per cell in row-major order. */
void gen_bernoulli(int32_t H, int32_t W, double p, uint64_t seed, uint64_t stream, uint8_t *occ)
{
    rng_t r;
    rng_seed(&r, seed, stream);
    const int64_t N = (int64_t)H * W;
    for (int64_t i = 0; i < N; ++i) occ[i] = rng_uniform(&r) < p ? 1 : 0;
}

/* Overlay n_rects filled axis-aligned obstacle rectangles.  Height and width
 * are independent U{side_min..side_max} (clipped to the grid), and the
 * top-left corner is uniform over positions that keep the rectangle inside. */
void gen_rectangles(int32_t H, int32_t W, int32_t n_rects, int32_t side_min, int32_t side_max,
                    uint64_t seed, uint64_t stream, uint8_t *occ)
{
    rng_t r;
    rng_seed(&r, seed, stream);
    for (int32_t k = 0; k < n_rects; ++k) {
        int32_t h = side_min + (int32_t)rng_below(&r, (uint64_t)(side_max - side_min + 1));
        int32_t w = side_min + (int32_t)rng_below(&r, (uint64_t)(side_max - side_min + 1));
        if (h > H) h = H;
        if (w > W) w = W;
        const int32_t r0 = (int32_t)rng_below(&r, (uint64_t)(H - h + 1));
        const int32_t c0 = (int32_t)rng_below(&r, (uint64_t)(W - w + 1));
        for (int32_t rr = r0; rr < r0 + h; ++rr)
            memset(occ + (int64_t)rr * W + c0, 1, (size_t)w);
    }
}

/* Randomised depth-first ("recursive backtracker") perfect maze.
 *
 * Lattice cells sit at even coordinates (2i, 2j), i < ceil(H/2), j < ceil(W/2);
 * every other cell starts as wall.  A DFS from a uniformly drawn lattice cell
 * repeatedly moves to a uniformly drawn unvisited lattice neighbour (4 directions)
 * and carves the wall cell between them, backtracking when none is left.  The
 * carved passages form a spanning tree of the lattice.  Then a fraction
 * `removal_frac` (rounded to nearest) of the inter-cell walls that are still
 * standing is removed, drawn uniformly without replacement.  Pillars (odd, odd)
 * and, for even sides, the last row / column stay wall.
 *
 * Returns the number of walls removed after the DFS, or -1 on allocation failure. */
int64_t gen_dfs_maze(int32_t H, int32_t W, double removal_frac, uint64_t seed, uint64_t stream,
                     uint8_t *occ)
{
    rng_t r;
    rng_seed(&r, seed, stream);
    const int64_t N = (int64_t)H * W;
    memset(occ, 1, (size_t)N);
    const int32_t kr = (H + 1) / 2, kc = (W + 1) / 2;
    const int64_t K = (int64_t)kr * kc;
    for (int32_t i = 0; i < kr; ++i)
        for (int32_t j = 0; j < kc; ++j) occ[(int64_t)(2 * i) * W + 2 * j] = 0;

    uint8_t *visited = (uint8_t *)calloc((size_t)K, 1);
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    if (!visited || !stack) { free(visited); free(stack); return -1; }
    static const int di[4] = {-1, 0, 1, 0};
    static const int dj[4] = {0, 1, 0, -1};
    int64_t sp = 0;
    const int32_t start = (int32_t)rng_below(&r, (uint64_t)K);
    visited[start] = 1;
    stack[sp++] = start;
    while (sp > 0) {
        const int32_t cur = stack[sp - 1];
        const int32_t ci = cur / kc, cj = cur % kc;
        int cand[4], nc = 0;
        for (int d = 0; d < 4; ++d) {
            const int ni = ci + di[d], nj = cj + dj[d];
            if (ni < 0 || nj < 0 || ni >= kr || nj >= kc) continue;
            if (!visited[(int64_t)ni * kc + nj]) cand[nc++] = d;
        }
        if (nc == 0) { --sp; continue; }
        const int d = cand[rng_below(&r, (uint64_t)nc)];
        const int ni = ci + di[d], nj = cj + dj[d];
        occ[(int64_t)(2 * ci + di[d]) * W + (2 * cj + dj[d])] = 0;
        visited[(int64_t)ni * kc + nj] = 1;
        stack[sp++] = ni * kc + nj;
    }
    free(visited);
    free(stack);

    /* Remaining walls between horizontally or vertically adjacent lattice cells. */
    int64_t n_walls = 0;
    for (int32_t i = 0; i < kr; ++i)
        for (int32_t j = 0; j < kc; ++j) {
            if (j + 1 < kc && occ[(int64_t)(2 * i) * W + 2 * j + 1]) ++n_walls;
            if (i + 1 < kr && occ[(int64_t)(2 * i + 1) * W + 2 * j]) ++n_walls;
        }
    int64_t *walls = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_walls > 0 ? n_walls : 1));
    if (!walls) return -1;
    int64_t w = 0;
    for (int32_t i = 0; i < kr; ++i)
        for (int32_t j = 0; j < kc; ++j) {
            if (j + 1 < kc && occ[(int64_t)(2 * i) * W + 2 * j + 1]) walls[w++] = (int64_t)(2 * i) * W + 2 * j + 1;
            if (i + 1 < kr && occ[(int64_t)(2 * i + 1) * W + 2 * j]) walls[w++] = (int64_t)(2 * i + 1) * W + 2 * j;
        }
    const int64_t m = (int64_t)llround(removal_frac * (double)n_walls);
    for (int64_t k = 0; k < m; ++k) {   /* partial Fisher-Yates */
        const int64_t pick = k + (int64_t)rng_below(&r, (uint64_t)(n_walls - k));
        const int64_t tmp = walls[k];
        walls[k] = walls[pick];
        walls[pick] = tmp;
        occ[walls[k]] = 0;
    }
    free(walls);
    return m;
}

/* ---- connected components (placement of sources and targets) ------------ */

static int32_t uf_find(int32_t *parent, int32_t x)
{
    int32_t root = x;
    while (parent[root] != root) root = parent[root];
    while (parent[x] != root) {
        const int32_t nxt = parent[x];
        parent[x] = root;
        x = nxt;
    }
    return root;
}

static void uf_union(int32_t *parent, int32_t a, int32_t b)
{
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) parent[b] = a; else parent[a] = b;
}

/* 8-connected components of the free cells by union-find.  label[x] is the
 * smallest linear index of x's component, or -1 for obstacles.  Returns the
 * number of components; *largest_label / *largest_size describe the biggest
 * one (ties: smallest label). */
int64_t gen_components(int32_t H, int32_t W, const uint8_t *occ, int32_t *label,
                       int32_t *largest_label, int64_t *largest_size)
{
    const int64_t N = (int64_t)H * W;
    for (int64_t i = 0; i < N; ++i) label[i] = occ[i] ? -1 : (int32_t)i;
    for (int32_t rr = 0; rr < H; ++rr) {
        for (int32_t c = 0; c < W; ++c) {
            const int64_t x = (int64_t)rr * W + c;
            if (occ[x]) continue;
            if (c > 0 && !occ[x - 1]) uf_union(label, (int32_t)x, (int32_t)(x - 1));
            if (rr > 0) {
                const int64_t up = x - W;
                if (!occ[up]) uf_union(label, (int32_t)x, (int32_t)up);
                if (c > 0 && !occ[up - 1]) uf_union(label, (int32_t)x, (int32_t)(up - 1));
                if (c + 1 < W && !occ[up + 1]) uf_union(label, (int32_t)x, (int32_t)(up + 1));
            }
        }
    }
    int64_t n_comp = 0;
    for (int64_t i = 0; i < N; ++i)
        if (label[i] >= 0) {
            label[i] = uf_find(label, (int32_t)i);
            if (label[i] == (int32_t)i) ++n_comp;
        }
    /* component sizes: count into the root slot via a temporary array */
    int32_t *size = (int32_t *)calloc((size_t)(N > 0 ? N : 1), sizeof(int32_t));
    int32_t best = -1;
    int64_t best_size = 0;
    if (size) {
        for (int64_t i = 0; i < N; ++i)
            if (label[i] >= 0) ++size[label[i]];
        for (int64_t i = 0; i < N; ++i)
            if (size[i] > best_size) { best_size = size[i]; best = (int32_t)i; }
        free(size);
    } else {
        n_comp = -1;
    }
    if (largest_label) *largest_label = best;
    if (largest_size) *largest_size = best_size;
    return n_comp;
}

/* Draw k cells uniformly from {x : label[x] == want} (want == -2: any free
 * cell, i.e. label >= 0) by rejection on the whole grid.  distinct != 0 draws
 * without replacement (requires k <= population).  Writes (row, col) pairs.
 * Returns k, or -1 if the population is empty or too small. */
int32_t gen_sample_cells(int32_t H, int32_t W, const int32_t *label, int32_t want, int32_t k,
                         int32_t distinct, int64_t population, uint64_t seed, uint64_t stream,
                         int32_t *out_rc)
{
    if (k <= 0) return 0;
    if (population <= 0 || (distinct && population < k)) return -1;
    rng_t r;
    rng_seed(&r, seed, stream);
    const uint64_t N = (uint64_t)H * (uint64_t)W;
    int32_t got = 0;
    while (got < k) {
        const int64_t x = (int64_t)rng_below(&r, N);
        const int32_t lx = label[x];
        if (want == -2 ? lx < 0 : lx != want) continue;
        const int32_t rr = (int32_t)(x / W), c = (int32_t)(x % W);
        if (distinct) {
            int dup = 0;
            for (int32_t j = 0; j < got; ++j)
                if (out_rc[2 * j] == rr && out_rc[2 * j + 1] == c) { dup = 1; break; }
            if (dup) continue;
        }
        out_rc[2 * got] = rr;
        out_rc[2 * got + 1] = c;
        ++got;
    }
    return got;
}

/* FNV-1a 64 over a byte buffer: content hash used to pin generator output. */
uint64_t gen_fnv1a(const uint8_t *p, int64_t n)
{
    uint64_t h = 0xcbf29ce484222325ULL;
    for (int64_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ULL;
    }
    return h;
}
