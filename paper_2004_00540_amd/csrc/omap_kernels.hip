// Device kernels of the oMAP planner for gfx950 (CDNA4, wave64) other than
// the tile sweeps (omap_sweep.h): ingest, seeding, reset, the run-time layer
// count, path lengths and walks, copy-out; and the launch wrappers, which
// dispatch the sweeps to the per-variant launch functions.

#include "omap_sweep.h"

namespace omap {

// ---------------------------------------------------------------------------
// ingest: occupancy bytes -> obstacle bit mask
// ---------------------------------------------------------------------------

__global__ void k_pack_mask(const uint8_t* __restrict__ occ, int32_t H, int32_t W,
                            uint32_t* __restrict__ mask, int32_t mpitch) {
    const int64_t n = (int64_t)H * mpitch;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = (int32_t)(i / mpitch);
        const int32_t w = (int32_t)(i - (int64_t)r * mpitch);
        const int32_t c0 = w * 32;
        const uint8_t* row = occ + (int64_t)r * W;
        uint32_t word = 0;
        if (c0 + 32 <= W) {
#pragma unroll
            for (int b = 0; b < 32; ++b) word |= (row[c0 + b] != 0 ? 1u : 0u) << b;
        } else {
            for (int b = 0; b < 32; ++b) {
                const int32_t c = c0 + b;
                const uint32_t bit = (c >= W) ? 1u : (row[c] != 0 ? 1u : 0u);
                word |= bit << b;
            }
        }
        mask[i] = word;
    }
}

// p[0 .. n) := value (int4 stores, then the last n mod 4 elements).
__global__ void k_fill(int32_t* __restrict__ p, int64_t n, int32_t value) {
    const int64_t n4 = n / 4;
    int4 v = make_int4(value, value, value, value);
    int4* q = reinterpret_cast<int4*>(p);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        q[i] = v;
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)(n - 4 * n4)) p[4 * n4 + threadIdx.x] = value;
}

__global__ void k_check_sources(const uint32_t* __restrict__ mask, int32_t mpitch,
                                const int32_t* __restrict__ src, int32_t n,
                                int32_t* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = src[2 * i], c = src[2 * i + 1];
    const uint32_t w = mask[(int64_t)r * mpitch + (c >> 5)];
    if ((w >> (c & 31)) & 1u) atomicAdd(bad, 1);
}

// Seed V := K at the sources (both buffers) and, when `schedule` is set,
// schedule the tiles whose interior or halo holds a source.
__global__ void k_seed(RoundArgs a, int32_t slot0, const int32_t* __restrict__ src,
                       const int32_t* __restrict__ src_slot, int32_t n, int32_t schedule,
                       int32_t* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int slot = src_slot != nullptr ? src_slot[i] : slot0;
    const MazeDev md = a.mazes[slot];
    const int32_t r = src[2 * i], c = src[2 * i + 1];
    const uint32_t w = md.mask[(int64_t)r * md.mpitch + (c >> 5)];
    if ((w >> (c & 31)) & 1u) {
        atomicAdd(bad, 1);
        return;
    }
    const int64_t x = (int64_t)r * md.pitch + c;
    md.V[0][x] = md.K;
    md.V[1][x] = md.K;
    if (md.R[0] != nullptr) {   // bit-sliced schedule: the source is in R_0 (both planes)
        const int64_t wx = (int64_t)r * md.mpitch + (c >> 5);
        atomicOr(&md.R[0][wx], 1u << (c & 31));
        atomicOr(&md.R[1][wx], 1u << (c & 31));
    }
    const int ty = r / a.tile_rows, tx = c / a.tile_cols;
    a.touched[md.tile_base + ty * md.tiles_x + tx] = 1;
    if (!schedule) return;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int ny = ty + dy, nx = tx + dx;
            if (ny < 0 || ny >= md.tiles_y || nx < 0 || nx >= md.tiles_x) continue;
            schedule_tile(a, md, slot, ny, nx);
        }
}

// Marks each of slots[0..n) for its first round: counters cleared, last round
// = r - 1; in the dense schedule the maze is flagged as changed so round r
// visits it.
__global__ void k_slot_reset(RoundArgs a, const int32_t* __restrict__ slots, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int slot = slots[i];
    a.maze_last_round[slot] = a.round_id - 1;
    for (int k = 0; k < kSpread; ++k) {
        a.maze_visits[slot * kSpread + k] = 0;
        a.maze_cell_visits[slot * kSpread + k] = 0;
    }
    if (a.dense) a.dchg_prev[slot] = 1;
}

// One wave per tile id in [tile_begin, tile_begin + n_tiles) whose maze is
// selected (sel == nullptr: every maze): zero the interior of touched tiles in
// both activity buffers (and, for the bit-sliced schedule, the interior words
// of both reached-set planes), and clear their touched flags.
__global__ __launch_bounds__(kBlockThreads) void k_clear_touched(RoundArgs a, int32_t tile_begin,
                                                                 int32_t n_tiles,
                                                                 const int32_t* __restrict__ sel) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = blockIdx.x * kWavesPerBlock + wave;
    if (t >= n_tiles) return;
    const int g = tile_begin + t;
    if (!a.touched[g]) return;
    const int slot = a.tile_maze[g];
    if (slot < 0 || (sel != nullptr && sel[slot] == 0)) return;
    const MazeDev md = a.mazes[slot];
    const int lt = g - md.tile_base;
    const int ty = lt / md.tiles_x, tx = lt - ty * md.tiles_x;
    const int r0 = ty * a.tile_rows, c0 = tx * a.tile_cols;
    const int rows = min(a.tile_rows, md.H - r0), cols = min(a.tile_cols, md.W - c0);
    for (int k = lane_id(); k < rows * cols; k += kLanes) {
        const int64_t x = (int64_t)(r0 + k / cols) * md.pitch + c0 + k % cols;
        md.V[0][x] = 0;
        md.V[1][x] = 0;
    }
    if (md.R[0] != nullptr) {   // bit tiles: 62 interior words per row
        const int w0 = c0 / 32, nw = min((cols + 31) / 32, md.mpitch - w0);
        for (int k = lane_id(); k < rows * nw; k += kLanes) {
            const int64_t x = (int64_t)(r0 + k / nw) * md.mpitch + w0 + k % nw;
            md.R[0][x] = 0;
            md.R[1][x] = 0;
        }
    }
    if (lane_id() == 0) a.touched[g] = 0;
}

// Packs the occupancy of several mazes (job j: words [word_begin[j],
// word_begin[j+1]) of the concatenated masks); one thread per mask word.
__global__ void k_pack_mask_many(const PackJob* __restrict__ jobs, int32_t n_jobs, int64_t total_words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total_words;
         i += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_jobs - 1;   // last job with word_begin <= i
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].word_begin <= i) lo = mid;
            else hi = mid - 1;
        }
        const PackJob jb = jobs[lo];
        const int64_t wi = i - jb.word_begin;
        const int32_t r = (int32_t)(wi / jb.mpitch);
        const int32_t w = (int32_t)(wi - (int64_t)r * jb.mpitch);
        const int32_t c0 = w * 32;
        const uint8_t* row = jb.occ + (int64_t)r * jb.W;
        uint32_t word = 0;
        for (int b = 0; b < 32; ++b) {
            const int32_t c = c0 + b;
            const uint32_t bit = (c >= jb.W) ? 1u : (row[c] != 0 ? 1u : 0u);
            word |= bit << b;
        }
        jb.mask[wi] = word;
    }
}

// Sources of several mazes on obstacles: bad[slot] counts them.
__global__ void k_check_sources_many(const MazeDev* __restrict__ mazes, const int32_t* __restrict__ src,
                                     const int32_t* __restrict__ src_slot, int32_t n, int32_t* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int slot = src_slot[i];
    const MazeDev md = mazes[slot];
    const int32_t r = src[2 * i], c = src[2 * i + 1];
    const uint32_t w = md.mask[(int64_t)r * md.mpitch + (c >> 5)];
    if ((w >> (c & 31)) & 1u) atomicAdd(&bad[slot], 1);
}

// ---------------------------------------------------------------------------
// finalize: smallest positive activity and reached-cell count per maze
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_reduce(const MazeDev* __restrict__ mazes,
                                                const int32_t* __restrict__ tile_maze,
                                                const uint8_t* __restrict__ touched,
                                                int32_t tile_begin, const int32_t* __restrict__ sel,
                                                int32_t tile_rows, int32_t tile_cols, int32_t parity,
                                                int32_t* __restrict__ maze_min,
                                                unsigned long long* __restrict__ maze_reached) {
    const int g = tile_begin + blockIdx.x;
    const int slot = tile_maze[g];
    // tiles never written since the last clear hold only zeros
    if (slot < 0 || (sel != nullptr && sel[slot] == 0) || !touched[g]) return;
    const MazeDev md = mazes[slot];
    const int lt = g - md.tile_base;
    const int ty = lt / md.tiles_x, tx = lt - ty * md.tiles_x;
    const int r0 = ty * tile_rows, c0 = tx * tile_cols;
    const int rows = min(tile_rows, md.H - r0), cols = min(tile_cols, md.W - c0);
    const int32_t* V = parity ? md.V[1] : md.V[0];
    int vmin = 0x7fffffff;
    int cnt = 0;
    for (int k = threadIdx.x; k < rows * cols; k += blockDim.x) {
        const int r = r0 + k / cols, c = c0 + k % cols;
        const int v = V[(int64_t)r * md.pitch + c];
        if (v > 0) {
            vmin = min(vmin, v);
            ++cnt;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        vmin = min(vmin, __shfl_xor(vmin, off));
        cnt += __shfl_xor(cnt, off);
    }
    __shared__ int smin[4], scnt[4];
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        smin[w] = vmin;
        scnt[w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = smin[0], n = scnt[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            m = min(m, smin[k]);
            n += scnt[k];
        }
        if (n > 0) {
            atomicMin(&maze_min[slot], m);
            atomicAdd(&maze_reached[slot], (unsigned long long)n);
        }
    }
}

// ---------------------------------------------------------------------------
// paths: lengths, offsets, gradient walk (one lane per target)
// ---------------------------------------------------------------------------

__global__ void k_path_lengths(const MazeDev* __restrict__ mazes, const int32_t* __restrict__ tslot,
                               const int32_t* __restrict__ trc, int32_t n, int32_t parity,
                               int32_t* __restrict__ len) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const MazeDev md = mazes[tslot[i]];
    const int32_t r = trc[2 * i], c = trc[2 * i + 1];
    const int v = (parity ? md.V[1] : md.V[0])[(int64_t)r * md.pitch + c];
    len[i] = v > 0 ? md.K - v : -1;
}

// Offsets of the paths (exclusive scan of length + 1 over reached targets),
// and optionally an order of the targets by path length, longest first (by
// the length's bit width: a bucket order, not a full sort), so that the walk
// starts the paths that take longest before the others.
// Takes a slot in bucket k for every lane with k >= 0 (wave-uniform call):
// one LDS atomic per distinct key in the wave, the lanes of a key numbered in
// lane order.  Returns the lane's slot, or -1 for k < 0.
__device__ __forceinline__ int wave_bucket_slot(int* bucket, int k) {
    const int lane = lane_id();
    int slot = -1;
    uint64_t todo = __ballot(k >= 0);
    while (todo != 0) {
        const int leader = __builtin_ctzll(todo);
        const int kk = __shfl(k, leader);
        const uint64_t same = __ballot(k == kk);
        int base = 0;
        if (lane == leader) base = atomicAdd(&bucket[kk], __popcll(same));
        base = __shfl(base, leader);
        if (k == kk) slot = base + __popcll(same & ((1ull << lane) - 1));
        todo &= ~same;
    }
    return slot;
}

__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ len, int32_t n,
                                               int64_t* __restrict__ off, int32_t* __restrict__ order) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = min(n, t * chunk), e = min(n, b + chunk);
    int64_t s = 0;
#pragma unroll 8
    for (int i = b; i < e; ++i) s += len[i] >= 0 ? (int64_t)len[i] + 1 : 0;
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t base = t ? part[t - 1] : 0;
    if (t == 0) off[0] = 0;
#pragma unroll 8
    for (int i = b; i < e; ++i) {
        base += len[i] >= 0 ? (int64_t)len[i] + 1 : 0;
        off[i + 1] = base;
    }
    if (order == nullptr) return;
    __shared__ int bucket[33];
    if (t < 33) bucket[t] = 0;
    __syncthreads();
    // key 0 = the longest lengths (32 - bit width of len + 1; unreached last);
    // elements in rows of 1024 (every thread runs the same number of rounds,
    // -1: past the end), eight rows' keys loaded together, one LDS atomic per
    // distinct key of a wave
    auto key = [&](int i) { return i >= n ? -1 : (len[i] < 0 ? 32 : __clz(len[i] + 1)); };
    constexpr int kRows = 8;
    const int rows = (n + 1023) / 1024;
    for (int j0 = 0; j0 < rows; j0 += kRows) {
        int kb[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) kb[u] = key((j0 + u) * 1024 + t);
#pragma unroll
        for (int u = 0; u < kRows; ++u) (void)wave_bucket_slot(bucket, kb[u]);
    }
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int k = 0; k < 33; ++k) {
            const int c = bucket[k];
            bucket[k] = acc;
            acc += c;
        }
    }
    __syncthreads();
    for (int j0 = 0; j0 < rows; j0 += kRows) {
        int kb[kRows];
#pragma unroll
        for (int u = 0; u < kRows; ++u) kb[u] = key((j0 + u) * 1024 + t);
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int slot = wave_bucket_slot(bucket, kb[u]);
            if (slot >= 0) order[slot] = (j0 + u) * 1024 + t;
        }
    }
}

__device__ __forceinline__ int dir_dr(int k) { return k < 3 ? -1 : (k < 5 ? 0 : 1); }
__device__ __forceinline__ int dir_dc(int k) {
    return (k == 0 || k == 3 || k == 5) ? -1 : ((k == 1 || k == 6) ? 0 : 1);
}

// The walk is a chain of dependent steps, so its time is the longest path
// times the latency of one step.  One wave follows one target through the
// activity map from a window of kWinRows x 64 cells held in LDS (one global
// round trip per window, 16-byte loads).
//
// A step from a reached non-source cell with activity v0 goes to its first
// neighbour (fixed order: row-major over the 3 x 3 block, centre skipped)
// whose activity is v0 + 1: the map's largest neighbour value is exactly
// v0 + 1 there (activity drops by one per move away from the sources), so
// this is the first maximal neighbour.  Three steps are resolved per LDS
// read: lane l reads the cell at (l / 8 - 3, l % 8 - 3) from the current
// cell, i.e. the 8 x 8 block around it, and three ballots mark the block's
// cells holding v0 + 1, v0 + 2 and v0 + 3.  Block cells are numbered
// row-major, so the 8 neighbours of block cell q, in the fixed order, are the
// set bits of kNbr << (q - 9), and step j moves to the lowest set bit of
// ballot j among the neighbours of the cell step j - 1 reached (a cell at
// most j - 1 from the centre, whose neighbours stay inside the block for
// j <= 3).  Window cells outside the grid read -1 and obstacles 0, so neither
// ever matches.  The window is placed so that the path's direction over the
// previous window has the most room ahead; it is reloaded when the 8 x 8
// block around the current cell no longer fits.
#ifndef OMAP_WALK_ROWS
#define OMAP_WALK_ROWS 48
#endif
constexpr int kWinRows = OMAP_WALK_ROWS;
constexpr int kWinCols = 64;                       // window row: 64 cells = 16 chunks of 4
constexpr int kWinChunks = kWinRows * kWinCols / 4;
static_assert(kWinRows >= 16 && kWinChunks % kLanes == 0, "walk window");
constexpr int kWalkWaves = 4;
// neighbours of block cell 9 (row 1, column 1): cells 0, 1, 2, 8, 10, 16, 17, 18
constexpr uint64_t kNbr = 0x70507ull;

__global__ __launch_bounds__(kLanes * kWalkWaves) void k_walk(
    const MazeDev* __restrict__ mazes, const int32_t* __restrict__ tslot, const int32_t* __restrict__ trc,
    int32_t n, int32_t parity, const int32_t* __restrict__ len, const int64_t* __restrict__ off,
    int32_t* __restrict__ cells, const int32_t* __restrict__ order) {
    __shared__ __attribute__((aligned(16))) int32_t win_all[kWalkWaves][kWinRows * kWinCols];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    const int w = blockIdx.x * kWalkWaves + wave;
    if (w >= n) return;
    // (order: longest paths first, see k_scan)
    const int i = order ? __builtin_amdgcn_readfirstlane(order[w]) : w;
    const int steps = __builtin_amdgcn_readfirstlane(len[i]);
    if (steps < 0) return;
    const int slot = __builtin_amdgcn_readfirstlane(tslot[i]);
    const MazeDev md = mazes[slot];
    const int32_t* __restrict__ V = parity ? md.V[1] : md.V[0];
    int32_t* win = win_all[wave];
    // this lane's cell of the 8 x 8 block, relative to the current cell
    const int my_off = ((lane >> 3) - 3) * kWinCols + ((lane & 7) - 3);
    int r = __builtin_amdgcn_readfirstlane(trc[2 * i]);
    int c = __builtin_amdgcn_readfirstlane(trc[2 * i + 1]);
    int64_t o = off[i];
    if (lane == 0) cells[o] = r * md.W + c;
    ++o;
    // the cells of a window's steps are logged one iteration (three steps)
    // per lane (lane k: iteration k of the window) as (window position of the
    // iteration's 8 x 8 block centre) << 18 | q1 << 12 | q2 << 6 | q3 (the
    // cells reached, numbered in the block), and stored when the window is left
    int log = 0, it = 0;
    int dr_prev = 0, dc_prev = 0;   // displacement over the previous window
    int v0 = 0;
    for (int s = 0; s < steps;) {
        // place the window: the current cell at row lr, column lc, with the
        // most room in the direction the path last went
        const int lr0 = dr_prev < 0 ? kWinRows - 5 : (dr_prev > 0 ? 3 : kWinRows / 2);
        const int lc0 = dc_prev < 0 ? 56 : (dc_prev > 0 ? 3 : 30);
        const int R0 = r - lr0, C0 = (c - lc0) & ~3;
        // every chunk's load is issued before the first is used, so the
        // window costs one global round trip
        v4i32 ld[kWinChunks / kLanes];
#pragma unroll
        for (int k = 0; k < kWinChunks / kLanes; ++k) {
            const int q = lane + kLanes * k;
            const int wr = q >> 4, wc = 4 * (q & 15);
            const int R = R0 + wr, cs = C0 + wc;
            const bool rok = R >= 0 && R < md.H;
            const bool cok = cs >= 0 && cs < md.pitch;   // a chunk lies wholly inside or outside a row
            ld[k] = *(const __attribute__((address_space(1))) v4i32*)(V + (int64_t)(rok ? R : 0) * md.pitch +
                                                                      (cok ? cs : 0));
        }
#pragma unroll
        for (int k = 0; k < kWinChunks / kLanes; ++k) {
            const int q = lane + kLanes * k;
            const int wr = q >> 4, wc = 4 * (q & 15);
            const int R = R0 + wr, cs = C0 + wc;
            const bool rok = R >= 0 && R < md.H;
            v4i32 m;
#pragma unroll
            for (int e = 0; e < 4; ++e) m[e] = (rok && cs + e >= 0 && cs + e < md.W) ? ld[k][e] : -1;
            *(__attribute__((address_space(3))) v4i32*)(win + wr * kWinCols + wc) = m;
        }
        // the same wave reads what its lanes wrote: LDS operations of a wave
        // complete in order; the wave barrier keeps the compiler from moving
        // the reads above the writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int lr = r - R0, lc = c - C0;
        if (s == 0) v0 = __builtin_amdgcn_readfirstlane(win[lr * kWinCols + lc]);
        const int s_start = s;
        // Whole iterations of three steps.  An iteration moves at most three
        // rows and three columns, so from the current cell the next n
        // iterations all start with their 8 x 8 block inside the window; the
        // bounds are checked once per such run.
        for (;;) {
            const int room = min(min(lr - 3, kWinRows - 5 - lr), min(lc - 3, kWinCols - 5 - lc));
            int n = room < 0 ? 0 : room / 3 + 1;
            n = min(n, min((steps - s) / 3, kLanes - it));
            if (n <= 0) break;
            for (int k = 0; k < n; ++k) {
                const int pos = lr * kWinCols + lc;
                const int d = win[pos + my_off] - v0;
                const uint64_t m1 = __ballot(d == 1);
                const uint64_t m2 = __ballot(d == 2);
                const uint64_t m3 = __ballot(d == 3);
                const int q1 = __builtin_ctzll(m1 & (kNbr << 18));   // neighbours of the centre, cell 27
                const int q2 = __builtin_ctzll(m2 & (kNbr << (q1 - 9)));
                const int q3 = __builtin_ctzll(m3 & (kNbr << (q2 - 9)));
                const int e = (pos << 18) | (q1 << 12) | (q2 << 6) | q3;
                log = lane == it + k ? e : log;
                lr += (q3 >> 3) - 3;
                lc += (q3 & 7) - 3;
                v0 += 3;
            }
            it += n;
            s += 3 * n;
        }
        // the path's last one or two steps, once their block fits
        if (s < steps && steps - s < 3 && it < kLanes && lr >= 3 && lr <= kWinRows - 5 && lc >= 3 &&
            lc <= kWinCols - 5) {
            const int pos = lr * kWinCols + lc;
            const int d = win[pos + my_off] - v0;
            const uint64_t m1 = __ballot(d == 1);
            const uint64_t m2 = __ballot(d == 2);
            const int todo = steps - s;
            const int q1 = __builtin_ctzll(m1 & (kNbr << 18));
            const int q2 = todo > 1 ? __builtin_ctzll(m2 & (kNbr << (q1 - 9))) : 0;
            const int q = todo > 1 ? q2 : q1;
            log = lane == it ? (pos << 18) | (q1 << 12) | (q2 << 6) : log;
            ++it;
            lr += (q >> 3) - 3;
            lc += (q & 7) - 3;
            v0 += todo;
            s += todo;
        }
        const int nst = s - s_start;   // steps taken in this window
        if (lane < it) {
            const int pos = log >> 18, pr = pos >> 6, pc = pos & 63;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (3 * lane + j < nst) {
                    const int q = (log >> (12 - 6 * j)) & 63;
                    cells[o + 3 * lane + j] = (R0 + pr - 3 + (q >> 3)) * md.W + (C0 + pc - 3 + (q & 7));
                }
            }
        }
        o += nst;
        it = 0;
        dr_prev = lr - (r - R0);
        dc_prev = lc - (c - C0);
        // a move of less than a third of the steps counts as no direction
        if (3 * abs(dr_prev) < nst) dr_prev = 0;
        if (3 * abs(dc_prev) < nst) dc_prev = 0;
        r = R0 + lr;
        c = C0 + lc;
        // the next window overwrites this one only after every lane's reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---- random ties and Euclidean reconstruction ------------------------------

// SplitMix64 output function on seed ^ (target << 32) ^ step: the counter-based
// random number of the random tie-break (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t tie_hash(uint64_t seed, uint64_t target, uint64_t step) {
    uint64_t z = seed ^ (target << 32) ^ step;
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int read_or(const int32_t* V, const MazeDev& md, int r, int c, int outside) {
    return (r >= 0 && r < md.H && c >= 0 && c < md.W) ? V[(int64_t)r * md.pitch + c] : outside;
}

// Simple reconstruction with random ties: at move s of target t (t = index in
// its maze's target list) the maximal 8-neighbours are counted in the fixed
// order and the one at position tie_hash(seed, t, s) mod count is taken.
__global__ void k_walk_random(const MazeDev* __restrict__ mazes, const int32_t* __restrict__ tslot,
                              const int32_t* __restrict__ trc, const int32_t* __restrict__ tlocal,
                              int32_t n, int32_t parity, uint64_t seed, const int32_t* __restrict__ len,
                              const int64_t* __restrict__ off, int32_t* __restrict__ cells) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int steps = len[i];
    if (steps < 0) return;
    const MazeDev md = mazes[tslot[i]];
    const int32_t* __restrict__ V = parity ? md.V[1] : md.V[0];
    int r = trc[2 * i], c = trc[2 * i + 1];
    int64_t o = off[i];
    cells[o++] = r * md.W + c;
    const uint64_t t = (uint64_t)tlocal[i];
    for (int s = 0; s < steps; ++s) {
        int nv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) nv[k] = read_or(V, md, r + dir_dr(k), c + dir_dc(k), -1);
        int bv = nv[0];
#pragma unroll
        for (int k = 1; k < 8; ++k) bv = max(bv, nv[k]);
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) cnt += nv[k] == bv;
        int j = (int)(tie_hash(seed, t, (uint64_t)s) % (uint64_t)cnt);
        int pick = 0;
#pragma unroll
        for (int k = 7; k >= 0; --k)
            if (nv[k] == bv) {      // walk maxima from the last: ends on the j-th in order
                if (--cnt == j) pick = k;
            }
        r += dir_dr(pick);
        c += dir_dc(pick);
        cells[o++] = r * md.W + c;
    }
}

// Euclidean reconstruction (Eq. 1 and straightening).  The walk climbs through
// 4-neighbours (first maximum in the order up, left, right, down), allows one
// sideways move to an equal 4-neighbour per activity level, and otherwise
// takes the first maximal 8-neighbour; the straightening pass (drop a point
// whose predecessor and successor are diagonal neighbours) runs on the fly.
// WRITE = false counts the final points (len = points - 1, -1 if no path);
// WRITE = true writes them at off[i].
template <bool WRITE>
__global__ void k_walk_euclid(const MazeDev* __restrict__ mazes, const int32_t* __restrict__ tslot,
                              const int32_t* __restrict__ trc, int32_t n, int32_t parity,
                              int32_t* __restrict__ len, const int64_t* __restrict__ off,
                              int32_t* __restrict__ cells) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const MazeDev md = mazes[tslot[i]];
    const int32_t* __restrict__ V = parity ? md.V[1] : md.V[0];
    int r = trc[2 * i], c = trc[2 * i + 1];
    int v = V[(int64_t)r * md.pitch + c];
    if (v <= 0) {
        if (!WRITE) len[i] = -1;
        return;
    }
    if (WRITE && len[i] < 0) return;
    int64_t o = WRITE ? off[i] : 0;
    int32_t count = 1;
    if (WRITE) cells[o++] = r * md.W + c;
    int kr = r, kc = c;            // last kept point
    int pr = -1, pc = -1;          // pending point (not yet decided)
    bool sideways_before = false;
    while (v != md.K) {
        // 4-neighbours: up, left, right, down
        const int u = read_or(V, md, r - 1, c, -1), l = read_or(V, md, r, c - 1, -1);
        const int rt = read_or(V, md, r, c + 1, -1), dn = read_or(V, md, r + 1, c, -1);
        int b4 = u, dr = -1, dc = 0;
        if (l > b4) { b4 = l; dr = 0; dc = -1; }
        if (rt > b4) { b4 = rt; dr = 0; dc = 1; }
        if (dn > b4) { b4 = dn; dr = 1; dc = 0; }
        if (b4 > v) {
            sideways_before = false;
        } else if (b4 == v && !sideways_before) {
            sideways_before = true;
        } else {
            int nv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) nv[k] = read_or(V, md, r + dir_dr(k), c + dir_dc(k), -1);
            int best = 0, bv = nv[0];
#pragma unroll
            for (int k = 1; k < 8; ++k)
                if (nv[k] > bv) {
                    bv = nv[k];
                    best = k;
                }
            b4 = bv;
            dr = dir_dr(best);
            dc = dir_dc(best);
            sideways_before = false;
        }
        r += dr;
        c += dc;
        v = b4;
        // straightening: the pending point is dropped when the last kept point
        // and the new point are diagonal neighbours
        if (pr >= 0) {
            const int ar = kr > r ? kr - r : r - kr, ac = kc > c ? kc - c : c - kc;
            if (!(ar == 1 && ac == 1)) {
                if (WRITE) cells[o++] = pr * md.W + pc;
                ++count;
                kr = pr;
                kc = pc;
            }
        }
        pr = r;
        pc = c;
    }
    if (pr >= 0) {
        if (WRITE) cells[o++] = pr * md.W + pc;
        ++count;
    }
    if (!WRITE) len[i] = count - 1;
}

// Index (in its maze's source list) of the source each path ends on; -1 if no
// path.  src_sorted holds per-maze (linear cell, first list index) pairs sorted
// by cell, src_base[t] / src_n[t] the target's maze's range.
__global__ void k_source_index(const MazeDev* __restrict__ mazes, const int32_t* __restrict__ tslot,
                               int32_t n, const int32_t* __restrict__ len,
                               const int64_t* __restrict__ off, const int32_t* __restrict__ cells,
                               const int32_t* __restrict__ src_sorted,
                               const int32_t* __restrict__ src_base,
                               const int32_t* __restrict__ src_n, int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (len[i] < 0) {
        out[i] = -1;
        return;
    }
    const int32_t end = cells[off[i + 1] - 1];
    const int32_t* p = src_sorted + 2 * (int64_t)src_base[i];
    int lo = 0, hi = src_n[i] - 1, found = -1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int32_t key = p[2 * mid];
        if (key == end) {
            found = p[2 * mid + 1];
            break;
        }
        if (key < end) lo = mid + 1; else hi = mid - 1;
    }
    out[i] = found;
}

// O = V - offset where V > 0, else 0 (offset = K - L - 1 maps the encoding back
// to the paper's activity values).
__global__ void k_activity(const MazeDev* __restrict__ mazes, int32_t slot, int32_t parity,
                           int32_t offset, int32_t* __restrict__ dst, int64_t dpitch,
                           int32_t col_blocks) {
    const MazeDev md = mazes[slot];
    const int64_t b = blockIdx.x;
    const int32_t r = (int32_t)(b / col_blocks);
    const int32_t c = (int32_t)(b - (int64_t)r * col_blocks) * blockDim.x + threadIdx.x;
    if (r >= md.H || c >= md.W) return;
    const int v = (parity ? md.V[1] : md.V[0])[(int64_t)r * md.pitch + c];
    dst[(int64_t)r * dpitch + c] = v > 0 ? v - offset : 0;
}

// Device self-check of the cross-lane moves and the saturating decrement.
__global__ void k_selftest(int32_t* out) {
    const int l = lane_id();
    out[l] = from_left_lane(l + 100);
    out[64 + l] = from_right_lane(l + 100);
    if (l == 0) {
        out[128] = (int32_t)sat_dec(0u);
        out[129] = (int32_t)sat_dec(5u);
        out[130] = (int32_t)sat_dec(kObstacleBit);
        out[131] = (int32_t)max(kObstacleBit, sat_dec(0x7fffffffu));
        out[132] = max3i((int)kObstacleBit, 3, -5);
    }
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------

static int grid_for(int64_t n, int block, int cap = 1 << 20) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_pack_mask(const uint8_t* occ, int32_t H, int32_t W, uint32_t* mask,
                            int32_t mpitch, hipStream_t s) {
    const int64_t n = (int64_t)H * mpitch;
    hipLaunchKernelGGL(k_pack_mask, dim3(grid_for(n, 256, 65536)), dim3(256), 0, s, occ, H, W, mask,
                       mpitch);
    return hipGetLastError();
}

hipError_t launch_fill(int32_t* p, int64_t n_elems, int32_t value, hipStream_t s) {
    if (n_elems <= 0) return hipSuccess;
    const int64_t n4 = n_elems / 4;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n4 > 0 ? n4 : 1, 256, 65536)), dim3(256), 0, s, p, n_elems, value);
    return hipGetLastError();
}

hipError_t launch_check_sources(const uint32_t* mask, int32_t mpitch, const int32_t* src_rc,
                                int32_t n_src, int32_t* bad_count, hipStream_t s) {
    hipLaunchKernelGGL(k_check_sources, dim3(grid_for(n_src, 256)), dim3(256), 0, s, mask, mpitch,
                       src_rc, n_src, bad_count);
    return hipGetLastError();
}

hipError_t launch_seed(const RoundArgs& a, int32_t slot, const int32_t* src_rc, const int32_t* src_slot,
                       int32_t n_src, int32_t* bad_count, hipStream_t s) {
    if (n_src <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed, dim3(grid_for(n_src, 256)), dim3(256), 0, s, a, slot, src_rc, src_slot, n_src,
                       a.dense ? 0 : 1, bad_count);
    return hipGetLastError();
}

hipError_t launch_slot_reset(const RoundArgs& a, const int32_t* slots, int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slot_reset, dim3(grid_for(n, 64)), dim3(64), 0, s, a, slots, n);
    return hipGetLastError();
}

hipError_t launch_pack_mask_many(const PackJob* jobs, int32_t n_jobs, int64_t total_words, hipStream_t s) {
    if (n_jobs <= 0 || total_words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_mask_many, dim3(grid_for(total_words, 256, 65536)), dim3(256), 0, s, jobs, n_jobs,
                       total_words);
    return hipGetLastError();
}

hipError_t launch_check_sources_many(const MazeDev* mazes, const int32_t* src_rc, const int32_t* src_slot,
                                     int32_t n, int32_t* bad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_sources_many, dim3(grid_for(n, 256)), dim3(256), 0, s, mazes, src_rc, src_slot, n,
                       bad);
    return hipGetLastError();
}

hipError_t launch_sweep(int T, int C, const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
#define X(t, c) \
    if (T == t && C == c) return launch_sweep_T##t##_C##c(a, grid, s, e0, e1);
    OMAP_SWEEP_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

static int sweep_blocks_per_cu(int T, int C) {
#define X(t, c) \
    if (T == t && C == c) return sweep_blocks_per_cu_T##t##_C##c();
    OMAP_SWEEP_VARIANTS(X)
#undef X
    return 0;
}

int sweep_max_waves_per_cu(int T, int C) {
    const int b = sweep_blocks_per_cu(T, C);
    return (b > 1 ? b : 1) * kWavesPerBlock;
}

bool bits_supported(int T) {
#define X(t) if (T == t) return true;
    OMAP_BITS_VARIANTS(X)
#undef X
    return false;
}

int bits_max_waves_per_cu(int T) {
    int b = 0;
#define X(t) if (T == t) b = bits_blocks_per_cu_T##t();
    OMAP_BITS_VARIANTS(X)
#undef X
    return (b > 1 ? b : 1) * kWavesPerBlock;
}

hipError_t launch_bits(int T, const RoundArgs& a, int32_t grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
#define X(t) if (T == t) return launch_bits_T##t(a, grid, s, e0, e1);
    OMAP_BITS_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

bool sweep_supported(int T, int C) {
#define X(t, c) if (T == t && C == c) return true;
    OMAP_SWEEP_VARIANTS(X)
#undef X
    return false;
}

hipError_t launch_reduce(const MazeDev* mazes, const int32_t* tile_maze, const uint8_t* touched,
                         int32_t tile_begin, int32_t tile_end, const int32_t* slot_select, int32_t tile_rows,
                         int32_t tile_cols, int32_t parity, int32_t* maze_min,
                         unsigned long long* maze_reached, hipStream_t s) {
    if (tile_end <= tile_begin) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(tile_end - tile_begin), dim3(256), 0, s, mazes, tile_maze, touched,
                       tile_begin, slot_select, tile_rows, tile_cols, parity, maze_min,
                       maze_reached);
    return hipGetLastError();
}

hipError_t launch_path_lengths(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                               int32_t n_tgt, int32_t parity, int32_t* len, hipStream_t s) {
    if (n_tgt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_path_lengths, dim3(grid_for(n_tgt, 256)), dim3(256), 0, s, mazes, tgt_slot,
                       tgt_rc, n_tgt, parity, len);
    return hipGetLastError();
}

hipError_t launch_scan_offsets(const int32_t* len, int32_t n, int64_t* offsets, hipStream_t s, int32_t* order) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, len, n, offsets, order);
    return hipGetLastError();
}

hipError_t launch_walk(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                       int32_t n_tgt, int32_t parity, const int32_t* len, const int64_t* offsets,
                       int32_t* cells, hipStream_t s, const int32_t* order) {
    if (n_tgt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk, dim3((n_tgt + kWalkWaves - 1) / kWalkWaves), dim3(kLanes * kWalkWaves), 0, s,
                       mazes, tgt_slot, tgt_rc, n_tgt, parity, len, offsets, cells, order);
    return hipGetLastError();
}

hipError_t launch_walk_random(const MazeDev* mazes, const int32_t* tgt_slot, const int32_t* tgt_rc,
                              const int32_t* tgt_local, int32_t n_tgt, int32_t parity, uint64_t seed,
                              const int32_t* len, const int64_t* offsets, int32_t* cells, hipStream_t s) {
    if (n_tgt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk_random, dim3(grid_for(n_tgt, 64)), dim3(64), 0, s, mazes, tgt_slot, tgt_rc,
                       tgt_local, n_tgt, parity, seed, len, offsets, cells);
    return hipGetLastError();
}

hipError_t launch_walk_euclid(bool write, const MazeDev* mazes, const int32_t* tgt_slot,
                              const int32_t* tgt_rc, int32_t n_tgt, int32_t parity, int32_t* len,
                              const int64_t* offsets, int32_t* cells, hipStream_t s) {
    if (n_tgt <= 0) return hipSuccess;
    if (write)
        hipLaunchKernelGGL(k_walk_euclid<true>, dim3(grid_for(n_tgt, 64)), dim3(64), 0, s, mazes, tgt_slot,
                           tgt_rc, n_tgt, parity, len, offsets, cells);
    else
        hipLaunchKernelGGL(k_walk_euclid<false>, dim3(grid_for(n_tgt, 64)), dim3(64), 0, s, mazes, tgt_slot,
                           tgt_rc, n_tgt, parity, len, offsets, cells);
    return hipGetLastError();
}

hipError_t launch_source_index(const MazeDev* mazes, const int32_t* tgt_slot, int32_t n_tgt,
                               const int32_t* len, const int64_t* offsets, const int32_t* cells,
                               const int32_t* src_sorted, const int32_t* src_base, const int32_t* src_n,
                               int32_t* out, hipStream_t s) {
    if (n_tgt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_source_index, dim3(grid_for(n_tgt, 256)), dim3(256), 0, s, mazes, tgt_slot, n_tgt,
                       len, offsets, cells, src_sorted, src_base, src_n, out);
    return hipGetLastError();
}

hipError_t launch_activity(const MazeDev* mazes, int32_t slot, int32_t H, int32_t W,
                           int32_t parity, int32_t offset, int32_t* dst, int64_t dpitch,
                           hipStream_t s) {
    const int32_t col_blocks = (W + 255) / 256;
    const int64_t blocks = (int64_t)H * col_blocks;
    hipLaunchKernelGGL(k_activity, dim3((uint32_t)blocks), dim3(256), 0, s, mazes, slot, parity,
                       offset, dst, dpitch, col_blocks);
    return hipGetLastError();
}

hipError_t launch_clear_touched(const RoundArgs& a, int32_t tile_begin, int32_t n_tiles, const int32_t* sel,
                                hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_touched, dim3((n_tiles + kWavesPerBlock - 1) / kWavesPerBlock),
                       dim3(kBlockThreads), 0, s, a, tile_begin, n_tiles, sel);
    return hipGetLastError();
}

__global__ void k_round_advance(int32_t* counter, int32_t add) { *counter += add; }

hipError_t launch_round_advance(int32_t* counter, int32_t add, hipStream_t s) {
    hipLaunchKernelGGL(k_round_advance, dim3(1), dim3(1), 0, s, counter, add);
    return hipGetLastError();
}

hipError_t launch_selftest(int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_selftest, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
}


}  // namespace omap
